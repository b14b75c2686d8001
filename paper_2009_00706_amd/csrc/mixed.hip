// Mixed-precision VMS assembly of libvms: placeholder.
#include "kernels.h"
namespace vmsk {
void launch_assemble_mixed(hipStream_t, const AsmArgs &, bool, bool, int) {}
}  // namespace vmsk

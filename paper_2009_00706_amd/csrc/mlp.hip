// Learned in-out filter of libvms (gfx950): placeholder until the network
// kernels are in place.
#include "mlp.h"
#include "../../include/vms.h"

namespace vmsm {

void Filter::release() {
    if (d_idx) (void)hipFree(d_idx);
    if (d_count) (void)hipFree(d_count);
    d_idx = nullptr;
    d_count = nullptr;
    cap = 0;
}

int classify_learned(hipStream_t, Filter &, const MlpDev *, const vmsk::SurfDev &, const double *,
                     const double *, const double *, int64_t, uint8_t *) {
    return VMS_EUNSUPPORTED;
}

}  // namespace vmsm

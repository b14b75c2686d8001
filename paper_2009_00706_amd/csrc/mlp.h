// Learned in-out filter of libvms (internal header).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace vmsm {

// Device-side description of the signed-distance network (see vms.h, vms_mlp).
struct MlpDev;

// Scratch kept by an in-out handle for the learned mode.
struct Filter {
    int64_t cap = 0;
    int64_t *d_idx = nullptr;                  // points sent to the exact test
    unsigned long long *d_count = nullptr;     // their number
    void release();
    ~Filter() { release(); }
};

int classify_learned(hipStream_t s, Filter &f, const MlpDev *net, const vmsk::SurfDev &S,
                     const double *px, const double *py, const double *pz, int64_t n,
                     uint8_t *labels);

}  // namespace vmsm

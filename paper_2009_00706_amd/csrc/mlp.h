// Learned in-out filter of libvms (internal header).
//
// Signed-distance network: features phi = [sin 2 pi B xh; cos 2 pi B xh] of the
// point mapped from the domain box to [-1, 1]^3 (B: 32 x 3, fixed), three
// hidden SiLU layers of width 64 and a linear output. Parameters (float):
// W1 (64x64, out x in), b1, W2, b2, W3, b3, w4 (64), b4 (1).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace vmsm {

constexpr int H = 64, NF = 32;
constexpr int OFF_W1 = 0, OFF_B1 = 4096, OFF_W2 = 4160, OFF_B2 = 8256, OFF_W3 = 8320, OFF_B3 = 12416,
              OFF_W4 = 12480, OFF_B4 = 12544, N_PARAMS = 12545;

using vmsk::MarginGrid;
using vmsk::Net;

// Scratch kept by an in-out handle for the learned mode.
struct Filter {
    int64_t cap = 0;
    int64_t *d_idx = nullptr;                  // points sent to the exact test
    unsigned long long *d_count = nullptr;     // their number
    float *d_pred = nullptr;                   // network output per point
    void release();
    ~Filter() { release(); }
};

struct MlpHandle;  // vms_mlp

// FP16-MFMA network outputs of n points.
void launch_predict(hipStream_t s, const Net &net, const double *px, const double *py,
                    const double *pz, int64_t n, float *pred);
// labels from the network where |pred| >= margin (of the point's cell when a
// grid is given), indices of the rest appended
void launch_decide(hipStream_t s, const float *pred, int64_t n, float margin, const MarginGrid &grid,
                   const double *px, const double *py, const double *pz, uint8_t *labels,
                   int64_t *idx, unsigned long long *count);

// Grow the filter's scratch to n points (no-op if it holds that many).
int reserve_filter(Filter &f, int64_t n);

// The handle's network, margin grid and scalar margin as the kernels see them.
Net mlp_net(const MlpHandle *h);
MarginGrid mlp_grid(const MlpHandle *h);
float mlp_margin(const MlpHandle *h);

int classify_learned(hipStream_t s, Filter &f, const MlpHandle *net, const vmsk::SurfDev &S,
                     const double *px, const double *py, const double *pz, int64_t n,
                     uint8_t *labels);

}  // namespace vmsm

// Device-side evaluation of the learned in-out filter's network (internal
// header of libvms, gfx950): FP16 MFMA (v_mfma_f32_16x16x32_f16) with FP32
// accumulation, 64 points per wave, neurons as M and points as N.
#pragma once
#include <hip/hip_runtime.h>

#include "mlp.h"

namespace vmsm {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));

constexpr int LDH = 72;  // fp16 row length of the activations in LDS (padding)

__device__ inline float silu(float a) { return a / (1.0f + __expf(-a)); }

// Network output for the calling lane's point P. All 64 lanes of the
// (one-wave) workgroup call it together; a lane with valid false contributes
// a dummy point. act: LDS scratch [64][LDH]. Outside the network's box
// (which contains the surface's box) the point is outside the body: +inf.
__device__ inline float net_output64(const Net &net, const double *P, bool valid,
                                     _Float16 (*act)[LDH]) {
    const int l = threadIdx.x;
    {
        float xh[3] = {0.f, 0.f, 0.f};
        if (valid)
            for (int k = 0; k < 3; ++k)
                xh[k] = (float)(2.0 * (P[k] - (double)net.lo[k]) * (double)net.inv[k] - 1.0);
        // features sin / cos of 2 pi z, z in revolutions
        for (int j = 0; j < NF; ++j) {
            const float z = net.B[3 * j] * xh[0] + net.B[3 * j + 1] * xh[1] + net.B[3 * j + 2] * xh[2];
            act[l][j] = (_Float16)__builtin_amdgcn_sinf(z);
            act[l][NF + j] = (_Float16)__builtin_amdgcn_cosf(z);
        }
    }
    __syncthreads();
    const int row = l & 15, g = l >> 4;
    const int offB[3] = {OFF_B1, OFF_B2, OFF_B3};
    for (int L = 0; L < 3; ++L) {
        // B operands: X[i][s] = act[s][i], lane holds s = 16 nt + row, i = 32 ks + 8 g + 0..7
        v8h X[4][2];
        for (int nt = 0; nt < 4; ++nt)
            for (int ks = 0; ks < 2; ++ks) X[nt][ks] = *(const v8h *)&act[16 * nt + row][32 * ks + 8 * g];
        __syncthreads();
        const _Float16 *W = net.w16 + L * H * H;
        for (int mt = 0; mt < 4; ++mt) {
            v8h A[2];
            for (int ks = 0; ks < 2; ++ks) A[ks] = *(const v8h *)&W[(16 * mt + row) * H + 32 * ks + 8 * g];
            float bias[4];
            for (int r = 0; r < 4; ++r) bias[r] = net.theta[offB[L] + 16 * mt + 4 * g + r];
            for (int nt = 0; nt < 4; ++nt) {
                v4f acc = {0.f, 0.f, 0.f, 0.f};
                acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[0], X[nt][0], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[1], X[nt][1], acc, 0, 0, 0);
                // output rows = neurons 16 mt + 4 g + r, column = point 16 nt + row
                for (int r = 0; r < 4; ++r) act[16 * nt + row][16 * mt + 4 * g + r] = (_Float16)silu(acc[r] + bias[r]);
            }
        }
        __syncthreads();
    }
    float y = net.theta[OFF_B4];
    for (int i = 0; i < H; i += 8) {
        const v8h a8 = *(const v8h *)&act[l][i];
        for (int e = 0; e < 8; ++e) y += net.theta[OFF_W4 + i + e] * (float)a8[e];
    }
    __syncthreads();  // act is reused by the caller's next batch
    if (valid)
        for (int k = 0; k < 3; ++k)
            if (P[k] < net.blo[k] || P[k] > net.bhi[k]) y = INFINITY;
    return y;
}

// Margin of a point: the scalar margin, or with a margin grid over the
// network box the margin of the point's cell.
__device__ inline float point_margin(const MarginGrid &g, float margin, const double *P) {
    if (!g.m) return margin;
    int c[3];
    for (int k = 0; k < 3; ++k) {
        const int v = (int)floor((P[k] - g.lo[k]) * g.inv[k]);
        c[k] = v < 0 ? 0 : (v >= g.n[k] ? g.n[k] - 1 : v);
    }
    return g.m[((int64_t)c[2] * g.n[1] + c[1]) * g.n[0] + c[0]];
}

}  // namespace vmsm

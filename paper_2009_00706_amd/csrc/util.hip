// Utility kernels of libvms (gfx950): fills, identity rows, FP64 norm.
#include "kernels.h"

namespace vmsk {

// ---------------------------------------------------------------------------
// small utility kernels
// ---------------------------------------------------------------------------

template <typename T>
__global__ void k_fill(T *p, int64_t n, T v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

static unsigned grid_for(int64_t n, int bs) {
    int64_t g = (n + bs - 1) / bs;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (unsigned)g;
}

void launch_fill_f64(hipStream_t s, double *p, int64_t n, double v) {
    if (n > 0) hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
}
void launch_fill_f32(hipStream_t s, float *p, int64_t n, float v) {
    if (n > 0) hipLaunchKernelGGL(k_fill<float>, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
}
// Dirichlet rows: node nodes[blockIdx.x]'s four rows (entries 16 nrow_ptr[n]
// .. 16 nrow_ptr[n + 1]) become identity rows; its residual entries zero
template <typename T>
__global__ void k_dirichlet_rows(T *vals, const int64_t *nrow_ptr, const int32_t *diag_pos,
                                 const int32_t *nodes, double *resid) {
    const int64_t n = nodes[blockIdx.x];
    const int64_t b0 = nrow_ptr[n], deg = nrow_ptr[n + 1] - b0;
    for (int64_t e = 16 * b0 + threadIdx.x; e < 16 * (b0 + deg); e += blockDim.x) vals[e] = (T)0;
    __syncthreads();
    if (threadIdx.x < 4) {
        const int c = threadIdx.x;
        vals[16 * b0 + 4 * c * deg + 4 * (int64_t)diag_pos[n] + c] = (T)1;
        if (resid) resid[4 * n + c] = 0.0;
    }
}

void launch_dirichlet_rows_f64(hipStream_t s, double *vals, const int64_t *nrow_ptr, const int32_t *diag_pos,
                               const int32_t *nodes, int64_t n, double *resid) {
    if (n > 0)
        hipLaunchKernelGGL(k_dirichlet_rows<double>, dim3((unsigned)n), dim3(64), 0, s, vals, nrow_ptr,
                           diag_pos, nodes, resid);
}
void launch_dirichlet_rows_f32(hipStream_t s, float *vals, const int64_t *nrow_ptr, const int32_t *diag_pos,
                               const int32_t *nodes, int64_t n, double *resid) {
    if (n > 0)
        hipLaunchKernelGGL(k_dirichlet_rows<float>, dim3((unsigned)n), dim3(64), 0, s, vals, nrow_ptr,
                           diag_pos, nodes, resid);
}

__global__ void k_norm2(const double *v, int64_t n, double *out) {
    __shared__ double part[4];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        acc += v[i] * v[i];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(out, part[0] + part[1] + part[2] + part[3]);
}

void launch_norm2(hipStream_t s, const double *v, int64_t n, double *out) {
    if (n > 0) hipLaunchKernelGGL(k_norm2, dim3(grid_for(n, 256) > 1024 ? 1024 : grid_for(n, 256)),
                                  dim3(256), 0, s, v, n, out);
}

__global__ void k_copy_rows(const double *x, double *y, const int32_t *nodes, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 4 * n) {
        const int64_t d = 4 * (int64_t)nodes[i >> 2] + (i & 3);
        y[d] = x[d];
    }
}

void launch_copy_rows(hipStream_t s, const double *x, double *y, const int32_t *nodes, int64_t n) {
    if (n > 0)
        hipLaunchKernelGGL(k_copy_rows, dim3((unsigned)((4 * n + 255) / 256)), dim3(256), 0, s, x, y,
                           nodes, n);
}

// Block-CSR product, 16 lanes per node row: lane l takes blocks l, l + 16, ...
// of the row (so a dof row's entries are read 64 at a time, contiguous), the
// four row sums are reduced over the 16 lanes in a fixed order.
template <typename T>
__global__ void k_bspmv(const int64_t *nrow_ptr, const int32_t *ncol, const T *vals, const double *x,
                        double *y, int64_t n) {
    const int64_t node = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
    const int l = threadIdx.x & 15;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (node < n) {
        const int64_t b0 = nrow_ptr[node], b1 = nrow_ptr[node + 1], deg = b1 - b0;
        const T *v = vals + 16 * b0;
        for (int64_t b = b0 + l; b < b1; b += 16) {
            const double *xc = x + 4 * (int64_t)ncol[b];
            const double x0 = xc[0], x1 = xc[1], x2 = xc[2], x3 = xc[3];
            const int64_t kb = 4 * (b - b0);
            for (int r = 0; r < 4; ++r) {
                const T *vr = v + r * 4 * deg + kb;
                acc[r] += (double)vr[0] * x0 + (double)vr[1] * x1 + (double)vr[2] * x2 +
                          (double)vr[3] * x3;
            }
        }
    }
    for (int off = 8; off > 0; off >>= 1)
        for (int r = 0; r < 4; ++r) acc[r] += __shfl_xor(acc[r], off, 16);
    if (node < n && l < 4) y[4 * node + l] = l == 0 ? acc[0] : (l == 1 ? acc[1] : (l == 2 ? acc[2] : acc[3]));
}

void launch_bspmv_f64(hipStream_t s, const int64_t *nrow_ptr, const int32_t *ncol, const double *vals,
                      const double *x, double *y, int64_t n_nodes) {
    if (n_nodes > 0)
        hipLaunchKernelGGL(k_bspmv<double>, dim3((unsigned)((16 * n_nodes + 255) / 256)), dim3(256), 0,
                           s, nrow_ptr, ncol, vals, x, y, n_nodes);
}
void launch_bspmv_f32(hipStream_t s, const int64_t *nrow_ptr, const int32_t *ncol, const float *vals,
                      const double *x, double *y, int64_t n_nodes) {
    if (n_nodes > 0)
        hipLaunchKernelGGL(k_bspmv<float>, dim3((unsigned)((16 * n_nodes + 255) / 256)), dim3(256), 0,
                           s, nrow_ptr, ncol, vals, x, y, n_nodes);
}

}  // namespace vmsk

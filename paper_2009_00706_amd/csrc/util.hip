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

template <typename T>
__global__ void k_set_ones(T *vals, const int64_t *idx, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) vals[idx[i]] = (T)1;
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
void launch_set_ones_f64(hipStream_t s, double *vals, const int64_t *idx, int64_t n) {
    if (n > 0)
        hipLaunchKernelGGL(k_set_ones<double>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                           vals, idx, n);
}
void launch_set_ones_f32(hipStream_t s, float *vals, const int64_t *idx, int64_t n) {
    if (n > 0)
        hipLaunchKernelGGL(k_set_ones<float>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                           vals, idx, n);
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

}  // namespace vmsk

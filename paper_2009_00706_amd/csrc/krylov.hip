// Vector kernels of the Krylov solves of Newton's linear step (BiCGStab and
// restarted GMRES, gfx950): block-Jacobi preconditioner from the 4x4 diagonal
// blocks of the assembled Jacobian, deterministic multi-dot products,
// combinations of Krylov vectors. All vectors are FP64 with 4 entries per node.
#include "kernels.h"

namespace vmsk {

namespace {
constexpr int KB = 256;  // threads per block of the vector kernels

unsigned blocks_for(int64_t n, int64_t cap) {
    int64_t g = (n + KB - 1) / KB;
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    return (unsigned)g;
}
}  // namespace

// Inverse of node n's diagonal block: its dof row 4 n + i starts at
// 16 nrow_ptr[n] + 4 i deg, and the block is entries 4 diag_pos[n] .. + 3 of
// each row. Gauss-Jordan with partial pivoting in FP64; a zero pivot marks the
// node in *bad (the caller reports it).
template <typename T>
__global__ void k_bjac_invert(const T *vals, const int64_t *nrow_ptr, const int32_t *diag_pos,
                              int64_t n_nodes, double *dinv, int *bad) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= n_nodes) return;
    const int64_t b0 = nrow_ptr[n], deg = nrow_ptr[n + 1] - b0;
    const T *v = vals + 16 * b0 + 4 * (int64_t)diag_pos[n];
    double a[4][8];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            a[i][j] = (double)v[4 * i * deg + j];
            a[i][4 + j] = i == j ? 1.0 : 0.0;
        }
    // partial pivoting by compare-and-swap against each lower row in turn (the
    // largest entry ends in the pivot row); fully unrolled so that every index
    // is static and the matrix stays in registers
#pragma unroll
    for (int c = 0; c < 4; ++c) {
#pragma unroll
        for (int r = c + 1; r < 4; ++r) {
            const bool sw = fabs(a[r][c]) > fabs(a[c][c]);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const double t = a[c][j];
                a[c][j] = sw ? a[r][j] : t;
                a[r][j] = sw ? t : a[r][j];
            }
        }
        if (a[c][c] == 0.0) {
            atomicOr(bad, 1);
            return;
        }
        const double ip = 1.0 / a[c][c];
#pragma unroll
        for (int j = 0; j < 8; ++j) a[c][j] *= ip;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (r == c) continue;
            const double f = a[r][c];
#pragma unroll
            for (int j = 0; j < 8; ++j) a[r][j] -= f * a[c][j];
        }
    }
    double *d = dinv + 16 * n;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) d[4 * i + j] = a[i][4 + j];
}

// y = blockdiag(dinv) x
__global__ void k_bjac_apply(const double *dinv, const double *x, double *y, int64_t n_nodes) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= n_nodes) return;
    const double *d = dinv + 16 * n;
    const double x0 = x[4 * n], x1 = x[4 * n + 1], x2 = x[4 * n + 2], x3 = x[4 * n + 3];
    for (int i = 0; i < 4; ++i)
        y[4 * n + i] = d[4 * i] * x0 + d[4 * i + 1] * x1 + d[4 * i + 2] * x2 + d[4 * i + 3] * x3;
}

// partial[k][blockIdx.x] = sum over the block's entries of V_k . w, for k =
// blockIdx.y (V_k = V + k ldv); fixed order inside a block (wave shuffles, then
// the four waves in order)
__global__ void k_multidot(const double *V, int64_t ldv, const double *w, int64_t n, double *partial) {
    __shared__ double part[KB / 64];
    const int k = blockIdx.y;
    const double *v = V + (int64_t)k * ldv;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * KB + threadIdx.x; i < n; i += (int64_t)gridDim.x * KB)
        acc += v[i] * w[i];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int q = 0; q < KB / 64; ++q) s += part[q];
        partial[(int64_t)k * gridDim.x + blockIdx.x] = s;
    }
}

// out[k] = sum of the nb partial sums of row k, in order (one wave per k)
__global__ void k_multidot_finish(const double *partial, int nb, double *out) {
    const int k = blockIdx.x, l = threadIdx.x;
    double s = 0.0;
    for (int b = l; b < nb; b += 64) s += partial[(int64_t)k * nb + b];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (l == 0) out[k] = s;
}

// mode 0: w -= sum_k c[k] V_k; mode 1: w = sum_k c[k] V_k (c on the device)
__global__ void k_combine(const double *V, int64_t ldv, int nk, const double *c, double *w, int64_t n,
                          int mode) {
    for (int64_t i = (int64_t)blockIdx.x * KB + threadIdx.x; i < n; i += (int64_t)gridDim.x * KB) {
        double s = 0.0;
        for (int k = 0; k < nk; ++k) s += c[k] * V[(int64_t)k * ldv + i];
        w[i] = mode == 0 ? w[i] - s : s;
    }
}

// out = a x + b y (host scalars; out may alias x or y)
__global__ void k_axpby(double a, const double *x, double b, const double *y, double *out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * KB + threadIdx.x; i < n; i += (int64_t)gridDim.x * KB)
        out[i] = a * x[i] + b * y[i];
}

// out = a x + b y + c z (host scalars; out may alias any input)
__global__ void k_axpbypcz(double a, const double *x, double b, const double *y, double c, const double *z,
                           double *out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * KB + threadIdx.x; i < n; i += (int64_t)gridDim.x * KB)
        out[i] = a * x[i] + b * y[i] + c * z[i];
}

void launch_axpbypcz(hipStream_t s, double a, const double *x, double b, const double *y, double c,
                     const double *z, double *out, int64_t n) {
    if (n > 0)
        hipLaunchKernelGGL(k_axpbypcz, dim3(blocks_for(n, 4096)), dim3(KB), 0, s, a, x, b, y, c, z, out, n);
}

void launch_bjac_invert_f64(hipStream_t s, const double *vals, const int64_t *nrow_ptr,
                            const int32_t *diag_pos, int64_t n_nodes, double *dinv, int *bad) {
    if (n_nodes > 0)
        hipLaunchKernelGGL(k_bjac_invert<double>, dim3((unsigned)((n_nodes + 127) / 128)), dim3(128), 0, s,
                           vals, nrow_ptr, diag_pos, n_nodes, dinv, bad);
}
void launch_bjac_invert_f32(hipStream_t s, const float *vals, const int64_t *nrow_ptr,
                            const int32_t *diag_pos, int64_t n_nodes, double *dinv, int *bad) {
    if (n_nodes > 0)
        hipLaunchKernelGGL(k_bjac_invert<float>, dim3((unsigned)((n_nodes + 127) / 128)), dim3(128), 0, s,
                           vals, nrow_ptr, diag_pos, n_nodes, dinv, bad);
}
void launch_bjac_apply(hipStream_t s, const double *dinv, const double *x, double *y, int64_t n_nodes) {
    if (n_nodes > 0)
        hipLaunchKernelGGL(k_bjac_apply, dim3((unsigned)((n_nodes + KB - 1) / KB)), dim3(KB), 0, s, dinv, x,
                           y, n_nodes);
}
int multidot_blocks(int64_t n) { return (int)blocks_for(n, 1024); }
void launch_multidot(hipStream_t s, const double *V, int64_t ldv, int nk, const double *w, int64_t n,
                     double *partial, double *out) {
    if (nk <= 0) return;
    const unsigned nb = blocks_for(n, 1024);
    hipLaunchKernelGGL(k_multidot, dim3(nb, (unsigned)nk), dim3(KB), 0, s, V, ldv, w, n, partial);
    hipLaunchKernelGGL(k_multidot_finish, dim3((unsigned)nk), dim3(64), 0, s, partial, (int)nb, out);
}
void launch_combine(hipStream_t s, const double *V, int64_t ldv, int nk, const double *c, double *w,
                    int64_t n, int mode) {
    if (n > 0)
        hipLaunchKernelGGL(k_combine, dim3(blocks_for(n, 4096)), dim3(KB), 0, s, V, ldv, nk, c, w, n, mode);
}
void launch_axpby(hipStream_t s, double a, const double *x, double b, const double *y, double *out,
                  int64_t n) {
    if (n > 0)
        hipLaunchKernelGGL(k_axpby, dim3(blocks_for(n, 4096)), dim3(KB), 0, s, a, x, b, y, out, n);
}

}  // namespace vmsk

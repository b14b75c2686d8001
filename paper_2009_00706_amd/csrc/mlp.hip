// Learned in-out filter of libvms (gfx950).
//
// A signed-distance network (negative inside the body) is trained on exact
// signed distances and used as a filter in front of the exact in-out test:
// a point whose prediction has |pred| >= margin takes the sign of the
// prediction, every other point goes to the exact test, so that labels are
// the exact ones whenever the margin exceeds the network's error.
//
//   training:   forward and reverse-mode backward in FP32 on the VALU, 32
//               samples per workgroup with activations in LDS, parameter
//               gradients summed by atomics; Adam update kernel.
//   inference:  FP16 MFMA (v_mfma_f32_16x16x32_f16) with FP32 accumulation,
//               64 points per wave, neurons as M, points as N.
//   samples:    exact signed distance clamped to [-T, T]: nearest triangle by
//               a uniform grid (closest point by Voronoi regions of the
//               triangle), sign from the exact in-out test.
#include "../../include/vms.h"
#include "inout_dev.h"
#include "mlp.h"
#include "mlp_dev.h"

#include <cmath>
#include <string>
#include <vector>

namespace vmsm {

void Filter::release() {
    if (d_idx) (void)hipFree(d_idx);
    if (d_count) (void)hipFree(d_count);
    if (d_pred) (void)hipFree(d_pred);
    d_idx = nullptr;
    d_count = nullptr;
    d_pred = nullptr;
    cap = 0;
}

__device__ inline float dsilu(float a) {
    const float s = 1.0f / (1.0f + __expf(-a));
    return s * (1.0f + a * (1.0f - s));
}

// ---------------------------------------------------------------------------
// training: loss and parameter gradient over a batch (FP32 VALU)
// ---------------------------------------------------------------------------

constexpr int S = 32;   // samples per workgroup
constexpr int LD = 65;  // padded row length in LDS

// One workgroup of 256 threads per 32 samples: thread (s, part) owns sample s
// and outputs [8 part, 8 part + 8) of every layer. LDS keeps the features and
// the three pre-activations (58 KB); silu and its derivative are recomputed.
__global__ __launch_bounds__(256) void k_grad(Net net, const double *px, const double *py,
                                              const double *pz, const double *sdf, int64_t n,
                                              int64_t first, int64_t count, float trunc,
                                              float *grad, double *loss) {
    __shared__ float sAct[4][S][LD];  // phi, a1, a2, a3
    __shared__ float sW[H][LD];
    __shared__ float sG[S][LD];
    __shared__ float sGy[S];
    const int t = threadIdx.x;
    const int s = t & (S - 1), part = t >> 5;
    const int64_t b0 = (int64_t)blockIdx.x * S;
    const bool valid = b0 + s < count;
    const int64_t gi = (first + b0 + s) % n;
    const float *th = net.theta;
    // features
    {
        float xh[3] = {0.f, 0.f, 0.f};
        if (valid) {
            const double P[3] = {px[gi], py[gi], pz[gi]};
            for (int k = 0; k < 3; ++k) xh[k] = (float)(2.0 * (P[k] - (double)net.lo[k]) * (double)net.inv[k] - 1.0);
        }
        for (int q = 0; q < 8; ++q) {
            const int i = 8 * part + q, j = i & 31;
            const float z = 6.283185307179586f * (net.B[3 * j] * xh[0] + net.B[3 * j + 1] * xh[1] + net.B[3 * j + 2] * xh[2]);
            sAct[0][s][i] = valid ? (i < 32 ? sinf(z) : cosf(z)) : 0.f;
        }
    }
    const int offW[3] = {OFF_W1, OFF_W2, OFF_W3}, offB[3] = {OFF_B1, OFF_B2, OFF_B3};
    // forward: a_{L+1} = W_L h_L + b_L, h_0 = phi, h_L = silu(a_L)
    for (int L = 0; L < 3; ++L) {
        for (int q = 0; q < 16; ++q) {
            const int e = t * 16 + q;
            sW[e >> 6][e & 63] = th[offW[L] + e];
        }
        __syncthreads();
        float acc[8];
        for (int q = 0; q < 8; ++q) acc[q] = th[offB[L] + 8 * part + q];
        for (int i = 0; i < H; ++i) {
            const float a = sAct[L][s][i];
            const float x = L == 0 ? a : silu(a);
            for (int q = 0; q < 8; ++q) acc[q] += sW[8 * part + q][i] * x;
        }
        for (int q = 0; q < 8; ++q) sAct[L + 1][s][8 * part + q] = acc[q];
        __syncthreads();
    }
    // output, loss, d loss / d y
    if (part == 0) {
        float y = th[OFF_B4];
        for (int i = 0; i < H; ++i) y += th[OFF_W4 + i] * silu(sAct[3][s][i]);
        float g = 0.f;
        if (valid) {
            const float tgt = fminf(fmaxf((float)sdf[gi], -trunc), trunc);
            const float r = y - tgt;
            atomicAdd(loss, (double)(0.5f * r * r));
            g = r;
        }
        sGy[s] = g / (float)count;
    }
    __syncthreads();
    if (t < 64) {
        float gw = 0.f;
        for (int q = 0; q < S; ++q) gw += sGy[q] * silu(sAct[3][q][t]);
        atomicAdd(grad + OFF_W4 + t, gw);
    } else if (t == 64) {
        float gb = 0.f;
        for (int q = 0; q < S; ++q) gb += sGy[q];
        atomicAdd(grad + OFF_B4, gb);
    }
    for (int q = 0; q < 8; ++q) {
        const int o = 8 * part + q;
        sG[s][o] = sGy[s] * th[OFF_W4 + o] * dsilu(sAct[3][s][o]);
    }
    __syncthreads();
    for (int L = 2; L >= 0; --L) {
        // parameter gradients: gW[o][i] = sum_s G[s][o] h_L[s][i], gb[o] = sum_s G[s][o]
        {
            const int o = t >> 2, i0 = 16 * (t & 3);
            float gw[16];
            for (int q = 0; q < 16; ++q) gw[q] = 0.f;
            for (int q = 0; q < S; ++q) {
                const float gq = sG[q][o];
                for (int r = 0; r < 16; ++r) {
                    const float a = sAct[L][q][i0 + r];
                    gw[r] += gq * (L == 0 ? a : silu(a));
                }
            }
            for (int r = 0; r < 16; ++r) atomicAdd(grad + offW[L] + o * H + i0 + r, gw[r]);
            if ((t & 3) == 0) {
                float gb = 0.f;
                for (int q = 0; q < S; ++q) gb += sG[q][o];
                atomicAdd(grad + offB[L] + o, gb);
            }
        }
        if (L == 0) break;
        // G_new[s][i] = (sum_o G[s][o] W_L[o][i]) dsilu(a_L[s][i])
        for (int q = 0; q < 16; ++q) {
            const int e = t * 16 + q;
            sW[e >> 6][e & 63] = th[offW[L] + e];
        }
        __syncthreads();
        float gh[8];
        for (int q = 0; q < 8; ++q) gh[q] = 0.f;
        for (int o = 0; o < H; ++o) {
            const float g = sG[s][o];
            for (int q = 0; q < 8; ++q) gh[q] += g * sW[o][8 * part + q];
        }
        __syncthreads();
        for (int q = 0; q < 8; ++q) {
            const int i = 8 * part + q;
            sG[s][i] = gh[q] * dsilu(sAct[L][s][i]);
        }
        __syncthreads();
    }
}

__global__ void k_adam(float *theta, float *m, float *v, const float *g, int n, float lr, float c1,
                       float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

__global__ void k_to_half(const float *theta, _Float16 *w16) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 3 * H * H) return;
    const int L = i / (H * H), e = i % (H * H);
    const int off = L == 0 ? OFF_W1 : (L == 1 ? OFF_W2 : OFF_W3);
    w16[i] = (_Float16)theta[off + e];
}

// ---------------------------------------------------------------------------
// inference: FP16 MFMA, 64 points per wave
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(64) void k_predict(Net net, const double *px, const double *py,
                                                const double *pz, int64_t n, float *pred) {
    __shared__ __attribute__((aligned(16))) _Float16 act[64][LDH];
    const int64_t gi = (int64_t)blockIdx.x * 64 + threadIdx.x;
    const bool valid = gi < n;
    double P[3] = {0.0, 0.0, 0.0};
    if (valid) { P[0] = px[gi]; P[1] = py[gi]; P[2] = pz[gi]; }
    const float y = net_output64(net, P, valid, act);
    if (valid) pred[gi] = y;
}

__global__ void k_decide(const float *pred, int64_t n, float margin, MarginGrid grid,
                         const double *px, const double *py, const double *pz, uint8_t *labels,
                         int64_t *idx, unsigned long long *count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float y = pred[i];
    const double P[3] = {px[i], py[i], pz[i]};
    if (fabsf(y) >= point_margin(grid, margin, P)) {
        labels[i] = y < 0.f ? 1 : 0;
    } else {
        const unsigned long long k = atomicAdd(count, 1ull);
        idx[k] = i;
    }
}

void launch_predict(hipStream_t s, const Net &net, const double *px, const double *py,
                    const double *pz, int64_t n, float *pred) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_predict, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, net, px, py, pz, n,
                       pred);
}

void launch_decide(hipStream_t s, const float *pred, int64_t n, float margin, const MarginGrid &grid,
                   const double *px, const double *py, const double *pz, uint8_t *labels,
                   int64_t *idx, unsigned long long *count) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_decide, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pred, n, margin,
                       grid, px, py, pz, labels, idx, count);
}

// ---------------------------------------------------------------------------
// exact signed distance, clamped to [-T, T]
// ---------------------------------------------------------------------------

struct DistGrid {
    double g0[3], cell;
    int n[3];
    const int32_t *off;  // [n0 n1 n2 + 1]
    const int32_t *ids;
};

__device__ inline double tri_dist2(const double *p, const double *a, const double *b, const double *c) {
    double ab[3], ac[3], ap[3], q[3];
    for (int k = 0; k < 3; ++k) { ab[k] = b[k] - a[k]; ac[k] = c[k] - a[k]; ap[k] = p[k] - a[k]; }
    auto dot = [](const double *x, const double *y) { return x[0] * y[0] + x[1] * y[1] + x[2] * y[2]; };
    const double d1 = dot(ab, ap), d2 = dot(ac, ap);
    if (d1 <= 0 && d2 <= 0) {
        for (int k = 0; k < 3; ++k) q[k] = a[k];
    } else {
        double bp[3], cp[3];
        for (int k = 0; k < 3; ++k) { bp[k] = p[k] - b[k]; cp[k] = p[k] - c[k]; }
        const double d3 = dot(ab, bp), d4 = dot(ac, bp), d5 = dot(ab, cp), d6 = dot(ac, cp);
        const double vc = d1 * d4 - d3 * d2, vb = d5 * d2 - d1 * d6, va = d3 * d6 - d5 * d4;
        if (d3 >= 0 && d4 <= d3) {
            for (int k = 0; k < 3; ++k) q[k] = b[k];
        } else if (vc <= 0 && d1 >= 0 && d3 <= 0) {
            const double v = d1 / (d1 - d3);
            for (int k = 0; k < 3; ++k) q[k] = a[k] + v * ab[k];
        } else if (d6 >= 0 && d5 <= d6) {
            for (int k = 0; k < 3; ++k) q[k] = c[k];
        } else if (vb <= 0 && d2 >= 0 && d6 <= 0) {
            const double w = d2 / (d2 - d6);
            for (int k = 0; k < 3; ++k) q[k] = a[k] + w * ac[k];
        } else if (va <= 0 && (d4 - d3) >= 0 && (d5 - d6) >= 0) {
            const double w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
            for (int k = 0; k < 3; ++k) q[k] = b[k] + w * (c[k] - b[k]);
        } else {
            const double den = 1.0 / (va + vb + vc), v = vb * den, w = vc * den;
            for (int k = 0; k < 3; ++k) q[k] = a[k] + ab[k] * v + ac[k] * w;
        }
    }
    const double d[3] = {p[0] - q[0], p[1] - q[1], p[2] - q[2]};
    return dot(d, d);
}

__global__ void k_sdf(vmsk::SurfDev S, DistGrid G, const double *px, const double *py,
                      const double *pz, int64_t n, double trunc, double *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double P[3] = {px[i], py[i], pz[i]};
    double best = trunc * trunc;
    int lo[3], hi[3];
    bool any = true;
    for (int k = 0; k < 3; ++k) {
        const double fl = fmin(fmax(floor((P[k] - trunc - G.g0[k]) / G.cell), -1.0), (double)G.n[k]);
        const double fh = fmin(fmax(floor((P[k] + trunc - G.g0[k]) / G.cell), -1.0), (double)G.n[k]);
        lo[k] = (int)fl;
        hi[k] = (int)fh;
        if (hi[k] < 0 || lo[k] >= G.n[k]) any = false;
        lo[k] = max(lo[k], 0);
        hi[k] = min(hi[k], G.n[k] - 1);
    }
    if (any)
        for (int z = lo[2]; z <= hi[2]; ++z)
            for (int y = lo[1]; y <= hi[1]; ++y)
                for (int x = lo[0]; x <= hi[0]; ++x) {
                    const int c = (z * G.n[1] + y) * G.n[0] + x;
                    for (int j = G.off[c]; j < G.off[c + 1]; ++j) {
                        const double *tv = S.tv + 9 * (int64_t)G.ids[j];
                        const double d2 = tri_dist2(P, tv, tv + 3, tv + 6);
                        if (d2 < best) best = d2;
                    }
                }
    const double d = sqrt(best);
    const int lab = vmsk::ray_label(S, P, nullptr);
    out[i] = lab ? -d : d;
}

}  // namespace vmsm

// ---------------------------------------------------------------------------
// C-ABI of the network
// ---------------------------------------------------------------------------

struct vmsm::MlpHandle {
    hipStream_t stream = nullptr;
    float *theta = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr, *B = nullptr;
    _Float16 *w16 = nullptr;
    double *loss = nullptr;
    double lo[3], hi[3];
    float trunc = 0.1f, margin = INFINITY;
    float *mgrid = nullptr;  // per-cell margins over the network box (nullable)
    int gn[3] = {0, 0, 0};
    int64_t step = 0;
    vmsm::MarginGrid grid() const {
        vmsm::MarginGrid g{};
        g.m = mgrid;
        for (int k = 0; k < 3; ++k) {
            g.n[k] = gn[k];
            g.lo[k] = lo[k];
            g.inv[k] = gn[k] > 0 ? gn[k] / (hi[k] - lo[k]) : 0.0;
        }
        return g;
    }
    vmsm::Net net() const {
        vmsm::Net t{};
        t.theta = theta;
        t.w16 = w16;
        t.B = B;
        for (int k = 0; k < 3; ++k) {
            t.lo[k] = (float)lo[k];
            t.inv[k] = (float)(1.0 / (hi[k] - lo[k]));
            t.blo[k] = lo[k];
            t.bhi[k] = hi[k];
        }
        return t;
    }
    ~MlpHandle() {
        for (void *p : {(void *)theta, (void *)m, (void *)v, (void *)grad, (void *)B, (void *)w16,
                        (void *)loss, (void *)mgrid})
            if (p) (void)hipFree(p);
    }
};

namespace vmsm {
__global__ void k_zero_count(unsigned long long *c) {
    if (threadIdx.x == 0) *c = 0ull;
}

int reserve_filter(Filter &f, int64_t n) {
    if (n <= f.cap) return VMS_OK;
    f.release();
    if (hipMalloc(&f.d_idx, n * sizeof(int64_t)) || hipMalloc(&f.d_count, sizeof(unsigned long long)) ||
        hipMalloc(&f.d_pred, n * sizeof(float))) {
        f.release();
        return VMS_ENOMEM;
    }
    f.cap = n;
    return VMS_OK;
}

Net mlp_net(const MlpHandle *h) { return h->net(); }
MarginGrid mlp_grid(const MlpHandle *h) { return h->grid(); }
float mlp_margin(const MlpHandle *h) { return h->margin; }

int classify_learned(hipStream_t s, Filter &f, const MlpHandle *h, const vmsk::SurfDev &S,
                     const double *px, const double *py, const double *pz, int64_t n,
                     uint8_t *labels) {
    if (n <= 0) return VMS_OK;
    int rc = reserve_filter(f, n);  // allocates only beyond the reserved capacity
    if (rc) return rc;
    hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(64), 0, s, f.d_count);
    launch_predict(s, h->net(), px, py, pz, n, f.d_pred);
    launch_decide(s, f.d_pred, n, h->margin, h->grid(), px, py, pz, labels, f.d_idx, f.d_count);
    vmsk::launch_point_labels_list(s, S, f.d_idx, f.d_count, n, px, py, pz, labels, nullptr);
    return VMS_OK;
}
}  // namespace vmsm

namespace {
std::string g_mlp_err = "no error";
int mfail(int code, const char *msg) {
    g_mlp_err = msg;
    return code;
}
}  // namespace

extern "C" {

int vms_mlp_create(vms_mlp **out, const double *lo, const double *hi, const float *theta,
                   const float *B, float trunc, void *stream) {
    if (!out || !lo || !hi || !theta || !B) return mfail(VMS_EINVAL, "null argument");
    *out = nullptr;
    for (int k = 0; k < 3; ++k)
        if (!(hi[k] > lo[k])) return mfail(VMS_EINVAL, "empty box");
    if (!(trunc > 0)) return mfail(VMS_EINVAL, "truncation must be positive");
    auto *h = new vmsm::MlpHandle();
    h->stream = (hipStream_t)stream;
    for (int k = 0; k < 3; ++k) { h->lo[k] = lo[k]; h->hi[k] = hi[k]; }
    h->trunc = trunc;
    const size_t P = vmsm::N_PARAMS * sizeof(float);
    if (hipMalloc(&h->theta, P) || hipMalloc(&h->m, P) || hipMalloc(&h->v, P) || hipMalloc(&h->grad, P) ||
        hipMalloc(&h->B, vmsm::NF * 3 * sizeof(float)) ||
        hipMalloc(&h->w16, 3 * vmsm::H * vmsm::H * sizeof(_Float16)) || hipMalloc(&h->loss, sizeof(double))) {
        delete h;
        return mfail(VMS_ENOMEM, "device allocation failed (network)");
    }
    if (hipMemcpyAsync(h->theta, theta, P, hipMemcpyHostToDevice, h->stream) ||
        hipMemcpyAsync(h->B, B, vmsm::NF * 3 * sizeof(float), hipMemcpyHostToDevice, h->stream) ||
        hipMemsetAsync(h->m, 0, P, h->stream) || hipMemsetAsync(h->v, 0, P, h->stream)) {
        delete h;
        return mfail(VMS_EHIP, "device copy failed (network)");
    }
    hipLaunchKernelGGL(vmsm::k_to_half, dim3((3 * 4096 + 255) / 256), dim3(256), 0, h->stream, h->theta, h->w16);
    if (hipStreamSynchronize(h->stream)) {
        delete h;
        return mfail(VMS_EHIP, "network initialisation failed");
    }
    *out = (vms_mlp *)h;
    return VMS_OK;
}

void vms_mlp_destroy(vms_mlp *m) {
    auto *h = (vmsm::MlpHandle *)m;
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    delete h;
}

int vms_mlp_get_params(vms_mlp *m, float *theta) {
    auto *h = (vmsm::MlpHandle *)m;
    if (!h || !theta) return mfail(VMS_EINVAL, "null argument");
    if (hipMemcpyAsync(theta, h->theta, vmsm::N_PARAMS * sizeof(float), hipMemcpyDeviceToHost, h->stream) ||
        hipStreamSynchronize(h->stream))
        return mfail(VMS_EHIP, "copy failed");
    return VMS_OK;
}

int vms_mlp_set_margin(vms_mlp *m, float margin) {
    auto *h = (vmsm::MlpHandle *)m;
    if (!h || !(margin >= 0)) return mfail(VMS_EINVAL, "bad margin");
    h->margin = margin;
    return VMS_OK;
}

int vms_mlp_set_margin_grid(vms_mlp *m, int nx, int ny, int nz, const float *margins) {
    auto *h = (vmsm::MlpHandle *)m;
    if (!h) return mfail(VMS_EINVAL, "null handle");
    if (h->mgrid) {
        (void)hipStreamSynchronize(h->stream);
        (void)hipFree(h->mgrid);
        h->mgrid = nullptr;
        h->gn[0] = h->gn[1] = h->gn[2] = 0;
    }
    if (nx == 0 && ny == 0 && nz == 0) return VMS_OK;
    if (nx <= 0 || ny <= 0 || nz <= 0 || !margins || (int64_t)nx * ny * nz > (1 << 24))
        return mfail(VMS_EINVAL, "bad margin grid");
    const int64_t nc = (int64_t)nx * ny * nz;
    for (int64_t c = 0; c < nc; ++c)
        if (!(margins[c] >= 0)) return mfail(VMS_EINVAL, "bad margin in grid");
    if (hipMalloc(&h->mgrid, nc * sizeof(float)) != hipSuccess) return mfail(VMS_ENOMEM, "allocation failed");
    if (hipMemcpy(h->mgrid, margins, nc * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
        return mfail(VMS_EHIP, "copy failed");
    h->gn[0] = nx;
    h->gn[1] = ny;
    h->gn[2] = nz;
    return VMS_OK;
}

static void launch_grad(vmsm::MlpHandle *h, const double *px, const double *py, const double *pz,
                        const double *sdf, int64_t n, int64_t first, int64_t count) {
    hipLaunchKernelGGL(vmsm::k_grad, dim3((unsigned)((count + vmsm::S - 1) / vmsm::S)), dim3(256), 0,
                       h->stream, h->net(), px, py, pz, sdf, n, first, count, h->trunc, h->grad, h->loss);
}

int vms_mlp_grad(vms_mlp *m, const double *px, const double *py, const double *pz, const double *sdf,
                 int64_t n, float *grad, double *loss) {
    auto *h = (vmsm::MlpHandle *)m;
    if (!h || !px || !py || !pz || !sdf || n <= 0) return mfail(VMS_EINVAL, "null argument or empty batch");
    if (hipMemsetAsync(h->grad, 0, vmsm::N_PARAMS * sizeof(float), h->stream) ||
        hipMemsetAsync(h->loss, 0, sizeof(double), h->stream))
        return mfail(VMS_EHIP, "memset failed");
    launch_grad(h, px, py, pz, sdf, n, 0, n);
    if (grad && hipMemcpyAsync(grad, h->grad, vmsm::N_PARAMS * sizeof(float), hipMemcpyDeviceToDevice, h->stream))
        return mfail(VMS_EHIP, "copy failed");
    double l = 0;
    if (hipMemcpyAsync(&l, h->loss, sizeof(double), hipMemcpyDeviceToHost, h->stream) ||
        hipStreamSynchronize(h->stream))
        return mfail(VMS_EHIP, "gradient kernel failed");
    if (loss) *loss = l / (double)n;
    return hipGetLastError() == hipSuccess ? VMS_OK : mfail(VMS_EHIP, "launch failed");
}

int vms_mlp_train(vms_mlp *m, const double *px, const double *py, const double *pz, const double *sdf,
                  int64_t n, int steps, int batch, float lr, double *last_loss) {
    auto *h = (vmsm::MlpHandle *)m;
    if (!h || !px || !py || !pz || !sdf || n <= 0 || steps < 0 || batch <= 0 || !(lr > 0))
        return mfail(VMS_EINVAL, "bad training arguments");
    double lsum = 0;
    for (int it = 0; it < steps; ++it) {
        const int64_t first = ((int64_t)it * batch) % n;
        if (hipMemsetAsync(h->grad, 0, vmsm::N_PARAMS * sizeof(float), h->stream) ||
            hipMemsetAsync(h->loss, 0, sizeof(double), h->stream))
            return mfail(VMS_EHIP, "memset failed");
        launch_grad(h, px, py, pz, sdf, n, first, batch);
        ++h->step;
        const float c1 = 1.0f - powf(0.9f, (float)h->step), c2 = 1.0f - powf(0.999f, (float)h->step);
        hipLaunchKernelGGL(vmsm::k_adam, dim3((vmsm::N_PARAMS + 255) / 256), dim3(256), 0, h->stream, h->theta,
                           h->m, h->v, h->grad, vmsm::N_PARAMS, lr, c1, c2);
        if (it == steps - 1) {
            if (hipMemcpyAsync(&lsum, h->loss, sizeof(double), hipMemcpyDeviceToHost, h->stream))
                return mfail(VMS_EHIP, "copy failed");
        }
    }
    hipLaunchKernelGGL(vmsm::k_to_half, dim3((3 * 4096 + 255) / 256), dim3(256), 0, h->stream, h->theta, h->w16);
    if (hipStreamSynchronize(h->stream) || hipGetLastError() != hipSuccess)
        return mfail(VMS_EHIP, "training kernels failed");
    if (last_loss) *last_loss = lsum / (double)batch;
    return VMS_OK;
}

int vms_mlp_adam_step(vms_mlp *m, const float *grad, float lr) {
    auto *h = (vmsm::MlpHandle *)m;
    if (!h || !grad) return mfail(VMS_EINVAL, "null argument");
    if (hipMemcpyAsync(h->grad, grad, vmsm::N_PARAMS * sizeof(float), hipMemcpyDeviceToDevice, h->stream))
        return mfail(VMS_EHIP, "copy failed");
    ++h->step;
    const float c1 = 1.0f - powf(0.9f, (float)h->step), c2 = 1.0f - powf(0.999f, (float)h->step);
    hipLaunchKernelGGL(vmsm::k_adam, dim3((vmsm::N_PARAMS + 255) / 256), dim3(256), 0, h->stream, h->theta, h->m,
                       h->v, h->grad, vmsm::N_PARAMS, lr, c1, c2);
    hipLaunchKernelGGL(vmsm::k_to_half, dim3((3 * 4096 + 255) / 256), dim3(256), 0, h->stream, h->theta, h->w16);
    return hipGetLastError() == hipSuccess ? VMS_OK : mfail(VMS_EHIP, "launch failed");
}

int vms_mlp_predict(vms_mlp *m, const double *px, const double *py, const double *pz, int64_t n, float *pred) {
    auto *h = (vmsm::MlpHandle *)m;
    if (!h || n < 0 || (n > 0 && (!px || !py || !pz || !pred))) return mfail(VMS_EINVAL, "bad arguments");
    vmsm::launch_predict(h->stream, h->net(), px, py, pz, n, pred);
    return hipGetLastError() == hipSuccess ? VMS_OK : mfail(VMS_EHIP, "launch failed");
}

const char *vms_mlp_last_error(void) { return g_mlp_err.c_str(); }

}  // extern "C"

// exact truncated signed distances for an in-out handle's surface
int vmsm_sdf(hipStream_t s, const vmsk::SurfDev &S, const std::vector<double> &tv, const double *lo,
             const double *hi, const double *px, const double *py, const double *pz, int64_t n,
             double trunc, double *out) {
    using namespace vmsm;
    if (n <= 0) return VMS_OK;
    DistGrid G{};
    double ext = 0;
    for (int k = 0; k < 3; ++k) ext = std::max(ext, hi[k] - lo[k] + 2 * trunc);
    G.cell = std::max(trunc, ext / 128.0);
    for (int k = 0; k < 3; ++k) {
        G.g0[k] = lo[k] - trunc;
        G.n[k] = std::max(1, (int)std::ceil((hi[k] - lo[k] + 2 * trunc) / G.cell));
    }
    const int64_t nt = (int64_t)tv.size() / 9, nc = (int64_t)G.n[0] * G.n[1] * G.n[2];
    std::vector<int32_t> cnt(nc + 1, 0), ids;
    auto cellr = [&](int64_t t, int k, int &a, int &b) {
        double mn = std::min(tv[9 * t + k], std::min(tv[9 * t + 3 + k], tv[9 * t + 6 + k]));
        double mx = std::max(tv[9 * t + k], std::max(tv[9 * t + 3 + k], tv[9 * t + 6 + k]));
        a = std::max(0, std::min(G.n[k] - 1, (int)std::floor((mn - G.g0[k]) / G.cell)));
        b = std::max(0, std::min(G.n[k] - 1, (int)std::floor((mx - G.g0[k]) / G.cell)));
    };
    for (int pass = 0; pass < 2; ++pass) {
        std::vector<int32_t> fill;
        if (pass == 1) { fill.assign(cnt.begin(), cnt.end() - 1); ids.assign(cnt.back(), 0); }
        for (int64_t t = 0; t < nt; ++t) {
            int a[3], b[3];
            for (int k = 0; k < 3; ++k) cellr(t, k, a[k], b[k]);
            for (int z = a[2]; z <= b[2]; ++z)
                for (int y = a[1]; y <= b[1]; ++y)
                    for (int x = a[0]; x <= b[0]; ++x) {
                        const int64_t c = ((int64_t)z * G.n[1] + y) * G.n[0] + x;
                        if (pass == 0) cnt[c + 1]++;
                        else ids[fill[c]++] = (int32_t)t;
                    }
        }
        if (pass == 0)
            for (int64_t c = 0; c < nc; ++c) cnt[c + 1] += cnt[c];
    }
    int32_t *doff = nullptr, *dids = nullptr;
    if (hipMalloc(&doff, cnt.size() * 4) || hipMalloc(&dids, std::max<size_t>(1, ids.size()) * 4)) {
        if (doff) (void)hipFree(doff);
        return VMS_ENOMEM;
    }
    int rc = VMS_OK;
    if (hipMemcpyAsync(doff, cnt.data(), cnt.size() * 4, hipMemcpyHostToDevice, s) ||
        (ids.size() && hipMemcpyAsync(dids, ids.data(), ids.size() * 4, hipMemcpyHostToDevice, s)))
        rc = VMS_EHIP;
    if (rc == VMS_OK) {
        G.off = doff;
        G.ids = dids;
        hipLaunchKernelGGL(k_sdf, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, s, S, G, px, py, pz, n,
                           trunc, out);
        if (hipStreamSynchronize(s) || hipGetLastError() != hipSuccess) rc = VMS_EHIP;
    }
    (void)hipFree(doff);
    (void)hipFree(dids);
    return rc;
}

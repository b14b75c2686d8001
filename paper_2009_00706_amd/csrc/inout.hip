// In-out tests and adaptive sub-cell quadrature of libvms (gfx950).
//
// Labels are exact point-in-polyhedron membership (1 = inside or on the
// surface, 0 = fluid), the truth that the paper's normal-based test (Alg. 5)
// and its ray-tracing fallback estimate:
//   * ray_label: parity of crossings of the segment from P along +x to a point
//     beyond the surface's box, against the triangles of P's (y, z) bin; on a
//     degenerate crossing (through an edge or a vertex) the next direction of
//     a fixed list is tried against all triangles;
//   * local_label: label(V) XOR parity(P -> V) for a corner V of the element
//     holding P, against the element's background triangles B_T (every
//     triangle whose box meets the closed element, so every triangle the
//     segment can cross). Used for sub-cell Gauss points; corners are tried
//     in order and ray_label is the last resort.
// Sub-cell quadrature (Section "Adaptive Quadrature" and the caption of its
// Gauss-point figure): an INTERCEPTED element is split; a sub-cell whose 8
// Gauss points are all fluid is kept whole, all solid dropped, mixed split
// again, and at the maximum level only fluid points are kept.
#include "inout_dev.h"

namespace vmsk {
using namespace vmsd;

__global__ void k_vertex_labels(SurfDev S, GeoArgs g, int64_t n, const int32_t *ix,
                                const int32_t *iy, const int32_t *iz, uint8_t *lab,
                                unsigned long long *ndeg) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double sc = ldexp(1.0, -g.max_level);
    double P[3];
    const int32_t *ii[3] = {ix, iy, iz};
    for (int k = 0; k < 3; ++k) P[k] = point_coord(g.origin[k], g.root_len, sc, ii[k][i], 0, 0.0);
    lab[i] = (uint8_t)ray_label(S, P, ndeg);
}

__global__ void k_point_labels(SurfDev S, int64_t n, const double *px, const double *py,
                               const double *pz, uint8_t *lab, unsigned long long *ndeg) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double P[3] = {px[i], py[i], pz[i]};
    lab[i] = (uint8_t)ray_label(S, P, ndeg);
}

__global__ void k_point_labels_list(SurfDev S, const int64_t *idx, const unsigned long long *count,
                                    int64_t cap, const double *px, const double *py,
                                    const double *pz, uint8_t *lab, unsigned long long *ndeg) {
    int64_t n = (int64_t)*count;
    if (n > cap) n = cap;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        int64_t i = idx[j];
        double P[3] = {px[i], py[i], pz[i]};
        lab[i] = (uint8_t)ray_label(S, P, ndeg);
    }
}

void launch_vertex_labels(hipStream_t s, const SurfDev &S, const GeoArgs &g, int64_t n,
                          const int32_t *ix, const int32_t *iy, const int32_t *iz, uint8_t *lab,
                          unsigned long long *ndeg) {
    if (n <= 0) return;
    int64_t nb = (n + 127) / 128;
    hipLaunchKernelGGL(k_vertex_labels, dim3((unsigned)nb), dim3(128), 0, s, S, g, n, ix, iy, iz,
                       lab, ndeg);
}

void launch_point_labels(hipStream_t s, const SurfDev &S, int64_t n, const double *px,
                         const double *py, const double *pz, uint8_t *lab,
                         unsigned long long *ndeg) {
    if (n <= 0) return;
    int64_t nb = (n + 127) / 128;
    hipLaunchKernelGGL(k_point_labels, dim3((unsigned)nb), dim3(128), 0, s, S, n, px, py, pz, lab,
                       ndeg);
}

void launch_point_labels_list(hipStream_t s, const SurfDev &S, const int64_t *idx,
                              const unsigned long long *count, int64_t cap, const double *px,
                              const double *py, const double *pz, uint8_t *lab,
                              unsigned long long *ndeg) {
    if (cap <= 0) return;
    int64_t nb = (cap + 127) / 128;
    if (nb > 8192) nb = 8192;
    hipLaunchKernelGGL(k_point_labels_list, dim3((unsigned)nb), dim3(128), 0, s, S, idx, count, cap,
                       px, py, pz, lab, ndeg);
}

// ---------------------------------------------------------------------------
// Adaptive sub-cell quadrature: one 64-lane workgroup per INTERCEPTED element
// ---------------------------------------------------------------------------

constexpr int SQ_MAXCELL = 512;   // cells of one level at depth <= 3
constexpr int SQ_MAXKEEP = 4096;  // 8 * 8^3 points

__global__ __launch_bounds__(64) void k_subquad(SurfDev S, GeoArgs g, SubqArgs a, int pass) {
    __shared__ uint32_t cells[2][SQ_MAXCELL];   // path digits, level 1 most significant
    __shared__ uint32_t keep[SQ_MAXKEEP];       // key << 2 | level
    __shared__ int ncell[2], nkeep;
    __shared__ double V[8][3];
    __shared__ uint8_t vl[8];
    const int lane = threadIdx.x;
    const int64_t i = blockIdx.x;
    if (i >= a.n) return;
    const int e = a.el[i];
    const int D = g.depth;
    const int M = g.max_level;
    const int F = M + D;
    const double scF = ldexp(1.0, -F);
    const int64_t SE = (int64_t)1 << (M - a.level[i] + D);  // element side, fine units
    const int64_t A0[3] = {(int64_t)a.ax[i] << D, (int64_t)a.ay[i] << D, (int64_t)a.az[i] << D};
    if (lane < 8) {
        for (int k = 0; k < 3; ++k)
            V[lane][k] = point_coord(g.origin[k], g.root_len, scF,
                                     A0[k] + (((lane >> k) & 1) ? SE : 0), 0, 0.0);
        vl[lane] = a.corner_lab[8 * i + lane];
    }
    if (lane == 0) {
        nkeep = 0;
        ncell[0] = 0;
        ncell[1] = 0;
    }
    __syncthreads();
    const int32_t *bt = a.bt_ids + a.bt_off[i];
    const int nbt = (int)(a.bt_off[i + 1] - a.bt_off[i]);
    int cur = 0;
    int lmin = 1;
    if (D == 0) {
        if (lane == 0) { cells[0][0] = 0; ncell[0] = 1; }
        lmin = 0;
    } else if (lane < 8) {
        cells[0][lane] = lane;
        if (lane == 0) ncell[0] = 8;
    }
    __syncthreads();
    unsigned long long nlab = 0;
    for (int l = lmin; l <= D; ++l) {
        const int nc = ncell[cur];
        const int nxt = cur ^ 1;
        if (lane == 0) ncell[nxt] = 0;
        __syncthreads();
        const int64_t S_l = SE >> l;
        for (int base = 0; base < nc * 8; base += 64) {
            const int idx = base + lane;
            const bool valid = idx < nc * 8;
            const int c = idx >> 3, gp = idx & 7;
            int lab = 1;
            uint32_t path = 0;
            if (valid) {
                path = cells[cur][c];
                int64_t A[3] = {A0[0], A0[1], A0[2]};
                for (int k = 1; k <= l; ++k) {
                    uint32_t dgt = (path >> (3 * (l - k))) & 7u;
                    for (int ax = 0; ax < 3; ++ax)
                        if ((dgt >> ax) & 1u) A[ax] += SE >> k;
                }
                double P[3];
                for (int ax = 0; ax < 3; ++ax)
                    P[ax] = point_coord(g.origin[ax], g.root_len, scF, A[ax], S_l,
                                        ((gp >> ax) & 1) ? VMS_GP : VMS_GM);
                lab = local_label(S, P, V, vl, bt, nbt, a.ndeg);
                ++nlab;
            }
            // labels of the 8 points of each cell in this chunk
            unsigned long long inmask = __ballot(valid && lab);
            int nin = __popcll((inmask >> (lane & ~7)) & 0xffull);
            if (valid) {
                bool leaf = (l == D) || nin == 0;
                if (leaf && !lab) {
                    int slot = atomicAdd(&nkeep, 1);
                    uint32_t key = (((path << 3) | (uint32_t)gp) << (3 * (D - l)));
                    if (slot < SQ_MAXKEEP) keep[slot] = (key << 2) | (uint32_t)l;
                } else if (!leaf && nin < 8 && gp == 0) {
                    int slot = atomicAdd(&ncell[nxt], 8);
                    for (int ch = 0; ch < 8; ++ch)
                        if (slot + ch < SQ_MAXCELL) cells[nxt][slot + ch] = (path << 3) | ch;
                }
            }
        }
        __syncthreads();
        cur = nxt;
    }
    if (nlab && pass == 0) atomicAdd(a.nlabel, nlab);
    const int nk = nkeep;
    if (pass == 0) {
        if (lane == 0) a.cnt[i] = nk;
        return;
    }
    if (nk != a.cnt[i]) {  // relabelling must reproduce the point count of the arena slot
        if (lane == 0) atomicOr(a.flag, 1u);
        return;
    }
    // bitonic sort of the kept entries (keys are unique), padded with ~0
    int np2 = 1;
    while (np2 < nk) np2 <<= 1;
    for (int j = nk + lane; j < np2; j += 64) keep[j] = 0xffffffffu;
    __syncthreads();
    for (int k = 2; k <= np2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = lane; t < np2; t += 64) {
                int p = t ^ j;
                if (p > t) {
                    uint32_t x = keep[t], y = keep[p];
                    bool up = (t & k) == 0;
                    if ((x > y) == up) { keep[t] = y; keep[p] = x; }
                }
            }
            __syncthreads();
        }
    }
    uint32_t *dst = a.entries + a.off[i];
    for (int j = lane; j < nk; j += 64) dst[j] = keep[j];
}

void launch_subquad(hipStream_t s, const SurfDev &S, const GeoArgs &g, const SubqArgs &a,
                    int pass) {
    if (a.n <= 0) return;
    hipLaunchKernelGGL(k_subquad, dim3((unsigned)a.n), dim3(64), 0, s, S, g, a, pass);
}

}  // namespace vmsk

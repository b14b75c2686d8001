// In-out tests and adaptive sub-cell quadrature of libvms (gfx950).
//
// Labels are exact point-in-polyhedron membership (1 = inside or on the
// surface, 0 = fluid), the truth that the paper's normal-based test (Alg. 5)
// and its ray-tracing fallback estimate:
//   * ray_label: parity of crossings of the segment from P along +x or -x
//     (towards the nearer end of the surface's box) to a point beyond that
//     box, against the triangles of P's (y, z) bin; on a degenerate crossing
//     (through an edge or a vertex) the next direction of a fixed list is
//     tried against all triangles;
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
#include "mlp_dev.h"

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

constexpr int SQ_MAXCELL = 512;  // cells of one level at depth <= 3
constexpr int SQ_KEYS = 4096;    // key space 8^(D+1) at depth 3
constexpr int SQ_BTMAX = 64;     // background triangles staged in LDS

// Exact label of P by local segments to the element corners V, with the
// element's background triangles read from LDS (tv: 9 doubles, tb: box);
// corners tried from v0 (the one nearest P: shortest segment, fewest
// triangle boxes crossed) in the order v0 ^ j.
__device__ static int local_label_lds(const SurfDev &S, const double *P, const double (*V)[3],
                                      const uint8_t *vlab, const double (*tv)[9],
                                      const double (*tb)[6], int nbt, unsigned long long *ndeg,
                                      int v0) {
    for (int j = 0; j < 8; ++j) {
        const int v = v0 ^ j;
        int cnt = 0;
        bool deg = false;
        const double *Q = V[v];
        for (int i = 0; i < nbt; ++i) {
            const double *bx = tb[i];
            bool miss = false;
            for (int k = 0; k < 3; ++k) {
                const double lo = fmin(P[k], Q[k]), hi = fmax(P[k], Q[k]);
                if (hi < bx[k] || lo > bx[3 + k]) miss = true;
            }
            if (miss) continue;
            const int r = segment_triangle(P, Q, tv[i], tv[i] + 3, tv[i] + 6);
            if (r == SEG_ON) return 1;
            if (r == SEG_DEGEN) deg = true;
            else cnt ^= r;
        }
        if (!deg) return vlab[v] ^ cnt;
        if (ndeg) atomicAdd(ndeg, 1ull);
    }
    return ray_label(S, P, ndeg);
}

// One 64-lane workgroup per INTERCEPTED element. Sub-cells are split level by
// level; a kept point sets the bit of its key (and records its level) in a
// bitmap over the key space, so that the canonical (ascending key) position
// of every kept point is the number of set bits below it: no sort is needed.
// FILT 1 (learned): on elements with at least min_bt background triangles
// the 64 candidate points of a batch first go through the signed-distance
// network; a point whose |prediction| reaches its margin takes the network's
// sign, every other point the exact test. FILT 2 (normal-based, Alg. 5 as a
// certified filter): a point strictly outside the plane of one background
// triangle of each of the element's bodies (all convex) is OUT; the others
// take the exact test.
template <int FILT>
__global__ __launch_bounds__(64) void k_subquad(SurfDev S, GeoArgs g, SubqArgs a, int pass) {
    constexpr bool LEARNED = FILT == 1, NORMAL = FILT == 2;
    __shared__ uint32_t cells[2][SQ_MAXCELL];  // path digits, level 1 most significant
    __shared__ unsigned long long kbits[SQ_KEYS / 64];
    __shared__ uint32_t klev[SQ_KEYS / 16];    // 2 bits per key
    __shared__ int ncell[2];
    __shared__ double V[8][3];
    __shared__ uint8_t vl[8];
    __shared__ double tv[SQ_BTMAX][9];
    __shared__ double tb[SQ_BTMAX][6];
    __shared__ uint8_t tlc[NORMAL ? SQ_BTMAX : 1];
    __shared__ __attribute__((aligned(16))) _Float16 act[LEARNED ? 64 : 1][vmsm::LDH];
    const int lane = threadIdx.x;
    const int64_t i = a.order ? (int64_t)a.order[blockIdx.x] : (int64_t)blockIdx.x;
    if (i < 0 || i >= a.n) return;
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
        ncell[0] = 0;
        ncell[1] = 0;
    }
    kbits[lane] = 0ull;
    for (int k = lane; k < SQ_KEYS / 16; k += 64) klev[k] = 0u;
    const int32_t *bt = a.bt_ids + a.bt_off[i];
    const int nbt = (int)(a.bt_off[i + 1] - a.bt_off[i]);
    const bool staged = nbt <= SQ_BTMAX;
    const bool use_net = LEARNED && nbt >= a.learned.min_bt;  // uniform over the workgroup
    const unsigned nmask = (NORMAL && staged && pass == 1) ? a.nmask[i] : 0u;
    if (staged)
        for (int t = lane; t < nbt; t += 64) {
            const int id = bt[t];
            for (int k = 0; k < 9; ++k) tv[t][k] = S.tv[9 * (int64_t)id + k];
            for (int k = 0; k < 6; ++k) tb[t][k] = S.tbox[6 * (int64_t)id + k];
            if constexpr (NORMAL) tlc[t] = a.bt_lc[a.bt_off[i] + t];
        }
    __syncthreads();
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
            double P[3] = {0.0, 0.0, 0.0};
            int v0 = 0;
            if (valid) {
                path = cells[cur][c];
                int64_t A[3] = {A0[0], A0[1], A0[2]};
                for (int k = 1; k <= l; ++k) {
                    uint32_t dgt = (path >> (3 * (l - k))) & 7u;
                    for (int ax = 0; ax < 3; ++ax)
                        if ((dgt >> ax) & 1u) A[ax] += SE >> k;
                }
                for (int ax = 0; ax < 3; ++ax)
                    P[ax] = point_coord(g.origin[ax], g.root_len, scF, A[ax], S_l,
                                        ((gp >> ax) & 1) ? VMS_GP : VMS_GM);
                // the corner nearest P: the element octant of P's sub-cell (a
                // sub-cell of level 1 or deeper never straddles the element's midplanes)
                for (int ax = 0; ax < 3; ++ax)
                    if (2 * (A[ax] - A0[ax]) + S_l > SE) v0 |= 1 << ax;
            }
            bool decided = false;
            if constexpr (LEARNED) {
                if (use_net) {
                    const float y = vmsm::net_output64(a.learned.net, P, valid, act);
                    if (valid && fabsf(y) >= vmsm::point_margin(a.learned.grid, a.learned.margin, P)) {
                        lab = y < 0.f ? 1 : 0;
                        decided = true;
                    }
                }
            }
            if constexpr (NORMAL) {
                if (valid && nmask) {
                    // strictly on the outer side of a triangle of every body present
                    unsigned got = 0;
                    for (int t = 0; t < nbt && got != nmask; ++t) {
                        const unsigned bit = 1u << tlc[t];
                        if (got & bit) continue;
                        if (orient3d(tv[t], tv[t] + 3, tv[t] + 6, P) < 0) got |= bit;
                    }
                    if (got == nmask) {
                        lab = 0;
                        decided = true;
                    }
                }
            }
            if (valid && !decided) {
                lab = staged ? local_label_lds(S, P, V, vl, tv, tb, nbt, a.ndeg, v0)
                             : local_label(S, P, V, vl, bt, nbt, a.ndeg, v0);
                ++nlab;
            }
            // labels of the 8 points of each cell in this chunk
            unsigned long long inmask = __ballot(valid && lab);
            int nin = __popcll((inmask >> (lane & ~7)) & 0xffull);
            if (valid) {
                bool leaf = (l == D) || nin == 0;
                if (leaf && !lab) {
                    const uint32_t key = (((path << 3) | (uint32_t)gp) << (3 * (D - l)));
                    atomicOr(&kbits[key >> 6], 1ull << (key & 63));
                    atomicOr(&klev[key >> 4], (uint32_t)l << (2 * (key & 15)));
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
    if (nlab && pass == 1 && a.nexact) atomicAdd(a.nexact, nlab);
    // kept points: set bits of the bitmap; lane w owns word w
    const unsigned long long word = kbits[lane];
    const int cw = __popcll(word);
    // exclusive prefix sum of the word counts over the 64 lanes
    int incl = cw;
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(incl, d, 64);
        if (lane >= d) incl += y;
    }
    const int nk = __shfl(incl, 63, 64);
    if (pass == 0) {
        if (lane == 0) a.cnt[i] = nk;
        return;
    }
    if (nk != a.cnt[i]) {  // relabelling must reproduce the point count of the arena slot
        if (lane == 0) atomicOr(a.flag, 1u);
        return;
    }
    // write the kept entries in ascending key order: (key << 2) | level
    uint32_t *dst = a.entries + a.off[i] + (incl - cw);
    unsigned long long wbits = word;
    int r = 0;
    while (wbits) {
        const int b = __ffsll((long long)wbits) - 1;
        wbits &= wbits - 1;
        const uint32_t key = (uint32_t)lane * 64u + (uint32_t)b;
        const uint32_t lv = (klev[key >> 4] >> (2 * (key & 15))) & 3u;
        dst[r++] = (key << 2) | lv;
    }
}

__global__ void k_zero_u64(unsigned long long *c) {
    if (threadIdx.x == 0) *c = 0ull;
}

void launch_zero_u64(hipStream_t s, unsigned long long *c) {
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, c);
}

void launch_subquad(hipStream_t s, const SurfDev &S, const GeoArgs &g, const SubqArgs &a,
                    int pass, int wg_per_cu) {
    const int64_t n = a.order ? a.n_order : a.n;
    if (n <= 0) return;
    if (a.learned.net.theta) {
        const size_t dyn = pass == 1 ? lds_for_cap((const void *)&k_subquad<1>, wg_per_cu) : 0;
        hipLaunchKernelGGL(k_subquad<1>, dim3((unsigned)n), dim3(64), dyn, s, S, g, a, pass);
    } else if (a.normal && pass == 1) {
        const size_t dyn = lds_for_cap((const void *)&k_subquad<2>, wg_per_cu);
        hipLaunchKernelGGL(k_subquad<2>, dim3((unsigned)n), dim3(64), dyn, s, S, g, a, pass);
    } else {
        const size_t dyn = pass == 1 ? lds_for_cap((const void *)&k_subquad<0>, wg_per_cu) : 0;
        hipLaunchKernelGGL(k_subquad<0>, dim3((unsigned)n), dim3(64), dyn, s, S, g, a, pass);
    }
}

int subquad_per_cu() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void *)&k_subquad<0>, 64, 0) != hipSuccess)
        return 0;
    return n;
}

__global__ void k_edge_convex(SurfDev S, const int32_t *t1, const int32_t *t2, const int8_t *corner,
                              int64_t n, uint8_t *bad) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const double *a = S.tv + 9 * (int64_t)t1[e];
    const double *v = S.tv + 9 * (int64_t)t2[e] + 3 * corner[e];
    bad[e] = orient3d(a, a + 3, a + 6, v) < 0 ? 1 : 0;
}

void launch_edge_convex(hipStream_t s, const SurfDev &S, const int32_t *t1, const int32_t *t2,
                        const int8_t *corner, int64_t n, uint8_t *bad) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_edge_convex, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, S, t1, t2, corner,
                       n, bad);
}

}  // namespace vmsk

// Device in-out tests of libvms (internal header, included by the .hip sources).
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
//     segment can cross). Corners are tried starting from a given one (the
//     nearest, for short segments) in the order v0 ^ j; ray_label is the last
//     resort.
#pragma once
#include "geom.h"
#include "kernels.h"

namespace vmsk {
using namespace vmsd;

__device__ inline int bin_of(double v, double v0, double inv, int n) {
    double t = __dmul_rn(__dsub_rn(v, v0), inv);
    int b = (int)floor(t);
    return b < 0 ? 0 : (b >= n ? n - 1 : b);
}

__device__ inline void tri_load(const SurfDev &S, int t, double a[3], double b[3], double c[3]) {
    const double *p = S.tv + 9 * (int64_t)t;
    for (int k = 0; k < 3; ++k) { a[k] = p[k]; b[k] = p[3 + k]; c[k] = p[6 + k]; }
}

__device__ inline bool seg_box_miss(const SurfDev &S, int t, const double *P, const double *Q) {
    const double *bx = S.tbox + 6 * (int64_t)t;
    for (int k = 0; k < 3; ++k) {
        double lo = fmin(P[k], Q[k]), hi = fmax(P[k], Q[k]);
        if (bx[3 + k] < lo || bx[k] > hi) return true;
    }
    return false;
}

// fallback: far point along direction d (index 1..9), all triangles
__device__ __noinline__ static int ray_label_dir(const SurfDev &S, const double *P, int d, bool &deg) {
    double Q[3] = {P[0], P[1], P[2]};
    if (d < 6) {
        int ax = d >> 1;
        Q[ax] = (d & 1) ? __dsub_rn(S.lo[ax], 1.0) : __dadd_rn(S.hi[ax], 1.0);
    } else {
        const double dir[4][3] = {{0.64, 0.48, 0.6}, {-0.6, 0.64, 0.48}, {0.48, -0.6, 0.64},
                                  {-0.48, -0.64, -0.6}};
        double span = (S.hi[0] - S.lo[0]) + (S.hi[1] - S.lo[1]) + (S.hi[2] - S.lo[2]) + 1.0;
        for (int k = 0; k < 3; ++k) Q[k] = P[k] + 2.0 * span * dir[d - 6][k];
    }
    int cnt = 0;
    deg = false;
    for (int t = 0; t < S.n_tri; ++t) {
        if (seg_box_miss(S, t, P, Q)) continue;
        double a[3], b[3], c[3];
        tri_load(S, t, a, b, c);
        int r = segment_triangle(P, Q, a, b, c);
        if (r == SEG_ON) return 1;
        if (r == SEG_DEGEN) deg = true;
        else cnt ^= r;
    }
    return cnt;
}

__device__ static int ray_label(const SurfDev &S, const double *P, unsigned long long *ndeg) {
    for (int k = 0; k < 3; ++k)
        if (P[k] < S.lo[k] || P[k] > S.hi[k]) return 0;
    int by = bin_of(P[1], S.y0, S.iny, S.nby), bz = bin_of(P[2], S.z0, S.inz, S.nbz);
    int bin = bz * S.nby + by;
    // along -x when the surface's box ends nearer on that side: only the
    // triangles of the bin on that side of P can be crossed
    const bool neg = __dsub_rn(P[0], S.lo[0]) < __dsub_rn(S.hi[0], P[0]);
    double Q[3] = {neg ? __dsub_rn(S.lo[0], 1.0) : __dadd_rn(S.hi[0], 1.0), P[1], P[2]};
    int cnt = 0;
    bool deg = false;
    for (int i = S.bin_off[bin]; i < S.bin_off[bin + 1]; ++i) {
        int t = S.bin_tri[i];
        const double *bx = S.tbox + 6 * (int64_t)t;
        if ((neg ? bx[0] > P[0] : bx[3] < P[0]) || bx[1] > P[1] || bx[4] < P[1] || bx[2] > P[2] ||
            bx[5] < P[2])
            continue;
        double a[3], b[3], c[3];
        tri_load(S, t, a, b, c);
        int r = segment_triangle(P, Q, a, b, c);
        if (r == SEG_ON) return 1;
        if (r == SEG_DEGEN) deg = true;
        else cnt ^= r;
    }
    if (!deg) return cnt;
    for (int d = 1; d < 10; ++d) {
        if (ndeg) atomicAdd(ndeg, 1ull);
        int lab = ray_label_dir(S, P, d, deg);
        if (!deg) return lab;
    }
    if (ndeg) atomicAdd(ndeg, 1ull);
    return 1;  // every direction degenerate: a point of the surface
}

__device__ static int local_label(const SurfDev &S, const double *P, const double (*V)[3],
                           const uint8_t *vlab, const int32_t *bt, int nbt,
                           unsigned long long *ndeg, int v0 = 0) {
    for (int j = 0; j < 8; ++j) {
        const int v = v0 ^ j;
        int cnt = 0;
        bool deg = false;
        for (int i = 0; i < nbt; ++i) {
            int t = bt[i];
            if (seg_box_miss(S, t, P, V[v])) continue;
            double a[3], b[3], c[3];
            tri_load(S, t, a, b, c);
            int r = segment_triangle(P, V[v], a, b, c);
            if (r == SEG_ON) return 1;
            if (r == SEG_DEGEN) deg = true;
            else cnt ^= r;
        }
        if (!deg) return vlab[v] ^ cnt;
        if (ndeg) atomicAdd(ndeg, 1ull);
    }
    return ray_label(S, P, ndeg);
}

}  // namespace vmsk

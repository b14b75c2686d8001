// Device geometry of libvms: point coordinates and exact orientation
// predicates (internal header, included by the .hip sources).
//
// Exactness: orient3d/orient2d first evaluate the determinant in double
// precision with a forward error bound (Shewchuk 1997, "Adaptive precision
// floating-point arithmetic and fast robust geometric predicates"); when the
// bound cannot certify the sign, the determinant is re-evaluated exactly as a
// sum of exact triple products of two-component differences, and the sign is
// read off the most significant component of the exactly grown expansion.
// All arithmetic uses explicitly rounded intrinsics, so no multiply-add is
// ever contracted.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vmsd {

// (1 -+ 1/sqrt 3) / 2 and 1/sqrt 3, correctly rounded
#define VMS_GM 0x1.b0cb174df99c7p-3
#define VMS_GP 0x1.93cd3a2c8198ep-1
#define VMS_XI 0x1.279a74590331cp-1

// x = origin + root_len * ((A + B*g) * 2^-F), in this order, each step rounded.
__host__ __device__ inline double point_coord(double origin, double root_len, double scale_F,
                                              int64_t A, int64_t B, double g) {
#if defined(__HIP_DEVICE_COMPILE__)
    double t1 = __dmul_rn((double)B, g);
    double t2 = __dadd_rn((double)A, t1);
    double t3 = __dmul_rn(t2, scale_F);  // exact: power of two
    double t4 = __dmul_rn(root_len, t3);
    return __dadd_rn(origin, t4);
#else
    volatile double t1 = (double)B * g;
    volatile double t2 = (double)A + t1;
    volatile double t3 = t2 * scale_F;
    volatile double t4 = root_len * t3;
    volatile double r = origin + t4;
    return r;
#endif
}

// ---- exact expansion helpers ---------------------------------------------

__device__ inline void tsum(double a, double b, double &s, double &e) {
    s = __dadd_rn(a, b);
    double bb = __dsub_rn(s, a);
    double aa = __dsub_rn(s, bb);
    e = __dadd_rn(__dsub_rn(a, aa), __dsub_rn(b, bb));
}

__device__ inline void tprod(double a, double b, double &p, double &e) {
    p = __dmul_rn(a, b);
    e = __fma_rn(a, b, -p);
}

// grow the nonoverlapping expansion h[0..n) (increasing magnitude) by x
__device__ inline int grow(double *h, int n, double x) {
    double q = x;
    int m = 0;
    for (int i = 0; i < n; ++i) {
        double s, e;
        tsum(q, h[i], s, e);
        q = s;
        if (e != 0.0) h[m++] = e;
    }
    if (q != 0.0 || m == 0) h[m++] = q;
    return m;
}

__device__ inline int sign_of(const double *h, int n) {
    for (int i = n - 1; i >= 0; --i) {
        if (h[i] > 0.0) return 1;
        if (h[i] < 0.0) return -1;
    }
    return 0;
}

// exact a*b*c as four doubles summing to the product exactly
__device__ inline void triple(double a, double b, double c, double out[4]) {
    double p, e;
    tprod(a, b, p, e);
    tprod(p, c, out[0], out[1]);
    tprod(e, c, out[2], out[3]);
}

// Exact sign of det[a-d; b-d; c-d] (rare path: only when the filter fails).
__device__ __noinline__ int orient3d_exact(const double *a, const double *b, const double *c,
                                          const double *d) {
    double ad[3][2], bd[3][2], cd[3][2];  // [axis][hi, lo]
    for (int k = 0; k < 3; ++k) {
        tsum(a[k], -d[k], ad[k][0], ad[k][1]);
        tsum(b[k], -d[k], bd[k][0], bd[k][1]);
        tsum(c[k], -d[k], cd[k][0], cd[k][1]);
    }
    // det = adz(bdx cdy - cdx bdy) + bdz(cdx ady - adx cdy) + cdz(adx bdy - bdx ady)
    const double *F[6][3] = {{ad[2], bd[0], cd[1]}, {ad[2], cd[0], bd[1]}, {bd[2], cd[0], ad[1]},
                             {bd[2], ad[0], cd[1]}, {cd[2], ad[0], bd[1]}, {cd[2], bd[0], ad[1]}};
    const double sg[6] = {1.0, -1.0, 1.0, -1.0, 1.0, -1.0};
    double h[200];
    int n = 0;
    for (int t = 0; t < 6; ++t)
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j)
                for (int k = 0; k < 2; ++k) {
                    double q[4];
                    triple(F[t][0][i], F[t][1][j], F[t][2][k], q);
                    for (int r = 0; r < 4; ++r)
                        if (q[r] != 0.0) n = grow(h, n, sg[t] * q[r]);
                }
    return sign_of(h, n);
}

__device__ inline int orient3d(const double *a, const double *b, const double *c, const double *d) {
    double adx = __dsub_rn(a[0], d[0]), ady = __dsub_rn(a[1], d[1]), adz = __dsub_rn(a[2], d[2]);
    double bdx = __dsub_rn(b[0], d[0]), bdy = __dsub_rn(b[1], d[1]), bdz = __dsub_rn(b[2], d[2]);
    double cdx = __dsub_rn(c[0], d[0]), cdy = __dsub_rn(c[1], d[1]), cdz = __dsub_rn(c[2], d[2]);
    double bxcy = __dmul_rn(bdx, cdy), cxby = __dmul_rn(cdx, bdy);
    double cxay = __dmul_rn(cdx, ady), axcy = __dmul_rn(adx, cdy);
    double axby = __dmul_rn(adx, bdy), bxay = __dmul_rn(bdx, ady);
    double det = __dadd_rn(__dadd_rn(__dmul_rn(adz, __dsub_rn(bxcy, cxby)),
                                     __dmul_rn(bdz, __dsub_rn(cxay, axcy))),
                           __dmul_rn(cdz, __dsub_rn(axby, bxay)));
    double perm = __dadd_rn(
        __dadd_rn(__dmul_rn(__dadd_rn(fabs(bxcy), fabs(cxby)), fabs(adz)),
                  __dmul_rn(__dadd_rn(fabs(cxay), fabs(axcy)), fabs(bdz))),
        __dmul_rn(__dadd_rn(fabs(axby), fabs(bxay)), fabs(cdz)));
    // (7 + 56 eps) eps with eps = 2^-53
    const double bound = __dmul_rn((7.0 + 56.0 * 0x1p-53) * 0x1p-53, perm);
    if (det > bound) return 1;
    if (-det > bound) return -1;
    return orient3d_exact(a, b, c, d);
}

// exact sign of det[a-c; b-c] in coordinates (i, j)
__device__ __noinline__ int orient2d_exact(const double *a, const double *b, const double *c,
                                          int i, int j) {
    double ai[2], aj[2], bi[2], bj[2];
    tsum(a[i], -c[i], ai[0], ai[1]);
    tsum(a[j], -c[j], aj[0], aj[1]);
    tsum(b[i], -c[i], bi[0], bi[1]);
    tsum(b[j], -c[j], bj[0], bj[1]);
    double h[40];
    int n = 0;
    for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y) {
            double p, e;
            tprod(ai[x], bj[y], p, e);
            if (p != 0.0) n = grow(h, n, p);
            if (e != 0.0) n = grow(h, n, e);
            tprod(aj[x], bi[y], p, e);
            if (p != 0.0) n = grow(h, n, -p);
            if (e != 0.0) n = grow(h, n, -e);
        }
    return sign_of(h, n);
}

__device__ inline int orient2d(const double *a, const double *b, const double *c, int i, int j) {
    double acx = __dsub_rn(a[i], c[i]), bcx = __dsub_rn(b[i], c[i]);
    double acy = __dsub_rn(a[j], c[j]), bcy = __dsub_rn(b[j], c[j]);
    double l = __dmul_rn(acx, bcy), r = __dmul_rn(acy, bcx);
    double det = __dsub_rn(l, r);
    // (3 + 16 eps) eps
    const double bound = __dmul_rn((3.0 + 16.0 * 0x1p-53) * 0x1p-53, __dadd_rn(fabs(l), fabs(r)));
    if (det > bound) return 1;
    if (-det > bound) return -1;
    return orient2d_exact(a, b, c, i, j);
}

// P in the closed triangle abc, P known to lie in its plane
__device__ __noinline__ bool coplanar_in_triangle(const double *P, const double *a, const double *b,
                                                 const double *c) {
    const int pi[3] = {0, 1, 0}, pj[3] = {1, 2, 2};
    for (int k = 0; k < 3; ++k) {
        int s = orient2d(a, b, c, pi[k], pj[k]);
        if (s == 0) continue;
        int s1 = orient2d(a, b, P, pi[k], pj[k]);
        int s2 = orient2d(b, c, P, pi[k], pj[k]);
        int s3 = orient2d(c, a, P, pi[k], pj[k]);
        return s1 * s >= 0 && s2 * s >= 0 && s3 * s >= 0;
    }
    return false;
}

enum { SEG_MISS = 0, SEG_CROSS = 1, SEG_DEGEN = 2, SEG_ON = 3 };

// Segment P -> Q against triangle abc (exact).
__device__ inline int segment_triangle(const double *P, const double *Q, const double *a,
                                       const double *b, const double *c) {
    int sp = orient3d(a, b, c, P);
    if (sp == 0) return coplanar_in_triangle(P, a, b, c) ? SEG_ON : SEG_MISS;
    int sq = orient3d(a, b, c, Q);
    if (sq == 0) return SEG_DEGEN;
    if (sp == sq) return SEG_MISS;
    int e1 = orient3d(P, Q, a, b);
    int e2 = orient3d(P, Q, b, c);
    int e3 = orient3d(P, Q, c, a);
    int np = (e1 > 0) + (e2 > 0) + (e3 > 0);
    int nn = (e1 < 0) + (e2 < 0) + (e3 < 0);
    if (np == 3 || nn == 3) return SEG_CROSS;
    if (np && nn) return SEG_MISS;
    return SEG_DEGEN;
}

}  // namespace vmsd

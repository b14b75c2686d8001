// VMS element assembly of libvms (gfx950): two-stage contraction with MFMA.
//
// Residual and Jacobian of the VMS weak form, eq. (vms), with the fine
// scales u' = -tau_M r_M (eq. uprime, f = 0, the viscous part of div sigma
// dropped for trilinear fields) and p' = -rho tau_C div u (eq. pprime),
// Crank-Nicolson in theta form (u_theta = theta u + (1-theta) u_prev), tau's
// frozen at the current state.
//
// At each quadrature point q (weight W) the element matrix gains
//   K[(a,i),(b,j)] += sum_{k,l} B[k][a] (W D^{ij}[k][l]) B[l][b],
// B = [N; dN/dx; dN/dy; dN/dz] of the constrained basis (B C, C the
// hanging-node operator M_e of Alg. 3) and D^{ij} the 4x4 coefficient block
// of the linearised integrand for test component i and trial component j:
//   D^{ij}[0][0] multiplies N_a N_b,  D^{ij}[0][1+l] N_a d_l N_b,
//   D^{ij}[1+k][0] d_k N_a N_b,       D^{ij}[1+k][1+l] d_k N_a d_l N_b.
// This is the precomputed-operator form of Alg. 6 / App. A (basis values and
// gradients tabulated at Gauss points; the element matrix is a contraction
// over points), split in two stages:
//   stage 1:  F_q[(i,k)][(b,j)] = sum_l W D^{ij}[k][l] B[l][b]
//   stage 2:  K[a][(b,j,i)]     = sum_{q,k} B_q[k][a] F_q[(i,k)][(b,j)]
// Stage 2 is a GEMM over the 8 basis rows a, the contraction over (point,
// derivative) and the 128 columns (b, j, i).
//
// Precision forms. FP64 runs both stages on v_mfma_f64_4x4x4 (four 4x4
// blocks per instruction, block = trial component j): stage 1 produces, per
// (i, b half), the 4x4 blocks F^{ij}[k][b] directly in the register layout of
// stage 2's second operand, and stage 2 adds them into the four 4x4 blocks of
// each 8x8 component-pair block (no idle rows, one point per k-step).
// MIXED_BF16 splits both stage-2 operands into three bf16 terms and
// MIXED_FP16 into two fp16 terms (with power-of-two scaling), accumulating in
// FP32 with v_mfma_f32_16x16x32 (eight points per k-step; rows a in 16-row
// tiles with the second split term in rows 8-15); stage 1 and everything
// before the contraction run in FP32 on the VALU and the result is written
// as FP32.
//
// One 64-lane workgroup per element, points in chunks of 8.
#include "geom.h"
#include "kernels.h"
#include "vms_point.h"

namespace vmsk {
using namespace vmsd;


typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));


__device__ inline const double *field_in(const AsmArgs &a, int f) {
    switch (f) {
        case 0: return a.f[0];
        case 1: return a.f[1];
        case 2: return a.f[2];
        case 3: return a.f[3];
        case 4: return a.f[4];
        case 5: return a.f[5];
        default: return a.f[6];
    }
}

// reference coordinates (double) and weight of point pt of the item
template <bool SUB>
__device__ inline void point_xw(const AsmArgs &a, uint32_t en, int pt, double h, double xi[3],
                                double &w) {
    if (!SUB) {
        for (int k = 0; k < 3; ++k) xi[k] = ((pt >> k) & 1) ? VMS_XI : -VMS_XI;
        const double hh = 0.5 * h;
        w = hh * hh * hh;
        return;
    }
    const int l = (int)(en & 3u), D = a.depth;
    const uint32_t key = en >> 2;
    const int gp = (int)((key >> (3 * (D - l))) & 7u);
    const double sl = ldexp(1.0, -l);
    for (int ax = 0; ax < 3; ++ax) {
        double f = 0.0;
        for (int k = 1; k <= l; ++k)
            if ((key >> (3 * (D - k + 1) + ax)) & 1u) f += ldexp(1.0, -k);
        f = __dadd_rn(f, sl * (((gp >> ax) & 1) ? VMS_GP : VMS_GM));
        xi[ax] = __dsub_rn(2.0 * f, 1.0);
    }
    const double hs = h * ldexp(1.0, -(l + 1));
    w = hs * hs * hs;
}

// split x into three bf16 terms with x ~= h + m + l
__device__ inline void split3(float x, __bf16 &h, __bf16 &m, __bf16 &l) {
    h = (__bf16)x;
    const float r1 = x - (float)h;
    m = (__bf16)r1;
    l = (__bf16)(r1 - (float)m);
}
__device__ inline void split2h(float x, _Float16 &h, _Float16 &l) {
    h = (_Float16)x;
    l = (_Float16)(x - (float)h);
}
// the same on pairs (one packed conversion per pair)
typedef float v2f __attribute__((ext_vector_type(2)));
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
typedef _Float16 v2h __attribute__((ext_vector_type(2)));
__device__ inline void split3x2(v2f x, v2bf &h, v2bf &m, v2bf &l) {
    h = __builtin_convertvector(x, v2bf);
    const v2f r1 = x - __builtin_convertvector(h, v2f);
    m = __builtin_convertvector(r1, v2bf);
    l = __builtin_convertvector(r1 - __builtin_convertvector(m, v2f), v2bf);
}
__device__ inline void split2hx2(v2f x, v2h &h, v2h &l) {
    h = __builtin_convertvector(x, v2h);
    l = __builtin_convertvector(x - __builtin_convertvector(h, v2f), v2h);
}

// LDS of one work item. Arrays are flat with padded strides so that the
// accesses of the phases below spread over the banks (64-bit accesses by 16
// lanes and 32-bit accesses by 32 lanes touch distinct banks):
//   U(f, s)          fields at the master slots, row stride 9
//   B(p, k, s)       constrained basis rows, point stride 40
//   I(p, f, k)       interpolated fields, field stride 5, point stride 5 NF
//   D(p, i, j, k, l) coefficient blocks, block stride 17, point stride 276
// NF fields: the state (u, p, u_prev: 7), plus the direction (x_u, x_p: 4) in
// the Jacobian action.
constexpr int LU = 9, LB = 40, LDB = 17, LDP = 16 * LDB + 4;
// PD = points whose D blocks are held at once (FP64: 4, mixed: 8); no D area
// without the matrix
template <typename T, int PD, bool MAT, int NF>
struct Smem {
    static constexpr int CP = 8;
    T sU[NF * LU];
    T sC[8][8];
    T sB[CP * LB];
    T sQ[CP][NQ2];
    union {  // the interpolated fields are dead once the point quantities exist
        T sI[CP * NF * 5];
        T sD[MAT ? PD * LDP : 1];  // weight folded in
    };
    T sSc[CP];       // fp16 form: per-point bound of the contraction operands
    int sM[8];
};
#define SU(f, s) sU[(f) * LU + (s)]
#define SB(p, k, s) sB[(p) * LB + (k) * 8 + (s)]
#define SI(p, f, k) sI[(p) * (NF * 5) + (f) * 5 + (k)]
#define SD(p, i, j, k, l) sD[(p) * LDP + ((i) * 4 + (j)) * LDB + (k) * 4 + (l)]


// One work item (an element, or a run of sub-cell points of one element) by
// one 64-lane workgroup. JV: the Jacobian action along the direction xd
// (DEVICE, 4 n_nodes doubles, dof 4 node + c) instead of the residual, no
// matrix.
// Per-lane element data of one OUT work item, loaded ahead of its use: the
// element, its level and hanging flag, the master of slot lane % 8, the
// constraint weight code of (corner lane / 8, slot lane % 8) and, for lanes
// < 56, nodal field lane / 8 at that master.
struct ItemPre {
    int32_t e, m, hang, level;
    uint32_t code;
    double fv;
};

// The loads of two OUT items interleaved, so that the second item's chain
// (item -> element -> masters -> fields) is in flight while the first is
// assembled.
__device__ inline void load_pre2(const AsmArgs &a, int64_t i0, int64_t i1, bool has1, ItemPre &P0,
                                 ItemPre &P1) {
    const int lane = threadIdx.x, s = lane & 7, bit = 2 * ((lane >> 3) * 8 + s);
    P0.e = a.items[i0];
    P1.e = has1 ? a.items[i1] : P0.e;
    P0.hang = a.has_hang[P0.e];
    P1.hang = a.has_hang[P1.e];
    P0.level = a.level[P0.e];
    P1.level = a.level[P1.e];
    P0.code = (a.ccode[4 * (int64_t)P0.e + (bit >> 5)] >> (bit & 31)) & 3u;
    P1.code = (a.ccode[4 * (int64_t)P1.e + (bit >> 5)] >> (bit & 31)) & 3u;
    P0.m = a.masters[8 * (int64_t)P0.e + s];
    P1.m = a.masters[8 * (int64_t)P1.e + s];
    P0.fv = (lane < 56 && P0.m >= 0) ? field_in(a, lane >> 3)[P0.m] : 0.0;
    P1.fv = (lane < 56 && P1.m >= 0) ? field_in(a, lane >> 3)[P1.m] : 0.0;
}

template <typename T, int MODE, bool SUB, bool MAT, int PD, bool JV = false>
__device__ __forceinline__ void asm_item(const AsmArgs &a, const int64_t item,
                                         Smem<T, PD, MAT, JV ? 11 : 7> &sm,
                                         const double *xd = nullptr, const ItemPre *pre = nullptr) {
    constexpr int CP = 8;  // points per chunk (one lane group of 8 per point)
    constexpr int NF = JV ? 11 : 7;
    static_assert(!(JV && MAT), "the Jacobian action has no matrix");
    static_assert(MODE == 0 || PD == 8, "the mixed forms take 8 points per MFMA k-step");
    static_assert(PD == 4 || PD == 8, "D blocks of 4 or 8 points at a time");
    auto &sU = sm.sU;
    auto &sC = sm.sC;
    auto &sB = sm.sB;
    auto &sI = sm.sI;
    auto &sQ = sm.sQ;
    auto &sD = sm.sD;
    auto &sSc = sm.sSc;
    auto &sM = sm.sM;
    const int lane = threadIdx.x;
    __syncthreads();  // the previous item of this workgroup is done with the LDS
    const int e = pre ? pre->e : a.items[item];
    const bool hang = (pre ? pre->hang : a.has_hang[e]) != 0;
    const int lev = pre ? pre->level : (int)a.level[e];
    const double hd = ldexp(a.root_len, -lev);
    const double two_over_h = ldexp(a.two_over_root, lev);
    const T h = (T)hd;
    if (lane < 8) sM[lane] = pre ? pre->m : a.masters[8 * (int64_t)e + lane];
    {
        const int v = lane >> 3, s = lane & 7, bit = 2 * (v * 8 + s);
        const uint32_t code = pre ? pre->code : (a.ccode[4 * (int64_t)e + (bit >> 5)] >> (bit & 31)) & 3u;
        sC[v][s] = code == 3u ? T(1) : (code == 2u ? T(0.5) : (code == 1u ? T(0.25) : T(0)));
    }
    if (pre && NF == 7) {
        if (lane < 56) SU(lane >> 3, lane & 7) = (T)pre->fv;
        __syncthreads();
    } else {
        __syncthreads();
        for (int idx = lane; idx < NF * 8; idx += 64) {
            const int f = idx >> 3, s = idx & 7, m = sM[s];
            double v = 0.0;
            if (m >= 0) v = f < 7 ? field_in(a, f)[m] : xd[4 * (int64_t)m + (f - 7)];
            SU(f, s) = (T)v;
        }
    }
    const int npts = SUB ? a.pt_cnt[item] : 8;
    const T rho = (T)a.rho, mu = (T)a.mu, th = (T)a.theta;
    const T idt = (T)a.idt, irho = (T)a.irho;
    // G = (2/h)^2 I: u.G.u = gG |u|^2; tau_M^-2 = c_t/dt^2 + gG |u|^2 + c_i nu^2 G:G;
    // tau_C = 1/(tau_M tr G) = (h^2/12)/tau_M
    const double gGd = two_over_h * two_over_h;
    const T gG = (T)gGd;
    const T tau0 = (T)(a.tau_a + a.tau_b * gGd * gGd);
    const T h2_12 = (T)(hd * hd * (1.0 / 12.0));
    // fp16 form: gradient rows of the basis scaled by h/2 (all rows within
    // [-1, 1]); s16 = exponent of the product scale (accumulators carry 2^s16)
    const float hhalf = (float)(0.5 * hd), gh = (float)two_over_h;
    int s16 = INT_MAX;

    // stage-2 accumulators and residual. FP64: 4x4x4 MFMA blocks (four per
    // instruction, block = trial component j); lane l holds, for every (i, a
    // half ah, b half bh), K^{ij}[4 ah + m][4 bh + n] with m = l / 16,
    // j = (l / 4) % 4, n = l % 4. Mixed: 16x16 blocks (see phase 5).
    double acc4[4][2][2];
    v4f accf[8];
    for (int i = 0; i < 4; ++i)
        for (int h = 0; h < 4; ++h) acc4[i][h >> 1][h & 1] = 0.0;
    for (int t = 0; t < 8; ++t) accf[t] = v4f{0, 0, 0, 0};
    T R = T(0);  // lanes < 32: residual of (a = lane & 7, i = lane >> 3)
    // FP64 with the matrix: the residual is one more 4x4x4 MFMA whose blocks
    // 0 and 1 are the two halves of the rows a (columns i carry r^i[k]): lane
    // l holds R[4 ((l / 4) % 4) + l / 16][l % 4] for (l / 4) % 4 < 2
    constexpr bool RES_MFMA = MODE == 0 && MAT;
    double accr = 0.0;
    // sub-cell entry of the lane's point (lane = (p, s)), loaded one chunk ahead
    const int64_t eoff = SUB ? a.pt_off[item] : 0;
    uint32_t en_cur = (SUB && (lane >> 3) < npts) ? a.entries[eoff + (lane >> 3)] : 0u;

    for (int base = 0; base < npts; base += CP) {
        const int np = min(CP, npts - base);
        const int pn = base + CP + (lane >> 3);
        const uint32_t en_next = (SUB && pn < npts) ? a.entries[eoff + pn] : 0u;
        // ---- phase 1: constrained basis at the chunk's points (lane = (p, s))
        for (int idx = lane; idx < CP * 8; idx += 64) {
            const int p = idx >> 3, s = idx & 7;
            T b[4] = {T(0), T(0), T(0), T(0)};
            double w = 0.0;
            if (p < np) {
                double xi[3];
                point_xw<SUB>(a, en_cur, base + p, hd, xi, w);
                // vertex v of the constrained slot s: v = s without hanging
                // corners, else every v with C[v][s] != 0
                const T xt[3] = {(T)xi[0], (T)xi[1], (T)xi[2]};
                const T hg = T(0.5) * (T)two_over_h;
                const int v0 = hang ? 0 : s, v1 = hang ? 8 : s + 1;
#pragma unroll 1
                for (int v = v0; v < v1; ++v) {
                    const T c = hang ? sC[v][s] : T(1);
                    if (c == T(0)) continue;
                    T f[3], g[3];
                    for (int k = 0; k < 3; ++k) {
                        const bool up = (v >> k) & 1;
                        f[k] = T(0.5) * (up ? T(1) + xt[k] : T(1) - xt[k]);
                        g[k] = up ? hg : -hg;
                    }
                    b[0] += c * (f[0] * f[1] * f[2]);
                    b[1] += c * (g[0] * f[1] * f[2]);
                    b[2] += c * (f[0] * g[1] * f[2]);
                    b[3] += c * (f[0] * f[1] * g[2]);
                }
            }
            for (int k = 0; k < 4; ++k) SB(p, k, s) = b[k];
            if (s == 0) {
                sQ[p][QW] = (T)w;
                sSc[p] = T(0);
            }
        }
        __syncthreads();
        // ---- phase 2: interpolation of the nodal fields (lane = (p, field))
        constexpr int FL = NF > 8 ? 16 : 8;
        for (int idx = lane; idx < CP * FL; idx += 64) {
            const int p = idx / FL, f = idx % FL;
            if (p < np && f < NF) {
                T v[4] = {T(0), T(0), T(0), T(0)};
                for (int s = 0; s < 8; ++s) {
                    const T u = SU(f, s);
                    for (int k = 0; k < 4; ++k) v[k] += SB(p, k, s) * u;
                }
                for (int k = 0; k < 4; ++k) SI(p, f, k) = v[k];
            }
        }
        __syncthreads();
        // ---- phase 3: point quantities, lane = (p, r). (a) Lanes r = 0..3 of
        // point p evaluate the point state; lane r < 3 writes row / component
        // c = r of it and momentum row c of the residual coefficients r^i[k]
        // (times W), lane r = 3 the scalars and the continuity row.
        if constexpr (JV) {
            // Jacobian action: the same coefficients differentiated along the
            // direction (fields 7..10: x_u, x_p at the new step) with tau_M,
            // tau_C and taubar frozen at the state; d(u_theta) = theta x_u,
            // d(a_t) = x_u / dt, d(p) = x_p
            const int p = lane >> 3, r = lane & 7;
            if (p < np && r < 4) {
                T ut[3], gu[3][3], dut[3], dgu[3][3], dat[3];
                for (int c = 0; c < 3; ++c) {
                    ut[c] = th * SI(p, c, 0) + (T(1) - th) * SI(p, 4 + c, 0);
                    dut[c] = th * SI(p, 7 + c, 0);
                    dat[c] = SI(p, 7 + c, 0) * idt;
                    for (int m = 0; m < 3; ++m) {
                        gu[c][m] = th * SI(p, c, 1 + m) + (T(1) - th) * SI(p, 4 + c, 1 + m);
                        dgu[c][m] = th * SI(p, 7 + c, 1 + m);
                    }
                }
                T up[3], dup[3];
                for (int c = 0; c < 3; ++c) {
                    const T atc = (SI(p, c, 0) - SI(p, 4 + c, 0)) * idt;
                    const T conv = ut[0] * gu[c][0] + ut[1] * gu[c][1] + ut[2] * gu[c][2];
                    const T dconv = dut[0] * gu[c][0] + dut[1] * gu[c][1] + dut[2] * gu[c][2] +
                                    ut[0] * dgu[c][0] + ut[1] * dgu[c][1] + ut[2] * dgu[c][2];
                    up[c] = rho * (atc + conv) + SI(p, 3, 1 + c);
                    dup[c] = rho * (dat[c] + dconv) + SI(p, 10, 1 + c);
                }
                const T s0 = tau0 + gG * (ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2]);
                const T tauM = rsq<T>(s0);
                const T tauC = h2_12 * s0 * tauM;
                for (int c = 0; c < 3; ++c) {
                    up[c] *= -tauM;
                    dup[c] *= -tauM;
                }
                const T ddiv = dgu[0][0] + dgu[1][1] + dgu[2][2];
                const T dpp = -rho * tauC * ddiv;
                const T upg = gG * (up[0] * up[0] + up[1] * up[1] + up[2] * up[2]);
                const T tb = upg > T(0) ? rsq<T>(upg) : T(0);
                T *q = sQ[p];
                const T W = q[QW];
                if (r < 3) {
                    // row c = r: its lane-indexed quantities come from LDS again
                    const int c = r;
                    T guc[3], dguc[3], dgcol[3];
                    for (int m = 0; m < 3; ++m) {
                        guc[m] = th * SI(p, c, 1 + m) + (T(1) - th) * SI(p, 4 + c, 1 + m);
                        dguc[m] = th * SI(p, 7 + c, 1 + m);
                        dgcol[m] = th * SI(p, 7 + m, 1 + c);
                    }
                    const T atc = (SI(p, c, 0) - SI(p, 4 + c, 0)) * idt;
                    const T datc = SI(p, 7 + c, 0) * idt;
                    const T convc = ut[0] * guc[0] + ut[1] * guc[1] + ut[2] * guc[2];
                    const T dconvc = dut[0] * guc[0] + dut[1] * guc[1] + dut[2] * guc[2] +
                                     ut[0] * dguc[0] + ut[1] * dguc[1] + ut[2] * dguc[2];
                    const T upc = -tauM * (rho * (atc + convc) + SI(p, 3, 1 + c));
                    const T dupc = -tauM * (rho * (datc + dconvc) + SI(p, 10, 1 + c));
                    T sv = T(0), dsv = T(0);
                    for (int m = 0; m < 3; ++m) {
                        sv += up[m] * guc[m];
                        dsv += dup[m] * guc[m] + up[m] * dguc[m];
                    }
                    const T dpr = SI(p, 10, 0);
                    q[QRC + 4 * c] = W * (rho * datc + rho * dconvc + dsv);
                    for (int k = 0; k < 3; ++k)
                        q[QRC + 4 * c + 1 + k] =
                            W * (mu * (dguc[k] + dgcol[k]) - (k == c ? dpr + dpp : T(0)) -
                                 dut[k] * upc - ut[k] * dupc - (dup[k] * upc + up[k] * dupc) * irho +
                                 tb * (dup[k] * sv + up[k] * dsv));
                } else {
                    q[QRC + 12] = W * ddiv;
                    for (int k = 0; k < 3; ++k) q[QRC + 13 + k] = -W * dup[k] * irho;
                }
            }
        } else {
            const int p = lane >> 3, r = lane & 7;
            if (p < np && r < 4) {
                T ut[3], gu[3][3], up[3];
                for (int c = 0; c < 3; ++c) {
                    ut[c] = th * SI(p, c, 0) + (T(1) - th) * SI(p, 4 + c, 0);
                    for (int m = 0; m < 3; ++m)
                        gu[c][m] = th * SI(p, c, 1 + m) + (T(1) - th) * SI(p, 4 + c, 1 + m);
                }
                T rM[3];
                for (int c = 0; c < 3; ++c) {
                    const T atc = (SI(p, c, 0) - SI(p, 4 + c, 0)) * idt;
                    const T conv = ut[0] * gu[c][0] + ut[1] * gu[c][1] + ut[2] * gu[c][2];
                    rM[c] = rho * (atc + conv) + SI(p, 3, 1 + c);
                }
                const T div = gu[0][0] + gu[1][1] + gu[2][2];
                const T s0 = tau0 + gG * (ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2]);
                const T tauM = rsq<T>(s0);
                const T tauC = h2_12 * s0 * tauM;  // (h^2/12) / tau_M
                for (int c = 0; c < 3; ++c) up[c] = -tauM * rM[c];
                const T pp = -rho * tauC * div;
                const T upg = gG * (up[0] * up[0] + up[1] * up[1] + up[2] * up[2]);
                const T tb = upg > T(0) ? rsq<T>(upg) : T(0);
                T *q = sQ[p];
                const T W = q[QW];
                if (r < 3) {
                    const int c = r;
                    T guc[3], gcol[3];
                    for (int m = 0; m < 3; ++m) {
                        guc[m] = th * SI(p, c, 1 + m) + (T(1) - th) * SI(p, 4 + c, 1 + m);
                        gcol[m] = th * SI(p, m, 1 + c) + (T(1) - th) * SI(p, 4 + m, 1 + c);
                    }
                    const T utc = th * SI(p, c, 0) + (T(1) - th) * SI(p, 4 + c, 0);
                    const T atc = (SI(p, c, 0) - SI(p, 4 + c, 0)) * idt;
                    const T convc = ut[0] * guc[0] + ut[1] * guc[1] + ut[2] * guc[2];
                    const T upc = -tauM * (rho * (atc + convc) + SI(p, 3, 1 + c));
                    const T svc = up[0] * guc[0] + up[1] * guc[1] + up[2] * guc[2];
                    const T pr = SI(p, 3, 0);
                    q[QUT + c] = utc;
                    q[QUP + c] = upc;
                    q[QSV + c] = svc;
                    for (int m = 0; m < 3; ++m) q[QG + 3 * c + m] = guc[m];
                    q[QRC + 4 * c] = W * (rho * atc + rho * convc + svc);
                    for (int k = 0; k < 3; ++k)
                        q[QRC + 4 * c + 1 + k] =
                            W * (mu * (guc[k] + gcol[k]) - (k == c ? pr + pp : T(0)) - ut[k] * upc -
                                 up[k] * upc * irho + tb * up[k] * svc);
                } else {
                    q[QTM] = tauM;
                    q[QTC] = tauC;
                    q[QTB] = tb;
                    q[QRC + 12] = W * div;
                    for (int k = 0; k < 3; ++k) q[QRC + 13 + k] = -W * up[k] * irho;
                }
            }
        }
        // (b) the factors of the D blocks from the stored point state, lane
        // (p, r): r < 3 the matrix rows c = r, 3 <= r < 6 the vector
        // components c = r - 3. The round trip through LDS bounds the registers
        // the point phase holds.
        if (MAT) {
            __syncthreads();
            const int p = lane >> 3, r = lane & 7;
            if (p < np && r < 6) {
                const T *qc = sQ[p];
                T *q = sQ[p];
                const T tauM = qc[QTM], tb = qc[QTB];
                const T tr = tauM * rho, tbtr = tb * tauM * rho, tbt = tb * tauM, tir = tauM * irho;
                if (r < 3) {
                    const int c = r;
                    for (int m = 0; m < 3; ++m) {
                        q[QA + 3 * c + m] = (c == m ? idt : T(0)) + th * qc[QG + 3 * c + m];
                        T v = T(0);
                        for (int k = 0; k < 3; ++k)
                            v += qc[QG + 3 * c + k] * ((k == m ? idt : T(0)) + th * qc[QG + 3 * k + m]);
                        q[QGA + 3 * c + m] = v;
                    }
                } else {
                    const int c = r - 3;
                    const T utc = qc[QUT + c], upc = qc[QUP + c], svc = qc[QSV + c];
                    q[QY + c] = tr * utc + tauM * upc;
                    q[QX + c] = -tbtr * upc;
                    q[QCP + c] = tauM * upc - tbtr * svc;
                    q[QYM + c] = tauM * utc + tir * upc;
                    q[QCM + c] = tir * upc - tbt * svc;
                    q[QXM + c] = -tbt * upc;
                }
            }
        }
        __syncthreads();
        if (MAT) {
            // ---- phases 4 and 5 over batches of PD points
            for (int pb = 0; pb < np; pb += PD) {
            const int nd = min(PD, np - pb);
            if (pb > 0) __syncthreads();  // the previous batch is done with the D blocks
            // ---- phase 4: D blocks (one (p, i, j) block per task), weight folded in.
            // Tasks are ordered by kind so that the lanes of a pass share a code
            // path: the 9 momentum/velocity blocks of every point first, then the
            // 7 simple blocks of every point.
            for (int t = lane; t < PD * 16; t += 64) {
                int p, i, j;
                const bool mv = t < 9 * PD;
                if (mv) {
                    p = t / 9;
                    i = (t % 9) / 3;
                    j = t % 3;
                } else {
                    const int u = t - 9 * PD, r = u % 7;
                    p = u / 7;
                    i = r < 3 ? r : 3;
                    j = r < 3 ? 3 : (r < 6 ? r - 3 : 3);
                }
                T D[4][4];
                if (p >= nd) {
                    for (int k = 0; k < 4; ++k)
                        for (int l = 0; l < 4; ++l) D[k][l] = T(0);
                } else if (mv) {
                    dblock_mv<T>(sQ[pb + p], i, j, rho, mu, th, D);
                } else {
                    dblock_simple<T>(sQ[pb + p], i, j, irho, th, D);
                }
                for (int k = 0; k < 4; ++k)
                    for (int l = 0; l < 4; ++l) SD(p, i, j, k, l) = D[k][l];
                if constexpr (MODE == 2) {
                    // bound of the point's stage-1 operands: row k is sum_l D[k][l] B[l][b]
                    // with |B| <= 1 for values and <= 2/h for gradients, times 2/h
                    // for gradient rows (their basis rows carry h/2)
                    if (p < nd) {
                        float bnd = 0.f;
                        for (int k = 0; k < 4; ++k) {
                            float v = fabsf((float)D[k][0]);
                            for (int l = 1; l < 4; ++l) v += gh * fabsf((float)D[k][l]);
                            bnd = fmaxf(bnd, k > 0 ? gh * v : v);
                        }
                        atomicMax((int *)&sSc[pb + p], __float_as_int(bnd));  // non-negative floats
                    }
                }
            }
            __syncthreads();
            // ---- phase 5: stage 1 (VALU) and stage 2 (MFMA)
            const int col = lane & 15, bb = col >> 2, jc = col & 3;
            if (MODE == 0) {
                // Both stages on 4x4x4 MFMA. Lane l carries, in every operand,
                // index l / 16 of the contraction, block (l / 4) % 4 = trial
                // component j and row / column l % 4. Stage 1, per (i, b half bh):
                // E^{ij}[k][4 bh + n] = sum_l D^{ij}[k][l] B[l][4 bh + n], with A =
                // D^{ij} read transposed from LDS and B = basis columns 4 bh + n;
                // its output lands in exactly the layout of stage 2's B operand
                // (k = l / 16, j, n = l % 4). Stage 2: K^{ij}[4 ah + m][4 bh + n] +=
                // sum_k B[k][4 ah + m] E^{ij}[k][4 bh + n]. The basis values A0 / A1
                // (rows 0-3 / 4-7) serve as stage 1's B and stage 2's A alike.
                const int k = lane >> 4, j4 = (lane >> 2) & 3, n4 = lane & 3;
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    if (p >= nd) break;
                    const double A0 = (double)SB(pb + p, k, n4), A1 = (double)SB(pb + p, k, 4 + n4);
                    const double Ar = j4 == 0 ? A0 : (j4 == 1 ? A1 : 0.0);
                    const double rc = (double)sQ[pb + p][QRC + 4 * n4 + k];
                    accr = __builtin_amdgcn_mfma_f64_4x4x4f64(Ar, rc, accr, 0, 0, 0);
                    for (int i = 0; i < 4; ++i) {
                        const double Dt = (double)SD(p, i, j4, n4, k);  // D^{ij}[n4][k]
                        for (int bh = 0; bh < 2; ++bh) {
                            const double E = __builtin_amdgcn_mfma_f64_4x4x4f64(Dt, bh ? A1 : A0, 0.0, 0, 0, 0);
                            acc4[i][0][bh] = __builtin_amdgcn_mfma_f64_4x4x4f64(A0, E, acc4[i][0][bh], 0, 0, 0);
                            acc4[i][1][bh] = __builtin_amdgcn_mfma_f64_4x4x4f64(A1, E, acc4[i][1][bh], 0, 0, 0);
                        }
                    }
                }
            } else {
                // k-step of 32 = 8 points x 4 derivative rows; lane group g holds points 2g, 2g+1
                const int g = lane >> 4, row = lane & 15;
                const int ar = row & 7;
                const bool hi_rows = row < 8;
                // fp16: powers of two put the chunk's largest product near 2^12 and
                // balance it between the two operands of each point (A about 2^ea, F
                // about 2^(s16 - ea)): both split terms stay in the normal fp16 range.
                // A later chunk with larger products lowers s16 and rescales the
                // accumulators (exact).
                int ea[2] = {0, 0};
                if constexpr (MODE == 2) {
                    float bm = 0.f;
                    for (int q = 0; q < CP; ++q) bm = fmaxf(bm, (float)sSc[q]);
                    if (bm > 0.f) {
                        const int sc = 12 - ilogbf(bm);
                        if (s16 == INT_MAX) {
                            s16 = sc;
                        } else if (sc < s16) {
                            const float f = ldexpf(1.0f, sc - s16);
                            for (int t = 0; t < 8; ++t)
                                for (int r = 0; r < 4; ++r) accf[t][r] *= f;
                            s16 = sc;
                        }
                    }
                    const int sv = s16 == INT_MAX ? 0 : s16;
                    for (int pp = 0; pp < 2; ++pp) {
                        const float bp = (float)sSc[2 * g + pp];
                        ea[pp] = bp > 0.f ? ((ilogbf(bp) + sv) >> 1) : 0;
                    }
                }
                float Av[8];
                for (int t = 0; t < 8; ++t) {
                    const int p = 2 * g + (t >> 2), k = t & 3;
                    float v = (float)SB(p, k, ar);
                    if (MODE == 2) v *= ldexpf(k == 0 ? 1.0f : hhalf, ea[t >> 2]);
                    Av[t] = v;
                }
                // basis values of the lane's two points at its two columns b
                float Bc[2][2][4];
                for (int pp = 0; pp < 2; ++pp)
                    for (int bh = 0; bh < 2; ++bh)
                        for (int m = 0; m < 4; ++m) Bc[pp][bh][m] = (float)SB(2 * g + pp, m, 4 * bh + bb);
                float fs[2][4];
                for (int pp = 0; pp < 2; ++pp)
                    for (int k = 0; k < 4; ++k)
                        fs[pp][k] = MODE == 2 ? ldexpf(k == 0 ? 1.0f : gh, (s16 == INT_MAX ? 0 : s16) - ea[pp])
                                              : 1.0f;
                if (MODE == 1) {
                    v8bf Ahm, Alo;
                    for (int t = 0; t < 8; ++t) {
                        __bf16 x1, x2, x3;
                        split3(Av[t], x1, x2, x3);
                        Ahm[t] = hi_rows ? x1 : x2;
                        Alo[t] = hi_rows ? x3 : (__bf16)0.0f;
                    }
                    for (int i = 0; i < 4; ++i) {
                        v8bf F1[2], F2[2], F3[2];
                        for (int t = 0; t < 8; t += 2) {
                            const int pp = t >> 2, p = 2 * g + pp, k = t & 3;
                            float d[2][4];
                            for (int m = 0; m < 4; ++m) {
                                d[0][m] = (float)SD(p, i, jc, k, m);
                                d[1][m] = (float)SD(p, i, jc, k + 1, m);
                            }
                            for (int bh = 0; bh < 2; ++bh) {
                                v2f F;
                                for (int e = 0; e < 2; ++e)
                                    F[e] = d[e][0] * Bc[pp][bh][0] + d[e][1] * Bc[pp][bh][1] +
                                           d[e][2] * Bc[pp][bh][2] + d[e][3] * Bc[pp][bh][3];
                                v2bf x1, x2, x3;
                                split3x2(F, x1, x2, x3);
                                F1[bh][t] = x1[0]; F1[bh][t + 1] = x1[1];
                                F2[bh][t] = x2[0]; F2[bh][t + 1] = x2[1];
                                F3[bh][t] = x3[0]; F3[bh][t + 1] = x3[1];
                            }
                        }
                        for (int bh = 0; bh < 2; ++bh) {
                            v4f acc = accf[2 * i + bh];
                            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ahm, F1[bh], acc, 0, 0, 0);
                            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ahm, F2[bh], acc, 0, 0, 0);
                            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ahm, F3[bh], acc, 0, 0, 0);
                            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Alo, F1[bh], acc, 0, 0, 0);
                            accf[2 * i + bh] = acc;
                        }
                    }
                } else {
                    v8h Ahm;
                    for (int t = 0; t < 8; ++t) {
                        _Float16 x1, x2;
                        split2h(Av[t], x1, x2);
                        Ahm[t] = hi_rows ? x1 : x2;
                    }
                    for (int i = 0; i < 4; ++i) {
                        v8h F1[2], F2[2];
                        for (int t = 0; t < 8; t += 2) {
                            const int pp = t >> 2, p = 2 * g + pp, k = t & 3;
                            float d[2][4];
                            for (int m = 0; m < 4; ++m) {
                                d[0][m] = (float)SD(p, i, jc, k, m);
                                d[1][m] = (float)SD(p, i, jc, k + 1, m);
                            }
                            for (int bh = 0; bh < 2; ++bh) {
                                // undo the basis scaling and the balance on this operand
                                v2f F;
                                for (int e = 0; e < 2; ++e)
                                    F[e] = (d[e][0] * Bc[pp][bh][0] + d[e][1] * Bc[pp][bh][1] +
                                            d[e][2] * Bc[pp][bh][2] + d[e][3] * Bc[pp][bh][3]) * fs[pp][k + e];
                                v2h x1, x2;
                                split2hx2(F, x1, x2);
                                F1[bh][t] = x1[0]; F1[bh][t + 1] = x1[1];
                                F2[bh][t] = x2[0]; F2[bh][t + 1] = x2[1];
                            }
                        }
                        for (int bh = 0; bh < 2; ++bh) {
                            v4f acc = accf[2 * i + bh];
                            acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(Ahm, F1[bh], acc, 0, 0, 0);
                            acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(Ahm, F2[bh], acc, 0, 0, 0);
                            accf[2 * i + bh] = acc;
                        }
                    }
                }
            }
            }  // batches of PD points
        }
        // residual: lanes < 32, (a = lane & 7, i = lane >> 3)
        if (!RES_MFMA && lane < 32) {
            const int av = lane & 7, i = lane >> 3;
            for (int p = 0; p < np; ++p)
                R += SB(p, 0, av) * sQ[p][QRC + 4 * i] + SB(p, 1, av) * sQ[p][QRC + 4 * i + 1] +
                     SB(p, 2, av) * sQ[p][QRC + 4 * i + 2] + SB(p, 3, av) * sQ[p][QRC + 4 * i + 3];
        }
        en_cur = en_next;
        __syncthreads();
    }

    // ---- element matrix out: one 1024-entry record per work item, block-major
    // (block (a, b) of master slots, entry 4 i + j), stored from the
    // accumulators; the CSR is summed from these records by the gather kernel
    // (no atomics, fixed summation order)
    if (MAT && a.vals) {
        // atomic scatter: no record; each entry is added into its CSR place
        // (the summation order is the hardware's)
        T *vals = (T *)a.vals;
        const int32_t *mst = a.masters + 8 * (int64_t)e;
        const uint16_t *kk = a.el_kk + 64 * (int64_t)e;
        if (MODE == 0) {
            const int m4 = lane >> 4, j4 = (lane >> 2) & 3, n4 = lane & 3;
            for (int ah = 0; ah < 2; ++ah) {
                const int av = 4 * ah + m4, ma = mst[av];
                if (ma < 0) continue;
                const int64_t r0 = a.nrow_ptr[ma], deg = a.nrow_ptr[ma + 1] - r0;
                for (int bh = 0; bh < 2; ++bh) {
                    const int b = 4 * bh + n4;
                    if (mst[b] < 0) continue;
                    T *dst = vals + 16 * r0 + 4 * (int64_t)kk[8 * av + b] + j4;
                    for (int i = 0; i < 4; ++i) atomicAdd(dst + 4 * i * deg, (T)acc4[i][ah][bh]);
                }
            }
        } else {
            const int col = lane & 15, bb = col >> 2, jc = col & 3;
            const float unscale = (MODE == 2 && s16 != INT_MAX) ? ldexpf(1.0f, -s16) : 1.0f;
            // rows av = 4 (lane / 16) + r of the lanes < 32, columns b = 4 h + bb
            int64_t rb[4], dg[4];
            bool ok[4];
            for (int r = 0; r < 4; ++r) {
                const int ma = mst[(4 * (lane >> 4) + r) & 7];
                ok[r] = ma >= 0;
                rb[r] = ok[r] ? a.nrow_ptr[ma] : 0;
                dg[r] = ok[r] ? a.nrow_ptr[ma + 1] - rb[r] : 0;
            }
            for (int t = 0; t < 8; ++t) {
                v4f v = accf[t];
                for (int r = 0; r < 4; ++r) v[r] = (v[r] + __shfl_down(v[r], 32, 64)) * unscale;
                const int i = t >> 1, b = 4 * (t & 1) + bb;
                if (lane < 32 && mst[b] >= 0) {
                    for (int r = 0; r < 4; ++r) {
                        const int av = 4 * (lane >> 4) + r;
                        if (ok[r])
                            atomicAdd(vals + 16 * rb[r] + 4 * (int64_t)kk[8 * av + b] + 4 * i * dg[r] + jc,
                                      (T)v[r]);
                    }
                }
            }
        }
    } else if (MAT) {
        const int col = lane & 15, bb = col >> 2, jc = col & 3;
        T *dst = (T *)a.em + (a.slot0 + item) * 1024;
        if (MODE == 0) {
            const int m4 = lane >> 4, j4 = (lane >> 2) & 3, n4 = lane & 3;
            for (int i = 0; i < 4; ++i)
                for (int ah = 0; ah < 2; ++ah)
                    for (int bh = 0; bh < 2; ++bh)
                        dst[((4 * ah + m4) * 8 + 4 * bh + n4) * 16 + 4 * i + j4] = (T)acc4[i][ah][bh];
        } else {
            // rows 8..15 carry the second split term: fold them onto rows 0..7
            const float unscale = (MODE == 2 && s16 != INT_MAX) ? ldexpf(1.0f, -s16) : 1.0f;
            for (int t = 0; t < 8; ++t) {
                v4f v = accf[t];
                for (int r = 0; r < 4; ++r) v[r] = (v[r] + __shfl_down(v[r], 32, 64)) * unscale;
                if (lane < 32) {
                    const int i = t >> 1, b = 4 * (t & 1) + bb;
                    for (int r = 0; r < 4; ++r) {
                        const int av = 4 * (lane >> 4) + r;  // output row = 4 (lane / 16) + r
                        dst[(av * 8 + b) * 16 + 4 * i + jc] = (T)v[r];
                    }
                }
            }
        }
    }
    // residual record of the work item (entry 4 a + i); the residual is summed
    // from the records by node, in a fixed order
    if (RES_MFMA) {
        const int blk = (lane >> 2) & 3;
        if (blk < 2 && a.rrec) {
            const int av = 4 * blk + (lane >> 4), i = lane & 3;
            a.rrec[(a.slot0 + item) * 32 + 4 * av + i] = accr;
        }
    } else if (lane < 32 && a.rrec) {
        const int av = lane & 7, i = lane >> 3;
        a.rrec[(a.slot0 + item) * 32 + 4 * av + i] = (double)R;
    }
}

// waves per SIMD the register allocation aims for: the LDS of one item
// allows 8 (FP64) or 11 (mixed) one-wave workgroups per CU (4 SIMDs)
#ifndef VMS_WPE64
#define VMS_WPE64 2
#endif
#ifndef VMS_WPEMX
#define VMS_WPEMX 3
#endif
#define VMS_ASM_BOUNDS(MODE) \
    __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu((MODE) == 0 ? VMS_WPE64 : VMS_WPEMX, 8)))

// OUT elements (SUB = false) two per workgroup: the second element's data
// and fields load while the first is assembled
template <typename T, int MODE, bool SUB, bool MAT>
__global__ VMS_ASM_BOUNDS(MODE) void k_asm2(AsmArgs a) {
    __shared__ Smem<T, MODE == 0 ? 4 : 8, MAT, 7> sm;
    if constexpr (SUB) {
        asm_item<T, MODE, SUB, MAT, MODE == 0 ? 4 : 8>(a, blockIdx.x, sm);
    } else {
        const int64_t i0 = 2 * (int64_t)blockIdx.x, i1 = i0 + 1;
        const bool has1 = i1 < a.n_items;
        ItemPre P0, P1;
        load_pre2(a, i0, i1, has1, P0, P1);
        asm_item<T, MODE, SUB, MAT, MODE == 0 ? 4 : 8>(a, i0, sm, nullptr, &P0);
        if (has1) asm_item<T, MODE, SUB, MAT, MODE == 0 ? 4 : 8>(a, i1, sm, nullptr, &P1);
    }
}

// Jacobian action y = J x along x (the residual output of a receives y)
template <typename T, bool SUB>
__global__ VMS_ASM_BOUNDS(1) void k_asm2_jv(AsmArgs a, const double *x) {
    constexpr int MODE = sizeof(T) == 8 ? 0 : 1;
    __shared__ Smem<T, MODE == 0 ? 4 : 8, false, 11> sm;
    asm_item<T, MODE, SUB, false, MODE == 0 ? 4 : 8, true>(a, blockIdx.x, sm, x);
}

// Persistent form over many contexts: every workgroup takes units of work
// from a device counter until none is left, in the order of the unit list
// (heaviest first); a unit is a run of OUT elements or of sub-cell work items
// of one tree. One launch for all units.
template <typename T, int MODE>
__global__ VMS_ASM_BOUNDS(MODE) void k_asm_batch(const AsmArgs *std_args, const AsmArgs *sub_args,
                                                 const BatchUnit *units, int64_t n_units,
                                                 unsigned long long *counter) {
    constexpr int PTS = MODE == 0 ? 4 : 8;
    __shared__ Smem<T, PTS, true, 7> sm;
    __shared__ int64_t su;
    __shared__ AsmArgs sa;  // the unit's tree, read from LDS where used
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) su = (int64_t)atomicAdd(counter, 1ull);
        __syncthreads();
        const int64_t u = su;
        if (u >= n_units) break;
        const BatchUnit U = units[u];
        if (threadIdx.x == 0) sa = U.sub ? sub_args[U.tree] : std_args[U.tree];
        __syncthreads();
        if (U.sub) {
            for (int k = 0; k < U.count; ++k) asm_item<T, MODE, true, true, PTS>(sa, U.first + k, sm);
        } else {
            for (int k = 0; k < U.count; ++k) asm_item<T, MODE, false, true, PTS>(sa, U.first + k, sm);
        }
    }
}

__global__ void k_reset_counter(unsigned long long *c) {
    if (threadIdx.x < 2 && blockIdx.x == 0) c[threadIdx.x] = 0ull;
}

void launch_assemble_batch(hipStream_t s, int precision, const AsmArgs *std_args,
                           const AsmArgs *sub_args, const BatchUnit *units, int64_t n_units,
                           unsigned long long *counter, int n_groups) {
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, s, counter);
    if (n_units <= 0) return;
    dim3 grid((unsigned)n_groups), block(64);
    if (precision == 0)
        hipLaunchKernelGGL((k_asm_batch<double, 0>), grid, block, 0, s, std_args, sub_args, units, n_units,
                           counter);
    else if (precision == 1)
        hipLaunchKernelGGL((k_asm_batch<float, 1>), grid, block, 0, s, std_args, sub_args, units, n_units,
                           counter);
    else
        hipLaunchKernelGGL((k_asm_batch<float, 2>), grid, block, 0, s, std_args, sub_args, units, n_units,
                           counter);
}

// CSR values from the element-matrix records. A thread takes V consecutive
// entries of one row of a CSR block B (entries e0 .. e0+V-1, e = 4 i + j) and
// sums them over B's contributions in list order (ascending record), fetching
// the record entries V at a time and four contributions at a time; the CSR
// place of entry (i, j) is vbase[B] + i |vstride[B]| + j. A negative stride
// marks the diagonal block of an inactive node: it has no records and becomes
// an identity block. A positive stride may carry the VS_LATE flag (the block
// has records of sub-cell or surface items); SKIP_LATE leaves such blocks out.
template <typename T, int V, bool SKIP_LATE = false>
__device__ inline void gather_block(const T *em, const int64_t *cb_off, const int32_t *contrib,
                                    const int64_t *vbase, const int32_t *vstride, int64_t B, int e0,
                                    T *vals) {
    typedef T vec __attribute__((ext_vector_type(V)));
    const int st = vstride[B];
    if (SKIP_LATE && st > 0 && (st & VS_LATE)) return;
    const int64_t c0 = cb_off[B], c1 = cb_off[B + 1];
    const int64_t base = vbase[B];
    const int stride = st < 0 ? -st : (st & (VS_LATE - 1));
    double s[V];
    for (int q = 0; q < V; ++q) s[q] = (st < 0 && ((e0 + q) >> 2) == ((e0 + q) & 3)) ? 1.0 : 0.0;
    for (int64_t c = c0; c < c1; c += 4) {
        int32_t r[4];
        for (int u = 0; u < 4; ++u) r[u] = c + u < c1 ? contrib[c + u] : -1;
        vec v[4];
        for (int u = 0; u < 4; ++u)
            if (r[u] >= 0) v[u] = *(const vec *)(em + (int64_t)r[u] * 16 + e0);
        for (int u = 0; u < 4; ++u)
            if (r[u] >= 0)
                for (int q = 0; q < V; ++q) s[q] += (double)v[u][q];
    }
    // the CSR values are written once and not read again by this step:
    // streaming (non-temporal) stores keep them from displacing the records
    // in the caches (FP64 gather of the 10^7-octant workload 23.2 -> 20.8 ms)
    T *dst = vals + base + (int64_t)(e0 >> 2) * stride + (e0 & 3);
    vec o;
    for (int q = 0; q < V; ++q) o[q] = (T)s[q];
    __builtin_nontemporal_store(o, (vec *)dst);
}

template <typename T, int V, bool SKIP_LATE>
__global__ void k_gather(const T *em, const int64_t *cb_off, const int32_t *contrib,
                         const int64_t *vbase, const int32_t *vstride, int64_t nb, T *vals) {
    constexpr int TPB = 16 / V;  // threads per block
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t B = g / TPB;
    if (B >= nb) return;
    gather_block<T, V, SKIP_LATE>(em, cb_off, contrib, vbase, vstride, B, (int)(g % TPB) * V, vals);
}

// the listed blocks only (the late blocks, after the sub-cell and surface records)
template <typename T, int V>
__global__ void k_gather_list(const T *em, const int64_t *cb_off, const int32_t *contrib,
                              const int64_t *vbase, const int32_t *vstride, const int64_t *list, int64_t n,
                              T *vals) {
    constexpr int TPB = 16 / V;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t k = g / TPB;
    if (k >= n) return;
    gather_block<T, V>(em, cb_off, contrib, vbase, vstride, list[k], (int)(g % TPB) * V, vals);
}

// The same summations for every tree of a batch in one launch: the blocks of
// all trees one after the other (prefix[t] = first block of tree t), then the
// nodes of all trees for the residual (node_prefix).
__device__ inline int tree_of(const int64_t *prefix, int n, int64_t g) {
    int lo = 0, hi = n;  // prefix[lo] <= g < prefix[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= g) lo = mid;
        else hi = mid;
    }
    return lo;
}

template <typename T, int V>
__global__ void k_gather_batch(const GatherTab *tabs, const int64_t *prefix, int n_trees) {
    constexpr int TPB = 16 / V;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t Bg = g / TPB;
    if (Bg >= prefix[n_trees]) return;
    const int t = tree_of(prefix, n_trees, Bg);
    const GatherTab &G = tabs[t];
    gather_block<T, V>((const T *)G.em, G.cb_off, G.contrib, G.vbase, G.vstride, Bg - prefix[t],
                       (int)(g % TPB) * V, (T *)G.vals);
}

// residual by node from the residual records (one thread per node, its
// entries in ascending record order)
__device__ inline void res_node(const double *rrec, const int64_t *roff, const int32_t *rlist, int64_t n,
                                double *out) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int64_t c = roff[n]; c < roff[n + 1]; ++c) {
        const int64_t q = rlist[c];
        const v4d v = *(const v4d *)(rrec + (q >> 3) * 32 + 4 * (q & 7));
        s0 += v[0];
        s1 += v[1];
        s2 += v[2];
        s3 += v[3];
    }
    out[4 * n] = s0;
    out[4 * n + 1] = s1;
    out[4 * n + 2] = s2;
    out[4 * n + 3] = s3;
}

__global__ void k_res_gather(const double *rrec, const int64_t *roff, const int32_t *rlist, int64_t n_nodes,
                             double *out) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= n_nodes) return;
    res_node(rrec, roff, rlist, n, out);
}

__global__ void k_res_gather_batch(const GatherTab *tabs, const int64_t *prefix, int n_trees) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= prefix[n_trees]) return;
    const int t = tree_of(prefix, n_trees, g);
    const GatherTab &G = tabs[t];
    if (G.resid) res_node(G.rrec, G.roff, G.rlist, g - prefix[t], G.resid);
}

void launch_gather_batch(hipStream_t s, int precision, const GatherTab *tabs, const int64_t *blk_prefix,
                         int64_t n_blocks, const int64_t *node_prefix, int64_t n_nodes, int n_trees) {
    if (n_blocks > 0) {
        if (precision == 0)
            hipLaunchKernelGGL((k_gather_batch<double, 2>), dim3((unsigned)((8 * n_blocks + 255) / 256)),
                               dim3(256), 0, s, tabs, blk_prefix, n_trees);
        else
            hipLaunchKernelGGL((k_gather_batch<float, 4>), dim3((unsigned)((4 * n_blocks + 255) / 256)),
                               dim3(256), 0, s, tabs, blk_prefix, n_trees);
    }
    if (n_nodes > 0)
        hipLaunchKernelGGL(k_res_gather_batch, dim3((unsigned)((n_nodes + 255) / 256)), dim3(256), 0, s, tabs,
                           node_prefix, n_trees);
}

void launch_res_gather(hipStream_t s, const double *rrec, const int64_t *roff, const int32_t *rlist,
                       int64_t n_nodes, double *out) {
    if (n_nodes <= 0) return;
    hipLaunchKernelGGL(k_res_gather, dim3((unsigned)((n_nodes + 255) / 256)), dim3(256), 0, s, rrec, roff,
                       rlist, n_nodes, out);
}

void launch_gather_f64(hipStream_t s, const double *em, const int64_t *cb_off, const int32_t *contrib,
                       const int64_t *vbase, const int32_t *vstride, int64_t nb, double *vals,
                       bool skip_late) {
    if (nb <= 0) return;
    const dim3 grid((unsigned)((8 * nb + 255) / 256));
    if (skip_late)
        hipLaunchKernelGGL((k_gather<double, 2, true>), grid, dim3(256), 0, s, em, cb_off, contrib, vbase,
                           vstride, nb, vals);
    else
        hipLaunchKernelGGL((k_gather<double, 2, false>), grid, dim3(256), 0, s, em, cb_off, contrib, vbase,
                           vstride, nb, vals);
}
void launch_gather_f32(hipStream_t s, const float *em, const int64_t *cb_off, const int32_t *contrib,
                       const int64_t *vbase, const int32_t *vstride, int64_t nb, float *vals,
                       bool skip_late) {
    if (nb <= 0) return;
    const dim3 grid((unsigned)((4 * nb + 255) / 256));
    if (skip_late)
        hipLaunchKernelGGL((k_gather<float, 4, true>), grid, dim3(256), 0, s, em, cb_off, contrib, vbase,
                           vstride, nb, vals);
    else
        hipLaunchKernelGGL((k_gather<float, 4, false>), grid, dim3(256), 0, s, em, cb_off, contrib, vbase,
                           vstride, nb, vals);
}
void launch_gather_list(hipStream_t s, bool fp64, const void *em, const int64_t *cb_off, const int32_t *contrib,
                        const int64_t *vbase, const int32_t *vstride, const int64_t *list, int64_t n,
                        void *vals) {
    if (n <= 0) return;
    if (fp64)
        hipLaunchKernelGGL((k_gather_list<double, 2>), dim3((unsigned)((8 * n + 255) / 256)), dim3(256), 0, s,
                           (const double *)em, cb_off, contrib, vbase, vstride, list, n, (double *)vals);
    else
        hipLaunchKernelGGL((k_gather_list<float, 4>), dim3((unsigned)((4 * n + 255) / 256)), dim3(256), 0, s,
                           (const float *)em, cb_off, contrib, vbase, vstride, list, n, (float *)vals);
}

// dynamic LDS that holds a kernel to at most wg_per_cu resident workgroups per
// CU (160 KB of LDS each; 512 bytes of slack so that the rounding of the
// allocation cannot cut one more)
size_t lds_for_cap(const void *kernel, int wg_per_cu) {
    if (wg_per_cu <= 0) return 0;
    hipFuncAttributes at{};
    if (hipFuncGetAttributes(&at, kernel) != hipSuccess) return 0;
    const size_t want = (size_t)163840 / (size_t)wg_per_cu - 512;
    return want > at.sharedSizeBytes ? want - at.sharedSizeBytes : 0;
}

int sub_items_per_cu(int precision) {
    const void *k = precision == 0 ? (const void *)&k_asm2<double, 0, true, true>
                    : precision == 1 ? (const void *)&k_asm2<float, 1, true, true>
                                     : (const void *)&k_asm2<float, 2, true, true>;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, 64, 0) != hipSuccess) return 0;
    return n;
}

void launch_assemble_f64(hipStream_t s, const AsmArgs &a, bool sub, bool mat, int wg_per_cu) {
    if (a.n_items <= 0) return;
    dim3 grid((unsigned)(sub ? a.n_items : (a.n_items + 1) / 2)), block(64);
    if (!sub) {
        if (mat) hipLaunchKernelGGL((k_asm2<double, 0, false, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_asm2<double, 0, false, false>), grid, block, 0, s, a);
    } else {
        if (mat) {
            const size_t dyn = lds_for_cap((const void *)&k_asm2<double, 0, true, true>, wg_per_cu);
            hipLaunchKernelGGL((k_asm2<double, 0, true, true>), grid, block, dyn, s, a);
        } else {
            hipLaunchKernelGGL((k_asm2<double, 0, true, false>), grid, block, 0, s, a);
        }
    }
}

void launch_assemble_mixed(hipStream_t s, const AsmArgs &a, bool sub, bool mat, int fp16, int wg_per_cu) {
    if (a.n_items <= 0) return;
    dim3 grid((unsigned)(sub ? a.n_items : (a.n_items + 1) / 2)), block(64);
#define VMS_L(MODE)                                                                              \
    do {                                                                                         \
        if (!sub) {                                                                              \
            if (mat) hipLaunchKernelGGL((k_asm2<float, MODE, false, true>), grid, block, 0, s, a); \
            else hipLaunchKernelGGL((k_asm2<float, MODE, false, false>), grid, block, 0, s, a);    \
        } else {                                                                                 \
            if (mat) hipLaunchKernelGGL((k_asm2<float, MODE, true, true>), grid, block,            \
                                        lds_for_cap((const void *)&k_asm2<float, MODE, true, true>, \
                                                    wg_per_cu), s, a);                             \
            else hipLaunchKernelGGL((k_asm2<float, MODE, true, false>), grid, block, 0, s, a);     \
        }                                                                                        \
    } while (0)
    if (fp16) VMS_L(2);
    else VMS_L(1);
#undef VMS_L
}

void launch_jacobian_action(hipStream_t s, const AsmArgs &a, bool sub, bool fp64, const double *x) {
    if (a.n_items <= 0) return;
    dim3 grid((unsigned)a.n_items), block(64);
    if (fp64) {
        if (sub) hipLaunchKernelGGL((k_asm2_jv<double, true>), grid, block, 0, s, a, x);
        else hipLaunchKernelGGL((k_asm2_jv<double, false>), grid, block, 0, s, a, x);
    } else {
        if (sub) hipLaunchKernelGGL((k_asm2_jv<float, true>), grid, block, 0, s, a, x);
        else hipLaunchKernelGGL((k_asm2_jv<float, false>), grid, block, 0, s, a, x);
    }
}

}  // namespace vmsk

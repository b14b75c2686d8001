// Per-point factors and D blocks of the VMS integrand (internal header of
// libvms, gfx950), shared by the trilinear and the triquadratic element
// kernels. At a quadrature point of weight W the element matrix gains
//   K[(a,i),(b,j)] += sum_{k,l} B[k][a] (W D^{ij}[k][l]) B[l][b],
// B = [N; dN/dx; dN/dy; dN/dz], and the residual gains
//   R[(a,i)] += sum_k B[k][a] r^i[k];
// the per-point factors below make every D entry and every r^i[k] a short sum.
#pragma once
#include <hip/hip_runtime.h>

namespace vmsk {

// per-point quantities in LDS: stabilisation parameters, interpolated state and
// the factors that make every D entry a short sum (see dblock)
enum {
    QW = 0, QTM, QTC, QTB,
    QUT = 4, QUP = 7, QA = 10, QG = 19, QGA = 28,  // u_theta, u', A = I/dt + theta grad u, grad u, grad u A
    QY = 37, QX = 40, QCP = 43, QYM = 46, QCM = 49, QXM = 52,
    QRC = 55,  // 16 residual coefficients r^i[k] (weight folded in)
    QSV = 71,  // s = (u'.grad) u
    NQ2 = 74
};

template <typename T> __device__ inline T rsq(T x);
template <> __device__ inline double rsq<double>(double x) { return rsqrt(x); }
template <> __device__ inline float rsq<float>(float x) { return __frsqrt_rn(x); }

// D^{ij} (4x4) at one point, times W, from the per-point factors:
//   momentum/velocity: D00 = rho A_ij - tau rho (grad u A)_ij
//     D0l = d_ij theta(rho u_l + u'_l) - theta tau rho g_ij u_l
//     Dk0 = A_ij Y_k + A_kj c_i - theta d_kj u'_i + (grad u A)_ij X_k
//     Dkl = al_k u_l + be_k u'_l + mu theta (d_ij d_kl + d_kj d_il) + rho tau_C theta d_ki d_lj
//       al_k = theta (d_ij (tau rho u_k + tau u'_k) + d_kj c_i - taubar tau rho g_ij u'_k)
//       be_k = theta d_ij taubar u'_k
//   with Y = tau(rho u + u'), X = -taubar tau rho u', c = tau u' - taubar tau rho s,
//   s = (u'.grad) u (the al/be form collects the products theta(tau rho u_k u_l +
//   tau u'_k u_l + taubar u'_k u'_l) of d_ij and -taubar tau rho theta u'_k u_l of g_ij);
//   momentum/pressure: D0l = -tau g_il, Dk0 = -d_ki,
//     Dkl = d_li Ym_k + d_kl cm_i + Xm_k g_il, Ym = tau u + tau/rho u',
//     cm = tau/rho u' - taubar tau s, Xm = -taubar tau u';
//   continuity/velocity: D0l = theta d_lj, Dk0 = tau A_kj, Dkl = tau theta d_kj u_l;
//   continuity/pressure: Dkl = tau/rho d_kl.
// Momentum test / velocity trial blocks (i, j < 3); the other kinds are in
// dblock_simple. Branch-free: every per-point factor is read unconditionally and
// the Kronecker terms enter through 0/1 vectors.
template <typename T>
__device__ inline void dblock_mv(const T *Q, int i, int j, T rho, T mu, T th, T D[4][4]) {
    const T W = Q[QW], tauM = Q[QTM], tb = Q[QTB], tC = Q[QTC];
    T u[3], up[3], Y[3], X[3], Acol[3], ei[3], ej[3];
    for (int l = 0; l < 3; ++l) {
        u[l] = Q[QUT + l];
        up[l] = Q[QUP + l];
        Y[l] = Q[QY + l];
        X[l] = Q[QX + l];
        Acol[l] = Q[QA + 3 * l + j];
        ei[l] = l == i ? T(1) : T(0);
        ej[l] = l == j ? T(1) : T(0);
    }
    const T Aij = Q[QA + 3 * i + j], gij = Q[QG + 3 * i + j], GAij = Q[QGA + 3 * i + j];
    const T cpi = Q[QCP + i], upi = Q[QUP + i];
    const T tr = tauM * rho;
    const T dth = (i == j) ? th * W : T(0);  // weight folded into every coefficient below
    const T thw = th * W;
    D[0][0] = W * (rho * Aij - tr * GAij);
    const T a0 = dth * rho - thw * tr * gij;
    for (int l = 0; l < 3; ++l) D[0][1 + l] = a0 * u[l] + dth * up[l];
    const T c1 = dth * tr, c2 = dth * tauM, c3 = -thw * tb * tr * gij, c4 = dth * tb;
    const T AW = Aij * W, GW = GAij * W, cW = cpi * W;
    const T mthw = mu * thw, rtcw = rho * tC * thw;
    const T dm = (i == j) ? mthw : T(0);
    for (int k = 0; k < 3; ++k) {
        const T kj = ej[k], ki = ei[k];
        D[1 + k][0] = AW * Y[k] + cW * Acol[k] + GW * X[k] - kj * (thw * upi);
        const T al = c1 * u[k] + (c2 + c3) * up[k] + kj * (thw * cpi);
        const T be = c4 * up[k];
        const T s1 = kj * mthw, s2 = ki * rtcw;
        for (int l = 0; l < 3; ++l) {
            T v = al * u[l] + be * up[l] + s1 * ei[l] + s2 * ej[l];
            if (k == l) v += dm;
            D[1 + k][1 + l] = v;
        }
    }
}

// D blocks of the three simple kinds in one code path (weight folded in):
// momentum test / pressure trial (i < 3, j = 3), continuity test / velocity
// trial (i = 3, j < 3) and continuity / pressure (i = j = 3); the kind weights
// are zero for the terms of the other kinds.
template <typename T>
__device__ inline void dblock_simple(const T *Q, int i, int j, T irho, T th, T D[4][4]) {
    const T W = Q[QW], tauM = Q[QTM];
    const bool mp = i < 3 && j == 3, cv = i == 3 && j < 3;
    const T wmp = mp ? W : T(0), wcv = cv ? W : T(0), wcc = (!mp && !cv) ? W : T(0);
    const int ii = i < 3 ? i : 0, jj = j < 3 ? j : 0;
    T g[3], Acol[3], ym[3], xm[3], u[3], ei[3], ej[3];
    for (int l = 0; l < 3; ++l) {
        g[l] = Q[QG + 3 * ii + l];
        Acol[l] = Q[QA + 3 * l + jj];
        ym[l] = Q[QYM + l];
        xm[l] = Q[QXM + l];
        u[l] = Q[QUT + l];
        ei[l] = l == i ? T(1) : T(0);  // zero for i = 3
        ej[l] = l == j ? T(1) : T(0);  // zero for j = 3
    }
    const T cmi = Q[QCM + ii];
    const T tw = wcv * tauM, tthw = tw * th, mtau = -wmp * tauM, thw = wcv * th;
    const T diag = wmp * cmi + wcc * tauM * irho;
    D[0][0] = T(0);
    for (int l = 0; l < 3; ++l) D[0][1 + l] = mtau * g[l] + thw * ej[l];
    for (int k = 0; k < 3; ++k) {
        D[1 + k][0] = tw * Acol[k] - wmp * ei[k];
        const T xk = wmp * xm[k], yk = wmp * ym[k], sk = tthw * ej[k];
        for (int l = 0; l < 3; ++l) {
            T v = xk * g[l] + sk * u[l] + yk * ei[l];
            if (k == l) v += diag;
            D[1 + k][1 + l] = v;
        }
    }
}

}  // namespace vmsk

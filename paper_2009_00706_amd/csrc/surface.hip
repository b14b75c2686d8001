// Weak (Nitsche) boundary terms of eq. (weakbc) on the surface Gauss points of
// libvms (gfx950). One 64-lane workgroup per item (an element and its surface
// points); lane (a, b) accumulates the 4x4 block of master slots a, b of the
// element matrix, lanes < 32 the residual of (a = lane & 7, i = lane >> 3).
//
// At a surface point (weight W, unit normal n of the fluid domain, v = u_theta
// - g, inflow indicator chi = [u_theta . n < 0] frozen, tau = tau_B), for the
// test functions w = N_a e_i and q = N_a:
//   momentum  W [N_a (p n_i - mu (d_k u_i + d_i u_k) n_k) - mu (v_i dN_a/dn
//              + n_i grad N_a . v) - chi rho (u . n) v_i N_a
//              + N_a (tau_T (v_i - n_i v.n) + tau_N n_i v.n)]
//   continuity -W N_a v.n
// and the Jacobian with respect to the new step (u_theta = theta u + ...,
// p at the new step), tau_B and chi frozen:
//   K[(a,i),(b,j)] = W [-mu theta N_a (d_ij dN_b/dn + d_i N_b n_j)
//                       - mu theta (d_ij N_b dN_a/dn + n_i d_j N_a N_b)
//                       - chi rho theta N_a N_b (n_j v_i + (u.n) d_ij)
//                       + theta N_a N_b (tau_T (d_ij - n_i n_j) + tau_N n_i n_j)]  (i, j < 3)
//   K[(a,i),(b,p)] = W N_a N_b n_i,   K[(a,p),(b,j)] = -W theta N_a N_b n_j.
// The work is small (a few points per cut element), all in FP64.
#include "kernels.h"

namespace vmsk {

template <typename TR, int MODE>
__global__ __launch_bounds__(64) void k_surface(SurfArgs a, const double *x) {
    constexpr bool MAT = MODE == 0, JV = MODE == 2;
    __shared__ int sM[8];
    __shared__ double sC[8][8];
    __shared__ double sU[11][8];
    __shared__ double sB[4][8];
    const int lane = threadIdx.x;
    const int64_t k = blockIdx.x;
    const int e = a.items[k];
    const bool hang = a.has_hang[e] != 0;
    const double hd = ldexp(a.root_len, -(int)a.level[e]);
    const double hg = 1.0 / hd;  // derivative of (1 +- xi)/2 with respect to x
    if (lane < 8) sM[lane] = a.masters[8 * (int64_t)e + lane];
    {
        const int v = lane >> 3, s = lane & 7, bit = 2 * (v * 8 + s);
        const uint32_t code = (a.ccode[4 * (int64_t)e + (bit >> 5)] >> (bit & 31)) & 3u;
        sC[v][s] = code == 3u ? 1.0 : (code == 2u ? 0.5 : (code == 1u ? 0.25 : 0.0));
    }
    __syncthreads();
    constexpr int NF = JV ? 11 : 7;
    for (int idx = lane; idx < NF * 8; idx += 64) {
        const int f = idx >> 3, s = idx & 7, m = sM[s];
        double v = 0.0;
        if (m >= 0) v = f < 7 ? a.f[f][m] : x[4 * (int64_t)m + (f - 7)];
        sU[f][s] = v;
    }
    const double rho = a.rho, mu = a.mu, th = a.theta;
    const int aa = lane >> 3, bb = lane & 7;         // block (a, b)
    const int ra = lane & 7, ri = lane >> 3;         // residual (a, i), lanes < 32
    double acc[16];
    for (int t = 0; t < 16; ++t) acc[t] = 0.0;
    double R = 0.0;
    const double tau = a.tau[k];
    for (int64_t q = a.pt_off[k]; q < a.pt_off[k + 1]; ++q) {
        __syncthreads();
        if (lane < 8) {
            // constrained basis of slot s = lane at the point
            const int s = lane;
            double b[4] = {0.0, 0.0, 0.0, 0.0};
            const double xi[3] = {a.xi[3 * q], a.xi[3 * q + 1], a.xi[3 * q + 2]};
            const int v0 = hang ? 0 : s, v1 = hang ? 8 : s + 1;
            for (int v = v0; v < v1; ++v) {
                const double c = hang ? sC[v][s] : 1.0;
                if (c == 0.0) continue;
                double f[3], g[3];
                for (int d = 0; d < 3; ++d) {
                    const bool up = (v >> d) & 1;
                    f[d] = 0.5 * (up ? 1.0 + xi[d] : 1.0 - xi[d]);
                    g[d] = up ? hg : -hg;
                }
                b[0] += c * (f[0] * f[1] * f[2]);
                b[1] += c * (g[0] * f[1] * f[2]);
                b[2] += c * (f[0] * g[1] * f[2]);
                b[3] += c * (f[0] * f[1] * g[2]);
            }
            for (int r = 0; r < 4; ++r) sB[r][s] = b[r];
        }
        __syncthreads();
        // state at the point (every lane, from the LDS)
        double ut[3] = {0, 0, 0}, gu[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, p = 0.0;
        for (int s = 0; s < 8; ++s) {
            for (int i = 0; i < 3; ++i) {
                const double uth = th * sU[i][s] + (1.0 - th) * sU[4 + i][s];
                ut[i] += sB[0][s] * uth;
                for (int j = 0; j < 3; ++j) gu[i][j] += sB[1 + j][s] * uth;
            }
            p += sB[0][s] * sU[3][s];
        }
        const double n[3] = {a.n[3 * q], a.n[3 * q + 1], a.n[3 * q + 2]};
        const double W = a.w[q];
        double v[3], vn = 0.0, un = 0.0;
        for (int i = 0; i < 3; ++i) {
            v[i] = ut[i] - a.g[i];
            vn += v[i] * n[i];
            un += ut[i] * n[i];
        }
        const double chi = un < 0.0 ? 1.0 : 0.0;
        if (MAT || JV) {
            const double Na = sB[0][aa], Nb = sB[0][bb];
            const double dNa[3] = {sB[1][aa], sB[2][aa], sB[3][aa]};
            const double dNb[3] = {sB[1][bb], sB[2][bb], sB[3][bb]};
            const double dnNa = dNa[0] * n[0] + dNa[1] * n[1] + dNa[2] * n[2];
            const double dnNb = dNb[0] * n[0] + dNb[1] * n[1] + dNb[2] * n[2];
            const double NN = Na * Nb;
            double K[16];
            for (int i = 0; i < 3; ++i) {
                for (int j = 0; j < 3; ++j) {
                    const double dij = i == j ? 1.0 : 0.0;
                    K[4 * i + j] = W * (-mu * th * Na * (dij * dnNb + dNb[i] * n[j]) -
                                        mu * th * (dij * Nb * dnNa + n[i] * dNa[j] * Nb) -
                                        chi * rho * th * NN * (n[j] * v[i] + un * dij) +
                                        th * NN * (tau * (dij - n[i] * n[j]) + tau * n[i] * n[j]));
                }
                K[4 * i + 3] = W * NN * n[i];
                K[12 + i] = -W * th * NN * n[i];
            }
            K[15] = 0.0;
            if (MAT) {
                for (int t = 0; t < 16; ++t) acc[t] += K[t];
            } else {
                for (int i = 0; i < 4; ++i)
                    for (int j = 0; j < 4; ++j) acc[i] += K[4 * i + j] * sU[7 + j][bb];
            }
        }
        if (!JV && lane < 32) {
            const double Na = sB[0][ra];
            const double dNa[3] = {sB[1][ra], sB[2][ra], sB[3][ra]};
            const double dnNa = dNa[0] * n[0] + dNa[1] * n[1] + dNa[2] * n[2];
            double r;
            if (ri < 3) {
                const int i = ri;
                const double epsn = (gu[i][0] + gu[0][i]) * n[0] + (gu[i][1] + gu[1][i]) * n[1] +
                                    (gu[i][2] + gu[2][i]) * n[2];
                const double gNv = dNa[0] * v[0] + dNa[1] * v[1] + dNa[2] * v[2];
                r = Na * (p * n[i] - mu * epsn) - mu * (v[i] * dnNa + n[i] * gNv) -
                    chi * rho * un * v[i] * Na + Na * (tau * (v[i] - n[i] * vn) + tau * n[i] * vn);
            } else {
                r = -Na * vn;
            }
            R += W * r;
        }
    }
    if (MAT) {
        TR *dst = (TR *)a.em + (a.slot0 + k) * 1024 + (aa * 8 + bb) * 16;
        for (int t = 0; t < 16; ++t) dst[t] = (TR)acc[t];
    }
    if (JV) {
        // y_a = sum_b K_ab x_b: reduce over the 8 lanes of slot a
        for (int off = 1; off < 8; off <<= 1)
            for (int i = 0; i < 4; ++i) acc[i] += __shfl_xor(acc[i], off, 8);
        if (bb == 0 && a.rrec)
            for (int i = 0; i < 4; ++i) a.rrec[(a.slot0 + k) * 32 + 4 * aa + i] = acc[i];
    } else if (a.rrec && lane < 32) {
        a.rrec[(a.slot0 + k) * 32 + 4 * ra + ri] = R;
    }
}

void launch_surface(hipStream_t s, const SurfArgs &a, int mode, bool fp64, const double *x) {
    if (a.n_items <= 0) return;
    dim3 grid((unsigned)a.n_items), block(64);
    if (mode == 0) {
        if (fp64) hipLaunchKernelGGL((k_surface<double, 0>), grid, block, 0, s, a, x);
        else hipLaunchKernelGGL((k_surface<float, 0>), grid, block, 0, s, a, x);
    } else if (mode == 1) {
        hipLaunchKernelGGL((k_surface<double, 1>), grid, block, 0, s, a, x);
    } else {
        hipLaunchKernelGGL((k_surface<double, 2>), grid, block, 0, s, a, x);
    }
}

}  // namespace vmsk

// VMS element assembly of libvms (gfx950), FP64 form.
//
// Residual and Jacobian of the VMS weak form, eq. (vms), with the fine
// scales u' = -tau_M r_M (eq. uprime, f = 0, the viscous part of div sigma
// dropped for trilinear fields) and p' = -rho tau_C div u (eq. pprime), Crank-
// Nicolson in theta form (u_theta = theta u + (1-theta) u_prev), tau's frozen.
//
// At every quadrature point q the Jacobian is B_q^T D_q B_q and the residual
// B_q^T r_q, where B_q (4 x 8) holds [N_s; dN_s/dx; dN_s/dy; dN_s/dz] of the
// *constrained* basis of master slot s (B C, with C the hanging-node operator
// M_e of Alg. 3), and D_q (16 x 16, blocks D^{ij} of 4 x 4 for test
// component i and trial component j) collects the coefficients of the
// linearised integrand:
//   D^{ij}[0][0]  multiplies N_a N_b,  D^{ij}[0][1+l] N_a d_l N_b,
//   D^{ij}[1+k][0] d_k N_a N_b,        D^{ij}[1+k][1+l] d_k N_a d_l N_b.
// This is the matrix form of the precomputed-operator assembly of Alg. 6 and
// App. A (basis values and gradients tabulated at Gauss points, element
// matrix as a contraction over points).
//
// One 64-lane workgroup per element. Lanes own 4x4 tiles of the 32x32
// element matrix: lane = (i, a-half, b-half, j) with j fastest, so that the
// atomic scatter of four consecutive lanes hits four consecutive CSR entries.
#include "geom.h"
#include "kernels.h"

namespace vmsk {
using namespace vmsd;

enum {
    Q_W = 0, Q_TM = 1, Q_TC = 2, Q_TB = 3, Q_UT = 4, Q_UP = 7, Q_GU = 10, Q_GA = 19, Q_S = 28,
    Q_R0 = 31, Q_P = 35, Q_PP = 36, NQ = 37
};

__device__ inline const double *field_ptr(const AsmArgs &a, int f) {
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

// reference coordinates and weight of point pt of the item
template <bool SUB>
__device__ inline void point_of(const AsmArgs &a, int64_t item, int pt, double h, double xi[3],
                                double &w) {
    if (!SUB) {
        for (int k = 0; k < 3; ++k) xi[k] = ((pt >> k) & 1) ? VMS_XI : -VMS_XI;
        double hh = 0.5 * h;
        w = hh * hh * hh;
        return;
    }
    const uint32_t en = a.entries[a.pt_off[item] + pt];
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
    double hs = h * ldexp(1.0, -(l + 1));
    w = hs * hs * hs;
}

// trilinear basis of vertex v at xi: value and physical gradient (scale 2/h)
__device__ inline void basis_at(const double xi[3], int v, double two_over_h, double b[4]) {
    double f[3], g[3];
    for (int k = 0; k < 3; ++k) {
        double sg = ((v >> k) & 1) ? 1.0 : -1.0;
        f[k] = 0.5 * (1.0 + sg * xi[k]);
        g[k] = 0.5 * sg * two_over_h;
    }
    b[0] = f[0] * f[1] * f[2];
    b[1] = g[0] * f[1] * f[2];
    b[2] = f[0] * g[1] * f[2];
    b[3] = f[0] * f[1] * g[2];
}

template <int CH, bool SUB, bool MAT>
__global__ __launch_bounds__(64) void k_asm_f64(AsmArgs a) {
    __shared__ double sU[7][8];
    __shared__ double sC[8][8];
    __shared__ double sB[CH][4][8];
    __shared__ double sQ[CH][NQ];
    __shared__ int sM[8];
    const int lane = threadIdx.x;
    const int64_t item = blockIdx.x;
    const int e = a.items[item];
    const bool hang = a.has_hang[e] != 0;
    const double h = ldexp(a.root_len, -(int)a.level[e]);
    const double two_over_h = 2.0 / h;
    if (lane < 8) sM[lane] = a.masters[8 * (int64_t)e + lane];
    {
        const int v = lane >> 3, s = lane & 7, bit = 2 * (v * 8 + s);
        const uint32_t code = (a.ccode[4 * (int64_t)e + (bit >> 5)] >> (bit & 31)) & 3u;
        sC[v][s] = code == 3u ? 1.0 : (code == 2u ? 0.5 : (code == 1u ? 0.25 : 0.0));
    }
    __syncthreads();
    if (lane < 56) {
        const int f = lane >> 3, s = lane & 7, m = sM[s];
        sU[f][s] = m >= 0 ? field_ptr(a, f)[m] : 0.0;
    }
    const int npts = SUB ? a.pt_cnt[item] : 8;
    const double rho = a.rho, mu = a.mu, dt = a.dt, th = a.theta;

    // tile ownership
    const int j = lane & 3, bh = (lane >> 2) & 1, ah = (lane >> 3) & 1, i = lane >> 4;
    const bool rlane = (j == 0) && (bh == 0);
    double K[4][4];
    double R[4];
    for (int x = 0; x < 4; ++x) {
        R[x] = 0.0;
        for (int y = 0; y < 4; ++y) K[x][y] = 0.0;
    }

    for (int base = 0; base < npts; base += CH) {
        const int np = min(CH, npts - base);
        // ---- constrained basis B'[k][s] = sum_v B[k][v] C[v][s] at the chunk's points
        for (int idx = lane; idx < np * 8; idx += 64) {
            const int pt = idx >> 3, s = idx & 7;
            double xi[3], w;
            point_of<SUB>(a, item, base + pt, h, xi, w);
            double b[4];
            if (!hang) {
                basis_at(xi, s, two_over_h, b);
            } else {
                b[0] = b[1] = b[2] = b[3] = 0.0;
                for (int v = 0; v < 8; ++v) {
                    const double c = sC[v][s];
                    if (c == 0.0) continue;
                    double bv[4];
                    basis_at(xi, v, two_over_h, bv);
                    for (int k = 0; k < 4; ++k) b[k] += c * bv[k];
                }
            }
            for (int k = 0; k < 4; ++k) sB[pt][k][s] = b[k];
            if (s == 0) sQ[pt][Q_W] = w;
        }
        __syncthreads();
        // ---- point quantities (one lane per point)
        if (lane < np) {
            const int pt = lane;
            double ut[3] = {0, 0, 0}, at[3] = {0, 0, 0}, gp[3] = {0, 0, 0}, p = 0.0;
            double gu[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
            for (int s = 0; s < 8; ++s) {
                const double b0 = sB[pt][0][s], b1 = sB[pt][1][s], b2 = sB[pt][2][s],
                             b3 = sB[pt][3][s];
                for (int c = 0; c < 3; ++c) {
                    const double un = sU[c][s], u0 = sU[4 + c][s];
                    const double uth = th * un + (1.0 - th) * u0;
                    ut[c] += b0 * uth;
                    at[c] += b0 * (un - u0);
                    gu[c][0] += b1 * uth;
                    gu[c][1] += b2 * uth;
                    gu[c][2] += b3 * uth;
                }
                const double ps = sU[3][s];
                p += b0 * ps;
                gp[0] += b1 * ps;
                gp[1] += b2 * ps;
                gp[2] += b3 * ps;
            }
            for (int c = 0; c < 3; ++c) at[c] /= dt;
            double conv[3], rM[3];
            for (int c = 0; c < 3; ++c) {
                conv[c] = ut[0] * gu[c][0] + ut[1] * gu[c][1] + ut[2] * gu[c][2];
                rM[c] = rho * (at[c] + conv[c]) + gp[c];
            }
            const double div = gu[0][0] + gu[1][1] + gu[2][2];
            const double g = 4.0 / (h * h);
            const double nu = mu / rho;
            const double uGu = g * (ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2]);
            const double tauM = 1.0 / sqrt(a.c_t / (dt * dt) + uGu + a.c_i * nu * nu * 3.0 * g * g);
            const double tauC = 1.0 / (tauM * 3.0 * g);
            double up[3];
            for (int c = 0; c < 3; ++c) up[c] = -tauM * rM[c];
            const double pp = -rho * tauC * div;
            const double upg = g * (up[0] * up[0] + up[1] * up[1] + up[2] * up[2]);
            const double tb = upg > 0.0 ? 1.0 / sqrt(upg) : 0.0;
            double* q = sQ[pt];
            q[Q_TM] = tauM;
            q[Q_TC] = tauC;
            q[Q_TB] = tb;
            for (int c = 0; c < 3; ++c) {
                q[Q_UT + c] = ut[c];
                q[Q_UP + c] = up[c];
                const double sc = up[0] * gu[c][0] + up[1] * gu[c][1] + up[2] * gu[c][2];
                q[Q_S + c] = sc;
                q[Q_R0 + c] = rho * at[c] + rho * conv[c] + sc;
                for (int m = 0; m < 3; ++m) {
                    q[Q_GU + 3 * c + m] = gu[c][m];
                    // (gu A)[c][m] with A[k][m] = delta_km / dt + theta gu[k][m]
                    double v = 0.0;
                    for (int k = 0; k < 3; ++k)
                        v += gu[c][k] * ((k == m ? 1.0 / dt : 0.0) + th * gu[k][m]);
                    q[Q_GA + 3 * c + m] = v;
                }
            }
            q[Q_R0 + 3] = div;
            q[Q_P] = p;
            q[Q_PP] = pp;
        }
        __syncthreads();
        // ---- contraction: K += B'^T (W D) B', R += B'^T (W r)
        for (int pt = 0; pt < np; ++pt) {
            const double *q = sQ[pt];
            const double W = q[Q_W], tauM = q[Q_TM], tauC = q[Q_TC], tb = q[Q_TB];
            const double ut[3] = {q[Q_UT], q[Q_UT + 1], q[Q_UT + 2]};
            const double up[3] = {q[Q_UP], q[Q_UP + 1], q[Q_UP + 2]};
            double D[4][4];
            if (MAT) {
                if (i < 3 && j < 3) {
                    const double gij = q[Q_GU + 3 * i + j];
                    const double Aij = (i == j ? 1.0 / dt : 0.0) + th * gij;
                    const double GAij = q[Q_GA + 3 * i + j];
                    const double si = q[Q_S + i];
                    const double dij = (i == j) ? 1.0 : 0.0;
                    D[0][0] = rho * Aij - tauM * rho * GAij;
                    for (int l = 0; l < 3; ++l)
                        D[0][1 + l] = th * (dij * (rho * ut[l] + up[l]) - tauM * rho * gij * ut[l]);
                    for (int k = 0; k < 3; ++k) {
                        const double Akj = (k == j ? 1.0 / dt : 0.0) + th * q[Q_GU + 3 * k + j];
                        const double dkj = (k == j) ? 1.0 : 0.0;
                        D[1 + k][0] = -th * dkj * up[i] + tauM * rho * ut[k] * Aij +
                                      tauM * (Akj * up[i] + up[k] * Aij) -
                                      tb * tauM * rho * (Akj * si + up[k] * GAij);
                        for (int l = 0; l < 3; ++l) {
                            const double dkl = (k == l) ? 1.0 : 0.0, dil = (i == l) ? 1.0 : 0.0;
                            const double dki = (k == i) ? 1.0 : 0.0, dlj = (l == j) ? 1.0 : 0.0;
                            D[1 + k][1 + l] =
                                mu * th * (dij * dkl + dkj * dil) + tauM * rho * th * dij * ut[k] * ut[l] +
                                rho * tauC * th * dki * dlj +
                                tauM * th * ut[l] * (dkj * up[i] + up[k] * dij) +
                                tb * (-tauM * rho * th * dkj * ut[l] * si -
                                      tauM * rho * th * up[k] * ut[l] * gij + th * dij * up[k] * up[l]);
                        }
                    }
                } else if (i < 3) {  // momentum test, pressure trial
                    const double si = q[Q_S + i];
                    D[0][0] = 0.0;
                    for (int l = 0; l < 3; ++l) D[0][1 + l] = -tauM * q[Q_GU + 3 * i + l];
                    for (int k = 0; k < 3; ++k) {
                        D[1 + k][0] = (k == i) ? -1.0 : 0.0;
                        for (int l = 0; l < 3; ++l) {
                            const double dkl = (k == l) ? 1.0 : 0.0, dli = (l == i) ? 1.0 : 0.0;
                            D[1 + k][1 + l] = tauM * ut[k] * dli +
                                              (tauM / rho) * (up[i] * dkl + up[k] * dli) -
                                              tb * tauM * (si * dkl + up[k] * q[Q_GU + 3 * i + l]);
                        }
                    }
                } else if (j < 3) {  // continuity test, velocity trial
                    D[0][0] = 0.0;
                    for (int l = 0; l < 3; ++l) D[0][1 + l] = (l == j) ? th : 0.0;
                    for (int k = 0; k < 3; ++k) {
                        D[1 + k][0] = tauM * ((k == j ? 1.0 / dt : 0.0) + th * q[Q_GU + 3 * k + j]);
                        for (int l = 0; l < 3; ++l)
                            D[1 + k][1 + l] = (k == j) ? tauM * th * ut[l] : 0.0;
                    }
                } else {  // continuity test, pressure trial
                    for (int k = 0; k < 4; ++k)
                        for (int l = 0; l < 4; ++l)
                            D[k][l] = (k == l && k > 0) ? tauM / rho : 0.0;
                }
                for (int k = 0; k < 4; ++k)
                    for (int l = 0; l < 4; ++l) D[k][l] *= W;
                // E[k][bb] = sum_l D[k][l] B'[l][b]
                double E[4][4];
                for (int bb = 0; bb < 4; ++bb) {
                    const int b = 4 * bh + bb;
                    const double B0 = sB[pt][0][b], B1 = sB[pt][1][b], B2 = sB[pt][2][b],
                                 B3 = sB[pt][3][b];
                    for (int k = 0; k < 4; ++k)
                        E[k][bb] = D[k][0] * B0 + D[k][1] * B1 + D[k][2] * B2 + D[k][3] * B3;
                }
                for (int aa = 0; aa < 4; ++aa) {
                    const int av = 4 * ah + aa;
                    const double A0 = sB[pt][0][av], A1 = sB[pt][1][av], A2 = sB[pt][2][av],
                                 A3 = sB[pt][3][av];
                    for (int bb = 0; bb < 4; ++bb)
                        K[aa][bb] += A0 * E[0][bb] + A1 * E[1][bb] + A2 * E[2][bb] + A3 * E[3][bb];
                }
            }
            if (rlane) {
                double r[4];
                if (i < 3) {
                    const double p = q[Q_P], pp = q[Q_PP], si = q[Q_S + i];
                    r[0] = q[Q_R0 + i];
                    for (int k = 0; k < 3; ++k)
                        r[1 + k] = mu * (q[Q_GU + 3 * i + k] + q[Q_GU + 3 * k + i]) -
                                   (k == i ? p + pp : 0.0) - ut[k] * up[i] - up[k] * up[i] / rho +
                                   tb * up[k] * si;
                } else {
                    r[0] = q[Q_R0 + 3];
                    for (int k = 0; k < 3; ++k) r[1 + k] = -up[k] / rho;
                }
                for (int aa = 0; aa < 4; ++aa) {
                    const int av = 4 * ah + aa;
                    R[aa] += W * (sB[pt][0][av] * r[0] + sB[pt][1][av] * r[1] +
                                  sB[pt][2][av] * r[2] + sB[pt][3][av] * r[3]);
                }
            }
        }
        __syncthreads();
    }
    // ---- scatter with the constraint already folded into B'
    if (MAT) {
        double *vals = (double *)a.vals;
        for (int aa = 0; aa < 4; ++aa) {
            const int sa = 4 * ah + aa;
            if (sM[sa] < 0) continue;
            const int64_t row = a.rowbase[8 * (int64_t)e + sa] + (int64_t)i * a.rowlen[8 * (int64_t)e + sa];
            for (int bb = 0; bb < 4; ++bb) {
                const int sb = 4 * bh + bb;
                if (sM[sb] < 0) continue;
                const int64_t idx = row + 4 * (int64_t)a.kk[64 * (int64_t)e + 8 * sa + sb] + j;
                atomicAdd(vals + idx, K[aa][bb]);
            }
        }
    }
    if (rlane && a.resid) {
        for (int aa = 0; aa < 4; ++aa) {
            const int sa = 4 * ah + aa;
            if (sM[sa] >= 0) atomicAdd(a.resid + 4 * (int64_t)sM[sa] + i, R[aa]);
        }
    }
}

void launch_assemble_f64(hipStream_t s, const AsmArgs &a, bool sub, bool mat) {
    if (a.n_items <= 0) return;
    dim3 grid((unsigned)a.n_items), block(64);
    if (!sub) {
        if (mat) hipLaunchKernelGGL((k_asm_f64<8, false, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_asm_f64<8, false, false>), grid, block, 0, s, a);
    } else {
        if (mat) hipLaunchKernelGGL((k_asm_f64<32, true, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_asm_f64<32, true, false>), grid, block, 0, s, a);
    }
}

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

/*
 * CPU reference ("oracle") for the VMS assembly and in-out hot path.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library. It shares no code with
 * the HIP library: the two are independent formulations of the same method.
 *
 * Everything here is plain, slow FP64 code that follows the paper's
 * definitions step by step:
 *   - VMS residual term by term, eq. (vms) with the fine scales of
 *     eqs. (uprime) and (pprime);
 *   - element Jacobian by complex-step differentiation of that residual with
 *     the stabilisation parameters frozen (the paper gives no linearisation);
 *   - hanging-node constraints applied by the chain rule, R_master = C^T R;
 *   - exact point-in-polyhedron labels by segment-crossing parity with exact
 *     orientation predicates (expansion arithmetic, Shewchuk 1997), which is
 *     the ground truth that the normal test of Alg. 5 and ray tracing
 *     approximate;
 *   - adaptive sub-cell quadrature of INTERCEPTED elements (Section
 *     "Adaptive Quadrature" and the caption of the Gauss-point figure),
 *     recursive depth-first;
 *   - exact unsigned distance to a triangle (closest point by Voronoi regions).
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -fPIC -shared (no fused
 * multiply-add contraction anywhere, so point coordinates are bit-identical
 * to the device formula).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ------------------------------------------------------------------------ */
/* Parameters                                                                */
/* ------------------------------------------------------------------------ */

typedef struct {
    double rho, mu, dt, theta, c_t, c_i;
    int32_t term_mask; /* bit k enables term k of the residual, see below */
    int32_t pad;
} or_params;

/* Term bits (eq. vms):
 *  0 Galerkin time derivative  w . rho du/dt
 *  1 Galerkin convection       w . rho (u . grad u)
 *  2 viscous                   eps(w) : 2 mu eps(u)
 *  3 pressure                  -p div w
 *  4 continuity                q div u
 *  5 SUPG / PSPG               -(u . grad w + grad q / rho) . u'
 *  6 fine-scale pressure       -p' div w
 *  7 cross stress              w . (u' . grad u)
 *  8 Reynolds stress           -(grad w / rho) : (u' (x) u')
 *  9 tau-bar term              (u' . grad w) taubar (u' . grad u)
 */
#define OR_ALL_TERMS 0x3FF

/* ------------------------------------------------------------------------ */
/* Trilinear basis on the reference cube [-1,1]^3, node a = (a&1, a>>1&1, a>>2&1) */
/* ------------------------------------------------------------------------ */

static void basis(const double xi[3], double h, double N[8], double dN[8][3]) {
    for (int a = 0; a < 8; ++a) {
        double s[3] = {(a & 1) ? 1.0 : -1.0, (a & 2) ? 1.0 : -1.0, (a & 4) ? 1.0 : -1.0};
        double f[3], g[3];
        for (int k = 0; k < 3; ++k) {
            f[k] = 0.5 * (1.0 + s[k] * xi[k]);
            g[k] = 0.5 * s[k] * (2.0 / h); /* d/dx = (2/h) d/dxi */
        }
        N[a] = f[0] * f[1] * f[2];
        dN[a][0] = g[0] * f[1] * f[2];
        dN[a][1] = f[0] * g[1] * f[2];
        dN[a][2] = f[0] * f[1] * g[2];
    }
}

/* Stabilisation parameters at one point from the real state (frozen). */
typedef struct { double tauM, tauC, taubar; } taus;

/* ------------------------------------------------------------------------ */
/* Residual of one element at a list of points.                             */
/*   Uv[a][c]  complex vertex values of the new step (c: ux,uy,uz,p)         */
/*   U0v[a][c] real vertex values of the previous step velocity             */
/*   Rv[a][c]  output, vertex test functions (before the constraint)         */
/* ------------------------------------------------------------------------ */

static void element_residual(const or_params *P, double h, int npt, const double *xi,
                             const double *w, const taus *tau, cplx Uv[8][4],
                             const double U0v[8][3], cplx Rv[8][4]) {
    const double rho = P->rho, mu = P->mu, dt = P->dt, th = P->theta;
    const int m = P->term_mask;
    for (int a = 0; a < 8; ++a)
        for (int c = 0; c < 4; ++c) Rv[a][c] = 0;
    for (int q = 0; q < npt; ++q) {
        double N[8], dN[8][3];
        basis(xi + 3 * q, h, N, dN);
        const double W = w[q];
        /* interpolation of u_theta, its gradient, du/dt, p, grad p */
        cplx ut[3] = {0, 0, 0}, gu[3][3] = {{0}}, at[3] = {0, 0, 0}, p = 0, gp[3] = {0, 0, 0};
        for (int a = 0; a < 8; ++a) {
            for (int i = 0; i < 3; ++i) {
                cplx uth = th * Uv[a][i] + (1.0 - th) * U0v[a][i];
                ut[i] += N[a] * uth;
                at[i] += N[a] * (Uv[a][i] - U0v[a][i]) / dt;
                for (int j = 0; j < 3; ++j) gu[i][j] += dN[a][j] * uth; /* d_j u_i */
            }
            p += N[a] * Uv[a][3];
            for (int j = 0; j < 3; ++j) gp[j] += dN[a][j] * Uv[a][3];
        }
        /* strong residuals (f = 0; the viscous part of div sigma vanishes
           for the reading that drops second derivatives of trilinear fields) */
        cplx rM[3], rC = gu[0][0] + gu[1][1] + gu[2][2];
        for (int i = 0; i < 3; ++i) {
            cplx conv = ut[0] * gu[i][0] + ut[1] * gu[i][1] + ut[2] * gu[i][2];
            rM[i] = rho * (at[i] + conv) + gp[i];
        }
        /* fine scales, eqs. (uprime), (pprime) */
        cplx up[3];
        for (int i = 0; i < 3; ++i) up[i] = -tau[q].tauM * rM[i];
        cplx pp = -rho * tau[q].tauC * rC;
        const double tb = tau[q].taubar;

        for (int a = 0; a < 8; ++a) {
            cplx u_dot_gradNa = ut[0] * dN[a][0] + ut[1] * dN[a][1] + ut[2] * dN[a][2];
            cplx up_dot_gradNa = up[0] * dN[a][0] + up[1] * dN[a][1] + up[2] * dN[a][2];
            for (int i = 0; i < 3; ++i) {
                cplx r = 0;
                cplx conv_i = ut[0] * gu[i][0] + ut[1] * gu[i][1] + ut[2] * gu[i][2];
                cplx upgu_i = up[0] * gu[i][0] + up[1] * gu[i][1] + up[2] * gu[i][2];
                if (m & (1 << 0)) r += N[a] * rho * at[i];
                if (m & (1 << 1)) r += N[a] * rho * conv_i;
                if (m & (1 << 2)) {
                    /* eps(w):2 mu eps(u) with w = N_a e_i */
                    cplx v = 0;
                    for (int j = 0; j < 3; ++j) v += dN[a][j] * (gu[i][j] + gu[j][i]);
                    r += mu * v;
                }
                if (m & (1 << 3)) r += -p * dN[a][i];
                if (m & (1 << 5)) r += -u_dot_gradNa * up[i];
                if (m & (1 << 6)) r += -pp * dN[a][i];
                if (m & (1 << 7)) r += N[a] * upgu_i;
                if (m & (1 << 8)) r += -(1.0 / rho) * up_dot_gradNa * up[i];
                if (m & (1 << 9)) r += up_dot_gradNa * tb * upgu_i;
                Rv[a][i] += W * r;
            }
            cplx rc = 0;
            if (m & (1 << 4)) rc += N[a] * rC;
            if (m & (1 << 5)) rc += -(1.0 / rho) * up_dot_gradNa;
            Rv[a][3] += W * rc;
        }
    }
}

/* Stabilisation parameters from the real state, one per point.
 * G = (2/h)^2 I for cubic octants; tau_M = (C_t/dt^2 + u.G.u + C_I nu^2 G:G)^(-1/2),
 * tau_C = 1/(tau_M tr G), taubar = (u'.G.u')^(-1/2) (0 if u' = 0). */
static void element_taus(const or_params *P, double h, int npt, const double *xi,
                         const double Uv[8][4], const double U0v[8][3], taus *tau) {
    const double rho = P->rho, dt = P->dt, th = P->theta, nu = P->mu / P->rho;
    const double g = 4.0 / (h * h);
    for (int q = 0; q < npt; ++q) {
        double N[8], dN[8][3];
        basis(xi + 3 * q, h, N, dN);
        double ut[3] = {0, 0, 0}, gu[3][3] = {{0}}, at[3] = {0, 0, 0}, gp[3] = {0, 0, 0};
        for (int a = 0; a < 8; ++a) {
            for (int i = 0; i < 3; ++i) {
                double uth = th * Uv[a][i] + (1.0 - th) * U0v[a][i];
                ut[i] += N[a] * uth;
                at[i] += N[a] * (Uv[a][i] - U0v[a][i]) / dt;
                for (int j = 0; j < 3; ++j) gu[i][j] += dN[a][j] * uth;
            }
            for (int j = 0; j < 3; ++j) gp[j] += dN[a][j] * Uv[a][3];
        }
        double uGu = g * (ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2]);
        double GG = 3.0 * g * g, trG = 3.0 * g;
        double tauM = 1.0 / sqrt(P->c_t / (dt * dt) + uGu + P->c_i * nu * nu * GG);
        double tauC = 1.0 / (tauM * trG);
        double up[3];
        for (int i = 0; i < 3; ++i) {
            double conv = ut[0] * gu[i][0] + ut[1] * gu[i][1] + ut[2] * gu[i][2];
            up[i] = -tauM * (rho * (at[i] + conv) + gp[i]);
        }
        double upGup = g * (up[0] * up[0] + up[1] * up[1] + up[2] * up[2]);
        tau[q].tauM = tauM;
        tau[q].tauC = tauC;
        tau[q].taubar = (upGup > 0.0) ? 1.0 / sqrt(upGup) : 0.0;
    }
}

/* One element: master values in, constrained residual (nm x 4) and Jacobian
 * ((nm*4) x (nm*4), row-major) out. C is 8 x nm (vertex a, master s). */
static void element_assemble(const or_params *P, double h, int npt, const double *xi,
                             const double *w, int nm, const double *C,
                             const double *Um /* nm x 4 */, const double *U0m /* nm x 3 */,
                             double *Rm, double *Jm) {
    double Uv[8][4], U0v[8][3];
    for (int a = 0; a < 8; ++a) {
        for (int c = 0; c < 4; ++c) {
            double s = 0;
            for (int t = 0; t < nm; ++t) s += C[a * nm + t] * Um[t * 4 + c];
            Uv[a][c] = s;
        }
        for (int c = 0; c < 3; ++c) {
            double s = 0;
            for (int t = 0; t < nm; ++t) s += C[a * nm + t] * U0m[t * 3 + c];
            U0v[a][c] = s;
        }
    }
    taus *tau = (taus *)malloc(sizeof(taus) * (npt > 0 ? npt : 1));
    element_taus(P, h, npt, xi, (const double(*)[4])Uv, (const double(*)[3])U0v, tau);

    const int nd = nm * 4;
    const double eps = 1e-30;
    cplx Ucv[8][4], Rv[8][4];
    for (int col = -1; col < nd; ++col) {
        /* perturb master dof col by i*eps, map to vertices through C */
        for (int a = 0; a < 8; ++a)
            for (int c = 0; c < 4; ++c) {
                cplx s = Uv[a][c];
                if (col >= 0 && (col % 4) == c) s += I * eps * C[a * nm + col / 4];
                Ucv[a][c] = s;
            }
        element_residual(P, h, npt, xi, w, tau, Ucv, (const double(*)[3])U0v, Rv);
        /* R_master[s][c] = sum_a C[a][s] R_vertex[a][c] */
        for (int s = 0; s < nm; ++s)
            for (int c = 0; c < 4; ++c) {
                cplx v = 0;
                for (int a = 0; a < 8; ++a) v += C[a * nm + s] * Rv[a][c];
                if (col < 0)
                    Rm[s * 4 + c] = creal(v);
                else
                    Jm[(s * 4 + c) * nd + col] = cimag(v) / eps;
            }
    }
    free(tau);
}

/* ------------------------------------------------------------------------ */
/* Global assembly into a given CSR pattern                                  */
/* ------------------------------------------------------------------------ */

static int64_t csr_find(const int64_t *row_ptr, const int32_t *col, int64_t r, int32_t c) {
    int64_t lo = row_ptr[r], hi = row_ptr[r + 1] - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (col[mid] == c) return mid;
        if (col[mid] < c) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* Elements: masters (up to 8) and constraint matrices C (8 x 8, vertex x
 * master slot, padded with zeros), size h, point lists [pt_off[e], pt_off[e+1]).
 * Fields are SoA over independent nodes. Outputs are accumulated (+=).
 * Returns 0, or -(e+1) if an entry is missing from the pattern. */
int64_t or_assemble(const or_params *P, int64_t n_el, const int32_t *el_nm,
                    const int32_t *el_master, const double *el_C, const double *el_h,
                    const int64_t *pt_off, const double *pt_xi, const double *pt_w,
                    const double *ux, const double *uy, const double *uz, const double *pr,
                    const double *ux0, const double *uy0, const double *uz0,
                    const int64_t *row_ptr, const int32_t *col, double *vals, double *resid,
                    int64_t el_begin, int64_t el_end) {
    if (el_end < 0 || el_end > n_el) el_end = n_el;
    for (int64_t e = el_begin; e < el_end; ++e) {
        const int nm = el_nm[e];
        const int npt = (int)(pt_off[e + 1] - pt_off[e]);
        if (npt == 0 || nm == 0) continue;
        const int32_t *ms = el_master + 8 * e;
        double C[64], Um[32], U0m[24], Rm[32], Jm[1024];
        for (int a = 0; a < 8; ++a)
            for (int s = 0; s < nm; ++s) C[a * nm + s] = el_C[64 * e + a * 8 + s];
        for (int s = 0; s < nm; ++s) {
            int32_t n = ms[s];
            Um[s * 4 + 0] = ux[n]; Um[s * 4 + 1] = uy[n]; Um[s * 4 + 2] = uz[n]; Um[s * 4 + 3] = pr[n];
            U0m[s * 3 + 0] = ux0[n]; U0m[s * 3 + 1] = uy0[n]; U0m[s * 3 + 2] = uz0[n];
        }
        element_assemble(P, el_h[e], npt, pt_xi + 3 * pt_off[e], pt_w + pt_off[e], nm, C, Um, U0m,
                         Rm, Jm);
        const int nd = nm * 4;
        for (int r = 0; r < nd; ++r) {
            int64_t grow = 4 * (int64_t)ms[r / 4] + (r % 4);
            if (resid) resid[grow] += Rm[r];
            if (!vals) continue;
            for (int c = 0; c < nd; ++c) {
                int32_t gcol = 4 * ms[c / 4] + (c % 4);
                int64_t k = csr_find(row_ptr, col, grow, gcol);
                if (k < 0) return -(e + 1);
                vals[k] += Jm[r * nd + c];
            }
        }
    }
    return 0;
}

/* Jacobian action y += J x, J the Jacobian of the residual with the
 * stabilisation parameters frozen at the state: the derivative of the
 * residual along x by one complex-step evaluation per element (the
 * directional derivative that defines the product, independent of the
 * column-by-column Jacobian above). x and y are indexed by dof 4 node + c. */
void or_apply_jacobian(const or_params *P, int64_t n_el, const int32_t *el_nm,
                       const int32_t *el_master, const double *el_C, const double *el_h,
                       const int64_t *pt_off, const double *pt_xi, const double *pt_w,
                       const double *ux, const double *uy, const double *uz, const double *pr,
                       const double *ux0, const double *uy0, const double *uz0, const double *x,
                       double *y) {
    const double eps = 1e-30;
    for (int64_t e = 0; e < n_el; ++e) {
        const int nm = el_nm[e];
        const int npt = (int)(pt_off[e + 1] - pt_off[e]);
        if (npt == 0 || nm == 0) continue;
        const int32_t *ms = el_master + 8 * e;
        const double *C = el_C + 64 * e; /* C[a * 8 + s] */
        double Uv[8][4], U0v[8][3], Xv[8][4];
        for (int a = 0; a < 8; ++a) {
            for (int c = 0; c < 4; ++c) {
                double su = 0, sx = 0;
                for (int t = 0; t < nm; ++t) {
                    const int32_t n = ms[t];
                    const double un = c == 0 ? ux[n] : c == 1 ? uy[n] : c == 2 ? uz[n] : pr[n];
                    su += C[a * 8 + t] * un;
                    sx += C[a * 8 + t] * x[4 * (int64_t)n + c];
                }
                Uv[a][c] = su;
                Xv[a][c] = sx;
            }
            for (int c = 0; c < 3; ++c) {
                double s0 = 0;
                for (int t = 0; t < nm; ++t) {
                    const int32_t n = ms[t];
                    s0 += C[a * 8 + t] * (c == 0 ? ux0[n] : c == 1 ? uy0[n] : uz0[n]);
                }
                U0v[a][c] = s0;
            }
        }
        taus *tau = (taus *)malloc(sizeof(taus) * npt);
        element_taus(P, el_h[e], npt, pt_xi + 3 * pt_off[e], (const double(*)[4])Uv,
                     (const double(*)[3])U0v, tau);
        cplx Ucv[8][4], Rv[8][4];
        for (int a = 0; a < 8; ++a)
            for (int c = 0; c < 4; ++c) Ucv[a][c] = Uv[a][c] + I * eps * Xv[a][c];
        element_residual(P, el_h[e], npt, pt_xi + 3 * pt_off[e], pt_w + pt_off[e], tau, Ucv,
                         (const double(*)[3])U0v, Rv);
        free(tau);
        for (int s = 0; s < nm; ++s)
            for (int c = 0; c < 4; ++c) {
                cplx v = 0;
                for (int a = 0; a < 8; ++a) v += C[a * 8 + s] * Rv[a][c];
                y[4 * (int64_t)ms[s] + c] += cimag(v) / eps;
            }
    }
}

/* ------------------------------------------------------------------------ */
/* Weak (Nitsche) boundary terms of eq. (weakbc) at surface points           */
/* ------------------------------------------------------------------------ */

/* tau_B (tangential, normal) and the prescribed velocity g on the surface */
typedef struct { double tauT, tauN, g[3]; } or_wbc;

/* Surface residual of one element at npt surface points: reference
 * coordinates xi, area weights ws, unit normal n of the fluid domain (into
 * the body) and the inflow indicator chi (1 where u_theta . n < 0 at the real
 * state, frozen like the taus). Velocity terms use u_theta, the pressure the
 * new step, as in the volume terms. For w = N_a e_i and q = N_a:
 *   -w.(-p n + 2 mu eps(u) n)   = N_a (p n_i - mu sum_k (d_k u_i + d_i u_k) n_k)
 *   -(2 mu eps(w) n).(u - g)    = -mu ((u - g)_i dN_a/dn + n_i grad N_a . (u - g))
 *   -(q n).(u - g)              = -N_a n . (u - g)
 *   -w.rho (u.n)(u - g) (inflow) = -chi rho (u . n) (u - g)_i N_a
 *   tangential and normal penalties: N_a (tauT ((u-g)_i - n_i (u-g).n) + tauN n_i (u-g).n) */
static void surface_residual(const or_params *P, const or_wbc *B, double h, int npt,
                             const double *xi, const double *ws, const double *nrm,
                             const double *chi, cplx Uv[8][4], const double U0v[8][3],
                             cplx Rv[8][4]) {
    const double rho = P->rho, mu = P->mu, th = P->theta;
    for (int a = 0; a < 8; ++a)
        for (int c = 0; c < 4; ++c) Rv[a][c] = 0;
    for (int q = 0; q < npt; ++q) {
        double N[8], dN[8][3];
        basis(xi + 3 * q, h, N, dN);
        const double *n = nrm + 3 * q;
        const double W = ws[q];
        cplx ut[3] = {0, 0, 0}, gu[3][3] = {{0}}, p = 0;
        for (int a = 0; a < 8; ++a) {
            for (int i = 0; i < 3; ++i) {
                cplx uth = th * Uv[a][i] + (1.0 - th) * U0v[a][i];
                ut[i] += N[a] * uth;
                for (int j = 0; j < 3; ++j) gu[i][j] += dN[a][j] * uth;
            }
            p += N[a] * Uv[a][3];
        }
        cplx v[3], vn = 0, un = 0;
        for (int i = 0; i < 3; ++i) {
            v[i] = ut[i] - B->g[i];
            vn += v[i] * n[i];
            un += ut[i] * n[i];
        }
        for (int a = 0; a < 8; ++a) {
            double dnNa = 0;
            cplx gNv = 0;
            for (int k = 0; k < 3; ++k) {
                dnNa += dN[a][k] * n[k];
                gNv += dN[a][k] * v[k];
            }
            for (int i = 0; i < 3; ++i) {
                cplx epsn = 0;
                for (int k = 0; k < 3; ++k) epsn += (gu[i][k] + gu[k][i]) * n[k];
                cplx r = N[a] * (p * n[i] - mu * epsn);
                r += -mu * (v[i] * dnNa + n[i] * gNv);
                r += -chi[q] * rho * un * v[i] * N[a];
                r += N[a] * (B->tauT * (v[i] - n[i] * vn) + B->tauN * n[i] * vn);
                Rv[a][i] += W * r;
            }
            Rv[a][3] += W * (-N[a] * vn);
        }
    }
}

/* Surface terms of the items (one element each, points [pt_off[k],
 * pt_off[k+1])), residual and complex-step Jacobian (tau_B and the inflow
 * indicator frozen at the real state), added into the CSR (+=). tau_b holds
 * each item's tau_B (tangential = normal). Returns 0 or -(k+1) if an entry is
 * missing from the pattern. */
int64_t or_surface_assemble(const or_params *P, const double *g, int64_t n_items,
                            const int32_t *item_el, const int32_t *el_nm,
                            const int32_t *el_master, const double *el_C, const double *el_h,
                            const int64_t *pt_off, const double *pt_xi, const double *pt_w,
                            const double *pt_n, const double *tau_b, const double *ux,
                            const double *uy, const double *uz, const double *pr,
                            const double *ux0, const double *uy0, const double *uz0,
                            const int64_t *row_ptr, const int32_t *col, double *vals,
                            double *resid) {
    const double eps = 1e-30;
    for (int64_t k = 0; k < n_items; ++k) {
        const int32_t e = item_el[k];
        const int nm = el_nm[e];
        const int npt = (int)(pt_off[k + 1] - pt_off[k]);
        if (npt == 0 || nm == 0) continue;
        const int32_t *ms = el_master + 8 * e;
        const double *C = el_C + 64 * (int64_t)e; /* C[a * 8 + s] */
        const double *xi = pt_xi + 3 * pt_off[k], *ws = pt_w + pt_off[k], *nr = pt_n + 3 * pt_off[k];
        or_wbc B = {tau_b[k], tau_b[k], {g[0], g[1], g[2]}};
        double Uv[8][4], U0v[8][3];
        for (int a = 0; a < 8; ++a) {
            for (int c = 0; c < 4; ++c) {
                double su = 0;
                for (int t = 0; t < nm; ++t) {
                    const int32_t n = ms[t];
                    su += C[a * 8 + t] * (c == 0 ? ux[n] : c == 1 ? uy[n] : c == 2 ? uz[n] : pr[n]);
                }
                Uv[a][c] = su;
            }
            for (int c = 0; c < 3; ++c) {
                double s0 = 0;
                for (int t = 0; t < nm; ++t) {
                    const int32_t n = ms[t];
                    s0 += C[a * 8 + t] * (c == 0 ? ux0[n] : c == 1 ? uy0[n] : uz0[n]);
                }
                U0v[a][c] = s0;
            }
        }
        /* inflow indicator from the real state */
        double *chi = (double *)malloc(sizeof(double) * npt);
        for (int q = 0; q < npt; ++q) {
            double N[8], dN[8][3], un = 0;
            basis(xi + 3 * q, el_h[e], N, dN);
            for (int i = 0; i < 3; ++i) {
                double u = 0;
                for (int a = 0; a < 8; ++a) u += N[a] * (P->theta * Uv[a][i] + (1.0 - P->theta) * U0v[a][i]);
                un += u * nr[3 * q + i];
            }
            chi[q] = un < 0.0 ? 1.0 : 0.0;
        }
        const int nd = nm * 4;
        double Rm[32], Jm[1024];
        cplx Ucv[8][4], Rv[8][4];
        for (int colx = -1; colx < nd; ++colx) {
            for (int a = 0; a < 8; ++a)
                for (int c = 0; c < 4; ++c) {
                    cplx s = Uv[a][c];
                    if (colx >= 0 && (colx % 4) == c) s += I * eps * C[a * 8 + colx / 4];
                    Ucv[a][c] = s;
                }
            surface_residual(P, &B, el_h[e], npt, xi, ws, nr, chi, Ucv, (const double(*)[3])U0v, Rv);
            for (int s = 0; s < nm; ++s)
                for (int c = 0; c < 4; ++c) {
                    cplx v = 0;
                    for (int a = 0; a < 8; ++a) v += C[a * 8 + s] * Rv[a][c];
                    if (colx < 0) Rm[s * 4 + c] = creal(v);
                    else Jm[(s * 4 + c) * nd + colx] = cimag(v) / eps;
                }
        }
        free(chi);
        for (int r = 0; r < nd; ++r) {
            int64_t grow = 4 * (int64_t)ms[r / 4] + (r % 4);
            if (resid) resid[grow] += Rm[r];
            if (!vals) continue;
            for (int c = 0; c < nd; ++c) {
                int32_t gcol = 4 * ms[c / 4] + (c % 4);
                int64_t kk = csr_find(row_ptr, col, grow, gcol);
                if (kk < 0) return -(k + 1);
                vals[kk] += Jm[r * nd + c];
            }
        }
    }
    return 0;
}

/* Single-element entry for tests: residual and Jacobian in master space. */
void or_element(const or_params *P, double h, int npt, const double *xi, const double *w, int nm,
                const double *C, const double *Um, const double *U0m, double *Rm, double *Jm) {
    element_assemble(P, h, npt, xi, w, nm, C, Um, U0m, Rm, Jm);
}

/* Frozen stabilisation parameters at points, for tests. out: npt x 3 */
void or_taus(const or_params *P, double h, int npt, const double *xi, const double *Uv,
             const double *U0v, double *out) {
    taus *t = (taus *)malloc(sizeof(taus) * (npt > 0 ? npt : 1));
    element_taus(P, h, npt, xi, (const double(*)[4])Uv, (const double(*)[3])U0v, t);
    for (int q = 0; q < npt; ++q) {
        out[3 * q] = t[q].tauM; out[3 * q + 1] = t[q].tauC; out[3 * q + 2] = t[q].taubar;
    }
    free(t);
}

/* ------------------------------------------------------------------------ */
/* Exact orientation predicates by floating-point expansion arithmetic       */
/* (Shewchuk, "Adaptive precision floating-point arithmetic and fast robust  */
/* geometric predicates", 1997). Expansions are stored least significant     */
/* component first, nonoverlapping, with zero components eliminated.         */
/* ------------------------------------------------------------------------ */

static inline void two_sum(double a, double b, double *x, double *y) {
    double s = a + b;
    double bv = s - a;
    double av = s - bv;
    *x = s;
    *y = (a - av) + (b - bv);
}

static inline void two_prod(double a, double b, double *x, double *y) {
    double p = a * b;
    *x = p;
    *y = fma(a, b, -p); /* exact rounding error of the product */
}

/* h = e + b (GROW-EXPANSION with zero elimination); returns length */
static int grow_expansion(int elen, const double *e, double b, double *h) {
    double q = b, hh;
    int hn = 0;
    for (int i = 0; i < elen; ++i) {
        two_sum(q, e[i], &q, &hh);
        if (hh != 0.0) h[hn++] = hh;
    }
    if (q != 0.0 || hn == 0) h[hn++] = q;
    return hn;
}

/* h = e + f, by repeated growth (EXPANSION-SUM); h may not alias e or f */
static int expansion_sum(int elen, const double *e, int flen, const double *f, double *h) {
    double tmp[2][256];
    int n = elen;
    const double *cur = e;
    int which = 0;
    for (int i = 0; i < flen; ++i) {
        n = grow_expansion(n, cur, f[i], tmp[which]);
        cur = tmp[which];
        which ^= 1;
    }
    memcpy(h, cur, sizeof(double) * n);
    return n;
}

/* h = b * e (SCALE-EXPANSION with zero elimination) */
static int scale_expansion(int elen, const double *e, double b, double *h) {
    double q, hh, p1, p0, sum;
    int hn = 0;
    two_prod(e[0], b, &q, &hh);
    if (hh != 0.0) h[hn++] = hh;
    for (int i = 1; i < elen; ++i) {
        two_prod(e[i], b, &p1, &p0);
        two_sum(q, p0, &sum, &hh);
        if (hh != 0.0) h[hn++] = hh;
        two_sum(p1, sum, &q, &hh);
        if (hh != 0.0) h[hn++] = hh;
    }
    if (q != 0.0 || hn == 0) h[hn++] = q;
    return hn;
}

/* h = e * f */
static int mult_expansion(int elen, const double *e, int flen, const double *f, double *h) {
    double part[256], acc[256], tmp[256];
    int an = 1;
    acc[0] = 0.0;
    for (int i = 0; i < flen; ++i) {
        int pn = scale_expansion(elen, e, f[i], part);
        an = expansion_sum(an, acc, pn, part, tmp);
        memcpy(acc, tmp, sizeof(double) * an);
    }
    memcpy(h, acc, sizeof(double) * an);
    return an;
}

static int negate(int n, const double *e, double *h) {
    for (int i = 0; i < n; ++i) h[i] = -e[i];
    return n;
}

static int exp_sign(int n, const double *e) {
    for (int i = n - 1; i >= 0; --i) {
        if (e[i] > 0) return 1;
        if (e[i] < 0) return -1;
    }
    return 0;
}

static int two_diff_exp(double a, double b, double *h) {
    double x, y;
    two_sum(a, -b, &x, &y);
    int n = 0;
    if (y != 0.0) h[n++] = y;
    if (x != 0.0 || n == 0) h[n++] = x;
    return n;
}

/* sign of det [a-d; b-d; c-d], exact */
int or_orient3d(const double *a, const double *b, const double *c, const double *d) {
    double ad[3][2], bd[3][2], cd[3][2];
    int an[3], bn[3], cn[3];
    for (int k = 0; k < 3; ++k) {
        an[k] = two_diff_exp(a[k], d[k], ad[k]);
        bn[k] = two_diff_exp(b[k], d[k], bd[k]);
        cn[k] = two_diff_exp(c[k], d[k], cd[k]);
    }
    /* det = ax (by cz - bz cy) + bx (cy az - cz ay) + cx (ay bz - az by) */
    double t1[16], t2[16], t3[16], m[32], s[192], acc[192], tmp[192];
    int n1, n2, nmn, ns, na = 1;
    acc[0] = 0.0;
    const double *X[3][2] = {{ad[0], bd[0]}, {bd[0], cd[0]}, {cd[0], ad[0]}};
    (void)X;
    /* term 1 */
    n1 = mult_expansion(bn[1], bd[1], cn[2], cd[2], t1);
    n2 = mult_expansion(bn[2], bd[2], cn[1], cd[1], t2);
    n2 = negate(n2, t2, t3);
    nmn = expansion_sum(n1, t1, n2, t3, m);
    ns = mult_expansion(nmn, m, an[0], ad[0], s);
    na = expansion_sum(na, acc, ns, s, tmp); memcpy(acc, tmp, sizeof(double) * na);
    /* term 2 */
    n1 = mult_expansion(cn[1], cd[1], an[2], ad[2], t1);
    n2 = mult_expansion(cn[2], cd[2], an[1], ad[1], t2);
    n2 = negate(n2, t2, t3);
    nmn = expansion_sum(n1, t1, n2, t3, m);
    ns = mult_expansion(nmn, m, bn[0], bd[0], s);
    na = expansion_sum(na, acc, ns, s, tmp); memcpy(acc, tmp, sizeof(double) * na);
    /* term 3 */
    n1 = mult_expansion(an[1], ad[1], bn[2], bd[2], t1);
    n2 = mult_expansion(an[2], ad[2], bn[1], bd[1], t2);
    n2 = negate(n2, t2, t3);
    nmn = expansion_sum(n1, t1, n2, t3, m);
    ns = mult_expansion(nmn, m, cn[0], cd[0], s);
    na = expansion_sum(na, acc, ns, s, tmp); memcpy(acc, tmp, sizeof(double) * na);
    return exp_sign(na, acc);
}

/* sign of det [a-c; b-c] in the plane of coordinates (i, j), exact */
int or_orient2d(const double *a, const double *b, const double *c, int i, int j) {
    double ac0[2], ac1[2], bc0[2], bc1[2], t1[8], t2[8], t3[8], r[16];
    int n0 = two_diff_exp(a[i], c[i], ac0), n1 = two_diff_exp(a[j], c[j], ac1);
    int m0 = two_diff_exp(b[i], c[i], bc0), m1 = two_diff_exp(b[j], c[j], bc1);
    int p = mult_expansion(n0, ac0, m1, bc1, t1);
    int q = mult_expansion(n1, ac1, m0, bc0, t2);
    q = negate(q, t2, t3);
    int nr = expansion_sum(p, t1, q, t3, r);
    return exp_sign(nr, r);
}

/* ------------------------------------------------------------------------ */
/* Exact point-in-polyhedron: parity of segment crossings                    */
/* ------------------------------------------------------------------------ */

/* Coplanar P in the closed triangle abc? (P already known to lie in its plane) */
static int coplanar_inside(const double *P, const double *a, const double *b, const double *c) {
    static const int pl[3][2] = {{0, 1}, {1, 2}, {0, 2}};
    for (int k = 0; k < 3; ++k) {
        int i = pl[k][0], j = pl[k][1];
        int s = or_orient2d(a, b, c, i, j);
        if (s == 0) continue; /* projection degenerate, try another plane */
        int s1 = or_orient2d(a, b, P, i, j), s2 = or_orient2d(b, c, P, i, j),
            s3 = or_orient2d(c, a, P, i, j);
        return (s1 * s >= 0) && (s2 * s >= 0) && (s3 * s >= 0);
    }
    return 0; /* triangle with zero area: contains nothing */
}

/* Segment P->Q against triangle abc.
 * 0: no crossing; 1: proper crossing; 2: degenerate (through an edge, a vertex,
 * or Q on the plane); 3: P lies on the closed triangle. */
int or_seg_tri(const double *P, const double *Q, const double *a, const double *b,
               const double *c) {
    int oP = or_orient3d(a, b, c, P);
    if (oP == 0) return coplanar_inside(P, a, b, c) ? 3 : 0;
    int oQ = or_orient3d(a, b, c, Q);
    if (oQ == 0) return 2;
    if (oP == oQ) return 0;
    int e1 = or_orient3d(P, Q, a, b), e2 = or_orient3d(P, Q, b, c), e3 = or_orient3d(P, Q, c, a);
    int pos = (e1 > 0) + (e2 > 0) + (e3 > 0), neg = (e1 < 0) + (e2 < 0) + (e3 < 0);
    if (pos == 3 || neg == 3) return 1;
    if (pos > 0 && neg > 0) return 0;
    return 2;
}

typedef struct {
    int64_t n_tri;
    const double *v;     /* 3 * n_vert */
    const int32_t *tri;  /* 3 * n_tri */
    double lo[3], hi[3]; /* bounding box of the vertices */
} or_surface;

static void surf_bbox(or_surface *S, int64_t n_vert) {
    for (int k = 0; k < 3; ++k) { S->lo[k] = INFINITY; S->hi[k] = -INFINITY; }
    for (int64_t i = 0; i < n_vert; ++i)
        for (int k = 0; k < 3; ++k) {
            double x = S->v[3 * i + k];
            if (x < S->lo[k]) S->lo[k] = x;
            if (x > S->hi[k]) S->hi[k] = x;
        }
}

/* label: 1 IN (solid, or on the surface), 0 OUT (fluid).
 * Far points: along +x, -x, +y, -y, +z, -z, then four oblique directions; the
 * first direction without a degenerate crossing decides. A point on the
 * surface is IN. *ndeg counts directions abandoned for degeneracy. */
static int label_point(const or_surface *S, const double *P, int64_t *ndeg) {
    for (int k = 0; k < 3; ++k)
        if (P[k] < S->lo[k] || P[k] > S->hi[k]) return 0;
    static const double dirs[10][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1},
                                       {0, 0, -1}, {0.8, 0.36, 0.48}, {-0.48, 0.8, 0.36},
                                       {0.36, -0.48, 0.8}, {-0.6, -0.64, -0.48}};
    double span = 0;
    for (int k = 0; k < 3; ++k) span += S->hi[k] - S->lo[k];
    const double L = 2.0 * span + 1.0;
    for (int d = 0; d < 10; ++d) {
        double Q[3];
        for (int k = 0; k < 3; ++k) Q[k] = P[k] + L * dirs[d][k];
        if (d < 6) { /* axis ray: leave the box along the axis exactly */
            int ax = d / 2;
            for (int k = 0; k < 3; ++k) Q[k] = P[k];
            Q[ax] = (d % 2 == 0) ? S->hi[ax] + 1.0 : S->lo[ax] - 1.0;
        }
        int cnt = 0, deg = 0;
        for (int64_t t = 0; t < S->n_tri; ++t) {
            const double *a = S->v + 3 * S->tri[3 * t], *b = S->v + 3 * S->tri[3 * t + 1],
                         *c = S->v + 3 * S->tri[3 * t + 2];
            /* exact reject: the segment's bounding box misses the triangle's */
            int miss = 0;
            for (int k = 0; k < 3 && !miss; ++k) {
                double smin = P[k] < Q[k] ? P[k] : Q[k], smax = P[k] < Q[k] ? Q[k] : P[k];
                double tmin = fmin(a[k], fmin(b[k], c[k])), tmax = fmax(a[k], fmax(b[k], c[k]));
                if (tmax < smin || tmin > smax) miss = 1;
            }
            if (miss) continue;
            int r = or_seg_tri(P, Q, a, b, c);
            if (r == 3) return 1;
            if (r == 2) deg = 1;
            else cnt += r;
        }
        if (!deg) return cnt & 1;
        if (ndeg) ++*ndeg;
    }
    return 1; /* every direction degenerate: treated as a point of the surface */
}

/* Labels of n points (xyz interleaved). Returns the number of degenerate
 * directions encountered. */
int64_t or_label_points(int64_t n_vert, const double *verts, int64_t n_tri, const int32_t *tris,
                        int64_t n, const double *xyz, uint8_t *labels) {
    or_surface S = {n_tri, verts, tris, {0}, {0}};
    surf_bbox(&S, n_vert);
    int64_t ndeg = 0;
    for (int64_t i = 0; i < n; ++i) labels[i] = (uint8_t)label_point(&S, xyz + 3 * i, &ndeg);
    return ndeg;
}

/* ------------------------------------------------------------------------ */
/* Point coordinates, identical on every implementation:                     */
/*   x = origin + root_len * ((A + B*g) * 2^-F)                              */
/* with integers A, B (fine-grid units, B a power of two), g in {0, g-, g+}, */
/* evaluated in this order without contraction.                              */
/* ------------------------------------------------------------------------ */

static const double G_MINUS = 0x1.b0cb174df99c7p-3; /* (1 - 1/sqrt 3) / 2, correctly rounded */
static const double G_PLUS = 0x1.93cd3a2c8198ep-1;  /* (1 + 1/sqrt 3) / 2, correctly rounded */

static double coord(double origin, double root_len, int F, int64_t A, int64_t B, double g) {
    double t1 = (double)B * g;
    double t2 = (double)A + t1;
    double t3 = ldexp(t2, -F);
    double t4 = root_len * t3;
    return origin + t4;
}

/* ------------------------------------------------------------------------ */
/* Adaptive quadrature of INTERCEPTED elements                               */
/* ------------------------------------------------------------------------ */

typedef struct {
    const or_surface *S;
    const double *origin;
    double root_len;
    int F;       /* max_level + depth */
    int depth;   /* maximum split level D */
    /* outputs */
    int64_t cap, n;
    int64_t *el;     /* element index */
    int32_t *key;    /* path digits (3 bits per level, level 1 first), then GP */
    uint8_t *lvl;    /* sub-cell level of the point (weight (h/2^(lvl+1))^3) */
    double *xyz;     /* coordinates */
    int64_t nlabel;  /* points classified */
    int64_t ndeg;
} subq_ctx;

static void emit(subq_ctx *Q, int64_t e, int32_t key, int l, const double *x) {
    if (Q->n < Q->cap) {
        Q->el[Q->n] = e; Q->key[Q->n] = key; Q->lvl[Q->n] = (uint8_t)l;
        memcpy(Q->xyz + 3 * Q->n, x, sizeof(double) * 3);
    }
    Q->n++;
}

/* key layout: digit of level k (1..D) at bits [3*(D-k+1)+3 ..); the GP index
 * in the three bits right after the last path digit, so that sorting keys
 * reproduces the depth-first order. */
static int32_t key_with(int32_t path, int l, int D, int gp) {
    /* path holds digits of levels 1..l, level 1 most significant, in 3 l bits */
    int32_t k = path;
    k = (k << 3) | gp;               /* 3 (l+1) bits */
    return k << (3 * (D - l));       /* pad to 3 (D+1) bits */
}

static void subcell(subq_ctx *Q, int64_t e, const int64_t A[3], int64_t B, int l, int32_t path) {
    double x[8][3];
    int lab[8], nin = 0;
    for (int g = 0; g < 8; ++g) {
        for (int k = 0; k < 3; ++k) {
            double gg = ((g >> k) & 1) ? G_PLUS : G_MINUS;
            x[g][k] = coord(Q->origin[k], Q->root_len, Q->F, A[k], B, gg);
        }
        lab[g] = label_point(Q->S, x[g], &Q->ndeg);
        nin += lab[g];
        Q->nlabel++;
    }
    if (l == Q->depth || nin == 0) {
        for (int g = 0; g < 8; ++g)
            if (!lab[g]) emit(Q, e, key_with(path, l, Q->depth, g), l, x[g]);
        return;
    }
    if (nin == 8) return;
    for (int c = 0; c < 8; ++c) {
        int64_t Ac[3] = {A[0] + ((c & 1) ? B / 2 : 0), A[1] + ((c & 2) ? B / 2 : 0),
                         A[2] + ((c & 4) ? B / 2 : 0)};
        subcell(Q, e, Ac, B / 2, l + 1, (path << 3) | c);
    }
}

/* Sub-cell quadrature points of the given INTERCEPTED elements, depth-first,
 * children in Morton order, Gauss points x fastest; only OUT points are kept.
 * Level 0 (the element) is always split unless depth == 0. Returns the number
 * of kept points (arrays are filled up to cap). */
int64_t or_subquad(int64_t n_vert, const double *verts, int64_t n_tri, const int32_t *tris,
                   const double *origin, double root_len, int max_level, int depth,
                   int64_t n_el, const int64_t *el_idx, const int32_t *ax, const int32_t *ay,
                   const int32_t *az, const uint8_t *level, int64_t cap, int64_t *out_el,
                   int32_t *out_key, uint8_t *out_lvl, double *out_xyz, int64_t *stats) {
    or_surface S = {n_tri, verts, tris, {0}, {0}};
    surf_bbox(&S, n_vert);
    subq_ctx Q = {&S, origin, root_len, max_level + depth, depth, cap, 0,
                  out_el, out_key, out_lvl, out_xyz, 0, 0};
    for (int64_t i = 0; i < n_el; ++i) {
        int64_t e = el_idx[i];
        int64_t B = (int64_t)1 << (max_level - level[e] + depth);
        int64_t A[3] = {(int64_t)ax[e] << depth, (int64_t)ay[e] << depth, (int64_t)az[e] << depth};
        if (depth == 0) {
            subcell(&Q, e, A, B, 0, 0);
        } else {
            for (int c = 0; c < 8; ++c) {
                int64_t Ac[3] = {A[0] + ((c & 1) ? B / 2 : 0), A[1] + ((c & 2) ? B / 2 : 0),
                                 A[2] + ((c & 4) ? B / 2 : 0)};
                subcell(&Q, e, Ac, B / 2, 1, c);
            }
        }
    }
    if (stats) { stats[0] = Q.nlabel; stats[1] = Q.ndeg; }
    return Q.n;
}

/* Coordinates of points given by fine-grid integers, for tests. */
void or_coords(const double *origin, double root_len, int F, int64_t n, const int64_t *A,
               const int64_t *B, const int8_t *gsel, double *out) {
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) {
            int s = gsel[3 * i + k];
            double g = s == 0 ? 0.0 : (s < 0 ? G_MINUS : G_PLUS);
            out[3 * i + k] = coord(origin[k], root_len, F, A[3 * i + k], B[i], g);
        }
}

/* ------------------------------------------------------------------------ */
/* Unsigned distance to a triangle set (closest point by Voronoi regions of  */
/* the triangle: vertices, edges, face), brute force over all triangles.     */
/* ------------------------------------------------------------------------ */

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static double tri_dist2(const double *p, const double *a, const double *b, const double *c) {
    double ab[3], ac[3], ap[3], q[3];
    for (int k = 0; k < 3; ++k) { ab[k] = b[k] - a[k]; ac[k] = c[k] - a[k]; ap[k] = p[k] - a[k]; }
    double d1 = dot3(ab, ap), d2 = dot3(ac, ap);
    if (d1 <= 0 && d2 <= 0) { memcpy(q, a, sizeof q); goto done; }        /* vertex a */
    double bp[3];
    for (int k = 0; k < 3; ++k) bp[k] = p[k] - b[k];
    double d3 = dot3(ab, bp), d4 = dot3(ac, bp);
    if (d3 >= 0 && d4 <= d3) { memcpy(q, b, sizeof q); goto done; }      /* vertex b */
    double vc = d1 * d4 - d3 * d2;
    if (vc <= 0 && d1 >= 0 && d3 <= 0) {                                  /* edge ab */
        double v = d1 / (d1 - d3);
        for (int k = 0; k < 3; ++k) q[k] = a[k] + v * ab[k];
        goto done;
    }
    double cp[3];
    for (int k = 0; k < 3; ++k) cp[k] = p[k] - c[k];
    double d5 = dot3(ab, cp), d6 = dot3(ac, cp);
    if (d6 >= 0 && d5 <= d6) { memcpy(q, c, sizeof q); goto done; }      /* vertex c */
    double vb = d5 * d2 - d1 * d6;
    if (vb <= 0 && d2 >= 0 && d6 <= 0) {                                  /* edge ac */
        double w = d2 / (d2 - d6);
        for (int k = 0; k < 3; ++k) q[k] = a[k] + w * ac[k];
        goto done;
    }
    double va = d3 * d6 - d5 * d4;
    if (va <= 0 && (d4 - d3) >= 0 && (d5 - d6) >= 0) {                   /* edge bc */
        double w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
        for (int k = 0; k < 3; ++k) q[k] = b[k] + w * (c[k] - b[k]);
        goto done;
    }
    {                                                                     /* face */
        double den = 1.0 / (va + vb + vc);
        double v = vb * den, w = vc * den;
        for (int k = 0; k < 3; ++k) q[k] = a[k] + ab[k] * v + ac[k] * w;
    }
done:;
    double d[3] = {p[0] - q[0], p[1] - q[1], p[2] - q[2]};
    return dot3(d, d);
}

void or_unsigned_dist(int64_t n_tri, const double *verts, const int32_t *tris, int64_t n,
                      const double *xyz, double *out) {
    for (int64_t i = 0; i < n; ++i) {
        double best = INFINITY;
        for (int64_t t = 0; t < n_tri; ++t) {
            double d = tri_dist2(xyz + 3 * i, verts + 3 * tris[3 * t], verts + 3 * tris[3 * t + 1],
                                 verts + 3 * tris[3 * t + 2]);
            if (d < best) best = d;
        }
        out[i] = sqrt(best);
    }
}

/* Residual (master space) at the state Ue with the stabilisation parameters
 * frozen at the state Ub; for finite-difference checks of the Jacobian. */
void or_element_frozen(const or_params *P, double h, int npt, const double *xi, const double *w,
                       int nm, const double *C, const double *Ub, const double *Ue,
                       const double *U0m, double *Rm) {
    double Ubv[8][4], U0v[8][3];
    cplx Uev[8][4], Rv[8][4];
    for (int a = 0; a < 8; ++a) {
        for (int c = 0; c < 4; ++c) {
            double sb = 0, se = 0;
            for (int t = 0; t < nm; ++t) {
                sb += C[a * nm + t] * Ub[t * 4 + c];
                se += C[a * nm + t] * Ue[t * 4 + c];
            }
            Ubv[a][c] = sb;
            Uev[a][c] = se;
        }
        for (int c = 0; c < 3; ++c) {
            double s = 0;
            for (int t = 0; t < nm; ++t) s += C[a * nm + t] * U0m[t * 3 + c];
            U0v[a][c] = s;
        }
    }
    taus *tau = (taus *)malloc(sizeof(taus) * (npt > 0 ? npt : 1));
    element_taus(P, h, npt, xi, (const double(*)[4])Ubv, (const double(*)[3])U0v, tau);
    element_residual(P, h, npt, xi, w, tau, Uev, (const double(*)[3])U0v, Rv);
    for (int s = 0; s < nm; ++s)
        for (int c = 0; c < 4; ++c) {
            cplx v = 0;
            for (int a = 0; a < 8; ++a) v += C[a * nm + s] * Rv[a][c];
            Rm[s * 4 + c] = creal(v);
        }
    free(tau);
}

/* ------------------------------------------------------------------------ */
/* Triquadratic (Q2, 27-node) elements on a uniform octree                   */
/*                                                                           */
/* The paper's matrix-assembly comparison (Table of matrix assembly times)   */
/* runs linear and quadratic bases on a uniform mesh; App. A tabulates the   */
/* basis values and gradients at the (bf+1)^d Gauss points. Node a of an     */
/* element is (a % 3, a / 3 % 3, a / 9) on the reference grid {-1, 0, 1}^3   */
/* (x fastest); the 1D basis on [-1, 1] is the Lagrange quadratic of the     */
/* nodes -1, 0, 1. The integrand is the same VMS residual as above (second   */
/* derivatives dropped from the strong residual, G = (2/h)^2 I), integrated  */
/* with the 3-point Gauss rule per axis; the Jacobian by complex step with   */
/* the stabilisation parameters frozen. No hanging nodes (all leaves on one  */
/* level), so nodes are the element nodes themselves.                        */
/* ------------------------------------------------------------------------ */

#define Q2_NB 27

static void q2_basis_1d(double x, double f[3], double g[3]) {
    f[0] = 0.5 * x * (x - 1.0);
    f[1] = 1.0 - x * x;
    f[2] = 0.5 * x * (x + 1.0);
    g[0] = x - 0.5;
    g[1] = -2.0 * x;
    g[2] = x + 0.5;
}

static void q2_basis(const double xi[3], double h, double N[Q2_NB], double dN[Q2_NB][3]) {
    double f[3][3], g[3][3];
    for (int k = 0; k < 3; ++k) q2_basis_1d(xi[k], f[k], g[k]);
    const double s = 2.0 / h;
    for (int a = 0; a < Q2_NB; ++a) {
        const int i = a % 3, j = (a / 3) % 3, l = a / 9;
        N[a] = f[0][i] * f[1][j] * f[2][l];
        dN[a][0] = s * g[0][i] * f[1][j] * f[2][l];
        dN[a][1] = s * f[0][i] * g[1][j] * f[2][l];
        dN[a][2] = s * f[0][i] * f[1][j] * g[2][l];
    }
}

/* the same integrand as element_residual, over the 27 nodes */
static void q2_residual(const or_params *P, double h, int npt, const double *xi, const double *w,
                        const taus *tau, cplx Uv[Q2_NB][4], const double U0v[Q2_NB][3],
                        cplx Rv[Q2_NB][4]) {
    const double rho = P->rho, mu = P->mu, dt = P->dt, th = P->theta;
    const int m = P->term_mask;
    for (int a = 0; a < Q2_NB; ++a)
        for (int c = 0; c < 4; ++c) Rv[a][c] = 0;
    for (int q = 0; q < npt; ++q) {
        double N[Q2_NB], dN[Q2_NB][3];
        q2_basis(xi + 3 * q, h, N, dN);
        const double W = w[q];
        cplx ut[3] = {0, 0, 0}, gu[3][3] = {{0}}, at[3] = {0, 0, 0}, p = 0, gp[3] = {0, 0, 0};
        for (int a = 0; a < Q2_NB; ++a) {
            for (int i = 0; i < 3; ++i) {
                cplx uth = th * Uv[a][i] + (1.0 - th) * U0v[a][i];
                ut[i] += N[a] * uth;
                at[i] += N[a] * (Uv[a][i] - U0v[a][i]) / dt;
                for (int j = 0; j < 3; ++j) gu[i][j] += dN[a][j] * uth;
            }
            p += N[a] * Uv[a][3];
            for (int j = 0; j < 3; ++j) gp[j] += dN[a][j] * Uv[a][3];
        }
        cplx rM[3], rC = gu[0][0] + gu[1][1] + gu[2][2];
        for (int i = 0; i < 3; ++i) {
            cplx conv = ut[0] * gu[i][0] + ut[1] * gu[i][1] + ut[2] * gu[i][2];
            rM[i] = rho * (at[i] + conv) + gp[i];
        }
        cplx up[3];
        for (int i = 0; i < 3; ++i) up[i] = -tau[q].tauM * rM[i];
        cplx pp = -rho * tau[q].tauC * rC;
        const double tb = tau[q].taubar;
        for (int a = 0; a < Q2_NB; ++a) {
            cplx u_dot_gradNa = ut[0] * dN[a][0] + ut[1] * dN[a][1] + ut[2] * dN[a][2];
            cplx up_dot_gradNa = up[0] * dN[a][0] + up[1] * dN[a][1] + up[2] * dN[a][2];
            for (int i = 0; i < 3; ++i) {
                cplx r = 0;
                cplx conv_i = ut[0] * gu[i][0] + ut[1] * gu[i][1] + ut[2] * gu[i][2];
                cplx upgu_i = up[0] * gu[i][0] + up[1] * gu[i][1] + up[2] * gu[i][2];
                if (m & (1 << 0)) r += N[a] * rho * at[i];
                if (m & (1 << 1)) r += N[a] * rho * conv_i;
                if (m & (1 << 2)) {
                    cplx v = 0;
                    for (int j = 0; j < 3; ++j) v += dN[a][j] * (gu[i][j] + gu[j][i]);
                    r += mu * v;
                }
                if (m & (1 << 3)) r += -p * dN[a][i];
                if (m & (1 << 5)) r += -u_dot_gradNa * up[i];
                if (m & (1 << 6)) r += -pp * dN[a][i];
                if (m & (1 << 7)) r += N[a] * upgu_i;
                if (m & (1 << 8)) r += -(1.0 / rho) * up_dot_gradNa * up[i];
                if (m & (1 << 9)) r += up_dot_gradNa * tb * upgu_i;
                Rv[a][i] += W * r;
            }
            cplx rc = 0;
            if (m & (1 << 4)) rc += N[a] * rC;
            if (m & (1 << 5)) rc += -(1.0 / rho) * up_dot_gradNa;
            Rv[a][3] += W * rc;
        }
    }
}

static void q2_taus(const or_params *P, double h, int npt, const double *xi,
                    const double Uv[Q2_NB][4], const double U0v[Q2_NB][3], taus *tau) {
    const double rho = P->rho, dt = P->dt, th = P->theta, nu = P->mu / P->rho;
    const double g = 4.0 / (h * h);
    for (int q = 0; q < npt; ++q) {
        double N[Q2_NB], dN[Q2_NB][3];
        q2_basis(xi + 3 * q, h, N, dN);
        double ut[3] = {0, 0, 0}, gu[3][3] = {{0}}, at[3] = {0, 0, 0}, gp[3] = {0, 0, 0};
        for (int a = 0; a < Q2_NB; ++a) {
            for (int i = 0; i < 3; ++i) {
                double uth = th * Uv[a][i] + (1.0 - th) * U0v[a][i];
                ut[i] += N[a] * uth;
                at[i] += N[a] * (Uv[a][i] - U0v[a][i]) / dt;
                for (int j = 0; j < 3; ++j) gu[i][j] += dN[a][j] * uth;
            }
            for (int j = 0; j < 3; ++j) gp[j] += dN[a][j] * Uv[a][3];
        }
        double uGu = g * (ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2]);
        double GG = 3.0 * g * g, trG = 3.0 * g;
        double tauM = 1.0 / sqrt(P->c_t / (dt * dt) + uGu + P->c_i * nu * nu * GG);
        double tauC = 1.0 / (tauM * trG);
        double up[3];
        for (int i = 0; i < 3; ++i) {
            double conv = ut[0] * gu[i][0] + ut[1] * gu[i][1] + ut[2] * gu[i][2];
            up[i] = -tauM * (rho * (at[i] + conv) + gp[i]);
        }
        double upGup = g * (up[0] * up[0] + up[1] * up[1] + up[2] * up[2]);
        tau[q].tauM = tauM;
        tau[q].tauC = tauC;
        tau[q].taubar = (upGup > 0.0) ? 1.0 / sqrt(upGup) : 0.0;
    }
}

/* One Q2 element: node values U (27 x 4), U0 (27 x 3); residual R (108) and
 * Jacobian J (108 x 108, row-major, dof 4 a + c) at the given points. */
void or_q2_element(const or_params *P, double h, int npt, const double *xi, const double *w,
                   const double *U, const double *U0, double *R, double *J) {
    double Uv[Q2_NB][4], U0v[Q2_NB][3];
    for (int a = 0; a < Q2_NB; ++a) {
        for (int c = 0; c < 4; ++c) Uv[a][c] = U[4 * a + c];
        for (int c = 0; c < 3; ++c) U0v[a][c] = U0[3 * a + c];
    }
    taus *tau = (taus *)malloc(sizeof(taus) * (npt > 0 ? npt : 1));
    q2_taus(P, h, npt, xi, (const double(*)[4])Uv, (const double(*)[3])U0v, tau);
    const double eps = 1e-30;
    cplx Ucv[Q2_NB][4], Rv[Q2_NB][4];
    for (int col = -1; col < 4 * Q2_NB; ++col) {
        for (int a = 0; a < Q2_NB; ++a)
            for (int c = 0; c < 4; ++c) Ucv[a][c] = Uv[a][c] + ((4 * a + c) == col ? I * eps : 0.0);
        q2_residual(P, h, npt, xi, w, tau, Ucv, (const double(*)[3])U0v, Rv);
        for (int a = 0; a < Q2_NB; ++a)
            for (int c = 0; c < 4; ++c) {
                if (col < 0) { if (R) R[4 * a + c] = creal(Rv[a][c]); }
                else if (J) J[(4 * a + c) * (4 * Q2_NB) + col] = cimag(Rv[a][c]) / eps;
            }
    }
    free(tau);
}

/* The real residual with the stabilisation parameters frozen at the state
 * Ub (for central differences of the frozen-tau Jacobian in tests). */
void or_q2_element_frozen(const or_params *P, double h, int npt, const double *xi, const double *w,
                          const double *Ub, const double *U, const double *U0, double *R) {
    double Bv[Q2_NB][4], U0v[Q2_NB][3];
    cplx Ucv[Q2_NB][4], Rv[Q2_NB][4];
    for (int a = 0; a < Q2_NB; ++a) {
        for (int c = 0; c < 4; ++c) { Bv[a][c] = Ub[4 * a + c]; Ucv[a][c] = U[4 * a + c]; }
        for (int c = 0; c < 3; ++c) U0v[a][c] = U0[3 * a + c];
    }
    taus *tau = (taus *)malloc(sizeof(taus) * (npt > 0 ? npt : 1));
    q2_taus(P, h, npt, xi, (const double(*)[4])Bv, (const double(*)[3])U0v, tau);
    q2_residual(P, h, npt, xi, w, tau, Ucv, (const double(*)[3])U0v, Rv);
    for (int a = 0; a < Q2_NB; ++a)
        for (int c = 0; c < 4; ++c) R[4 * a + c] = creal(Rv[a][c]);
    free(tau);
}

/* Global Q2 assembly: element e's nodes el_node[27 e ..] (global ids), size
 * el_h[e], the same npt points (xi, w scaled by the caller) in every element.
 * Outputs accumulated (+=) into the CSR of the node pairs. Returns 0 or
 * -(e+1) if an entry is missing from the pattern. */
int64_t or_q2_assemble(const or_params *P, int64_t n_el, const int32_t *el_node, const double *el_h,
                       int npt, const double *xi, const double *w_ref, const double *ux,
                       const double *uy, const double *uz, const double *pr, const double *ux0,
                       const double *uy0, const double *uz0, const int64_t *row_ptr,
                       const int32_t *col, double *vals, double *resid) {
    double U[4 * Q2_NB], U0[3 * Q2_NB], R[4 * Q2_NB];
    double *J = (double *)malloc(sizeof(double) * 16 * Q2_NB * Q2_NB);
    double *w = (double *)malloc(sizeof(double) * (npt > 0 ? npt : 1));
    for (int64_t e = 0; e < n_el; ++e) {
        const int32_t *nd = el_node + Q2_NB * e;
        const double d3 = (el_h[e] / 2.0) * (el_h[e] / 2.0) * (el_h[e] / 2.0);
        for (int q = 0; q < npt; ++q) w[q] = w_ref[q] * d3;
        for (int a = 0; a < Q2_NB; ++a) {
            const int32_t n = nd[a];
            U[4 * a] = ux[n]; U[4 * a + 1] = uy[n]; U[4 * a + 2] = uz[n]; U[4 * a + 3] = pr[n];
            U0[3 * a] = ux0[n]; U0[3 * a + 1] = uy0[n]; U0[3 * a + 2] = uz0[n];
        }
        or_q2_element(P, el_h[e], npt, xi, w, U, U0, R, vals ? J : NULL);
        for (int r = 0; r < 4 * Q2_NB; ++r) {
            const int64_t grow = 4 * (int64_t)nd[r / 4] + (r % 4);
            if (resid) resid[grow] += R[r];
            if (!vals) continue;
            for (int c = 0; c < 4 * Q2_NB; ++c) {
                const int32_t gcol = 4 * nd[c / 4] + (c % 4);
                const int64_t k = csr_find(row_ptr, col, grow, gcol);
                if (k < 0) { free(J); free(w); return -(e + 1); }
                vals[k] += J[r * 4 * Q2_NB + c];
            }
        }
    }
    free(J);
    free(w);
    return 0;
}

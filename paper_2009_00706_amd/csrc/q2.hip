// Triquadratic (Q2, 27-node) VMS element assembly of libvms (gfx950), FP64.
//
// The paper compares linear and quadratic bases in its matrix-assembly table
// (uniform 16^3 mesh) and tabulates the basis at the (bf+1)^d Gauss points
// (App. A): here 27 nodes, 3 x 3 x 3 Gauss points, element matrices of 108 x
// 108. The integrand is the trilinear kernel's (eq. (vms), (uprime), (pprime),
// taus frozen), with the same per-point factors and D blocks (vms_point.h).
//
// One workgroup of four waves per element:
//   phase 0  node ids and the 27 x 7 nodal fields to LDS;
//   phase 1  fields and gradients at the 27 points (tensor-product basis);
//   phase 2  per-point state (taus, u', p', residual coefficients, D factors);
//   phase 3  for each third of the points: the 16 D blocks of each point, then
//            wave i (test component i) contracts on v_mfma_f64_4x4x4 (four 4x4
//            blocks per instruction, block = trial component j):
//              stage 1  F^{ij}[k][b] = sum_l D^{ij}[k][l] B[l][b], per 4-column
//                       tile of b, lands in stage 2's second-operand layout;
//              stage 2  K^{ij}[a][b] += sum_k B[k][a] F^{ij}[k][b] over the
//                       7 x 7 tiles (rows and columns padded from 27 to 28);
//   phase 4  residual R[(a,i)] = sum_q sum_k B[k][a] r^i[k] on the VALU;
//   phase 5  the element matrix record, block-major (node pair, then i, j).
#include "kernels.h"
#include "vms_point.h"

namespace vmsk {

namespace {

constexpr double Q2_G = 0x1.8c97ef43f7248p-1;  // sqrt(3/5), correctly rounded
constexpr double Q2_W0 = 5.0 / 9.0, Q2_W1 = 8.0 / 9.0;
constexpr int NQP = NQ2 + 1;  // padded row of the per-point factors

// 1D quadratic Lagrange basis of the nodes -1, 0, 1 at Gauss point g (0..2):
// value of function i, and its xi-derivative
__device__ inline double q2f(int g, int i) {
    const double x = g == 0 ? -Q2_G : (g == 1 ? 0.0 : Q2_G);
    return i == 0 ? 0.5 * x * (x - 1.0) : (i == 1 ? 1.0 - x * x : 0.5 * x * (x + 1.0));
}
__device__ inline double q2g(int g, int i) {
    const double x = g == 0 ? -Q2_G : (g == 1 ? 0.0 : Q2_G);
    return i == 0 ? x - 0.5 : (i == 1 ? -2.0 * x : x + 0.5);
}

// B_q[d][a]: basis function a (d = 0) or its x/y/z derivative (d = 1..3, times
// s = 2/h) at Gauss point q; zero for the padding row a = 27
__device__ inline double q2basis(int q, int a, int d, double s) {
    if (a >= 27) return 0.0;
    const int qx = q % 3, qy = (q / 3) % 3, qz = q / 9;
    const int ax = a % 3, ay = (a / 3) % 3, az = a / 9;
    const double fx = d == 1 ? s * q2g(qx, ax) : q2f(qx, ax);
    const double fy = d == 2 ? s * q2g(qy, ay) : q2f(qy, ay);
    const double fz = d == 3 ? s * q2g(qz, az) : q2f(qz, az);
    return fx * fy * fz;
}

__device__ inline double q2w(int g) { return g == 1 ? Q2_W1 : Q2_W0; }

}  // namespace

__global__ __launch_bounds__(256) void k_q2(Q2Args A) {
    __shared__ int32_t sN[27];
    __shared__ double sU[27][8];
    __shared__ double sI[27][29];   // field f, entry d (value, gradient): 4 f + d
    __shared__ double sQ[27][NQP];
    __shared__ double sD[9][16][17];  // D blocks of a third of the points: [p][4 i + j][4 k + l]
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int64_t e = blockIdx.x;
    if (e >= A.n_el) return;
    const double h = A.h, s = 2.0 / h;

    // ---- phase 0
    if (t < 27) sN[t] = A.el_node[27 * e + t];
    __syncthreads();
    if (t < 189) sU[t / 7][t % 7] = A.f[t % 7][sN[t / 7]];
    __syncthreads();

    // ---- phase 1: 27 points x 7 fields x (value, gradient)
    for (int task = t; task < 27 * 28; task += 256) {
        const int q = task / 28, r = task % 28, f = r >> 2, d = r & 3;
        double v = 0.0;
        for (int a = 0; a < 27; ++a) v += q2basis(q, a, d, s) * sU[a][f];
        sI[q][r] = v;
    }
    __syncthreads();

    // ---- phase 2: per-point state (one thread per point)
    if (t < 27) {
        const int q = t;
        const double rho = A.rho, mu = A.mu, th = A.theta, idt = A.idt, irho = A.irho;
        const double g = s * s;  // G = g I
        const double W = q2w(q % 3) * q2w((q / 3) % 3) * q2w(q / 9) * (0.5 * h) * (0.5 * h) * (0.5 * h);
        const double *I = sI[q];
        double *Q = sQ[q];
        double ut[3], gu[3][3], up[3], rM[3];
        for (int c = 0; c < 3; ++c) {
            ut[c] = th * I[4 * c] + (1.0 - th) * I[4 * (4 + c)];
            for (int m = 0; m < 3; ++m) gu[c][m] = th * I[4 * c + 1 + m] + (1.0 - th) * I[4 * (4 + c) + 1 + m];
        }
        for (int c = 0; c < 3; ++c) {
            const double atc = (I[4 * c] - I[4 * (4 + c)]) * idt;
            const double conv = ut[0] * gu[c][0] + ut[1] * gu[c][1] + ut[2] * gu[c][2];
            rM[c] = rho * (atc + conv) + I[4 * 3 + 1 + c];
        }
        const double div = gu[0][0] + gu[1][1] + gu[2][2];
        const double s0 = A.tau_a + A.tau_b * g * g + g * (ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2]);
        const double tauM = rsq<double>(s0);
        const double tauC = (1.0 / (3.0 * g)) * s0 * tauM;  // 1 / (tau_M tr G)
        for (int c = 0; c < 3; ++c) up[c] = -tauM * rM[c];
        const double pp = -rho * tauC * div;
        const double upg = g * (up[0] * up[0] + up[1] * up[1] + up[2] * up[2]);
        const double tb = upg > 0.0 ? rsq<double>(upg) : 0.0;
        const double pr = I[4 * 3];
        Q[QW] = W;
        Q[QTM] = tauM;
        Q[QTC] = tauC;
        Q[QTB] = tb;
        for (int c = 0; c < 3; ++c) {
            const double atc = (I[4 * c] - I[4 * (4 + c)]) * idt;
            const double convc = ut[0] * gu[c][0] + ut[1] * gu[c][1] + ut[2] * gu[c][2];
            const double svc = up[0] * gu[c][0] + up[1] * gu[c][1] + up[2] * gu[c][2];
            Q[QUT + c] = ut[c];
            Q[QUP + c] = up[c];
            Q[QSV + c] = svc;
            for (int m = 0; m < 3; ++m) Q[QG + 3 * c + m] = gu[c][m];
            Q[QRC + 4 * c] = W * (rho * atc + rho * convc + svc);
            for (int k = 0; k < 3; ++k)
                Q[QRC + 4 * c + 1 + k] = W * (mu * (gu[c][k] + gu[k][c]) - (k == c ? pr + pp : 0.0) -
                                              ut[k] * up[c] - up[k] * up[c] * irho + tb * up[k] * svc);
        }
        Q[QRC + 12] = W * div;
        for (int k = 0; k < 3; ++k) Q[QRC + 13 + k] = -W * up[k] * irho;
        const double tr = tauM * rho, tbtr = tb * tauM * rho, tbt = tb * tauM, tir = tauM * irho;
        for (int c = 0; c < 3; ++c) {
            for (int m = 0; m < 3; ++m) {
                Q[QA + 3 * c + m] = (c == m ? idt : 0.0) + th * gu[c][m];
                double v = 0.0;
                for (int k = 0; k < 3; ++k) v += gu[c][k] * ((k == m ? idt : 0.0) + th * gu[k][m]);
                Q[QGA + 3 * c + m] = v;
            }
            const double svc = Q[QSV + c];
            Q[QY + c] = tr * ut[c] + tauM * up[c];
            Q[QX + c] = -tbtr * up[c];
            Q[QCP + c] = tauM * up[c] - tbtr * svc;
            Q[QYM + c] = tauM * ut[c] + tir * up[c];
            Q[QCM + c] = tir * up[c] - tbt * svc;
            Q[QXM + c] = -tbt * up[c];
        }
    }
    __syncthreads();

    // ---- phase 3: D blocks and the two contraction stages, a third of the points at a time
    // lane l: contraction index k = l / 16, block (trial component) j = (l / 4) % 4,
    // row / column n = l % 4; wave wv = test component i
    const int kk = lane >> 4, j4 = (lane >> 2) & 3, n4 = lane & 3, i = wv;
    double acc[7][7];
    for (int at = 0; at < 7; ++at)
        for (int bt = 0; bt < 7; ++bt) acc[at][bt] = 0.0;
    for (int c = 0; c < 3; ++c) {
        if (c > 0) __syncthreads();  // the previous third is done with sD
        if (t < 144) {
            const int p = t >> 4, ij = t & 15, bi = ij >> 2, bj = ij & 3;
            double D[4][4];
            if (bi < 3 && bj < 3) dblock_mv<double>(sQ[9 * c + p], bi, bj, A.rho, A.mu, A.theta, D);
            else dblock_simple<double>(sQ[9 * c + p], bi, bj, A.irho, A.theta, D);
            for (int k = 0; k < 4; ++k)
                for (int l = 0; l < 4; ++l) sD[p][ij][4 * k + l] = D[k][l];
        }
        __syncthreads();
        for (int p = 0; p < 9; ++p) {
            const int q = 9 * c + p;
            double Bt[7];  // B_q[k][4 t + n] (stage 1's second and stage 2's first operand)
            for (int tt = 0; tt < 7; ++tt) Bt[tt] = q2basis(q, 4 * tt + n4, kk, s);
            const double Dt = sD[p][4 * i + j4][4 * n4 + kk];  // D^{ij}[n][k]
            double E[7];
            for (int bt = 0; bt < 7; ++bt) E[bt] = __builtin_amdgcn_mfma_f64_4x4x4f64(Dt, Bt[bt], 0.0, 0, 0, 0);
            for (int at = 0; at < 7; ++at)
                for (int bt = 0; bt < 7; ++bt)
                    acc[at][bt] = __builtin_amdgcn_mfma_f64_4x4x4f64(Bt[at], E[bt], acc[at][bt], 0, 0, 0);
        }
    }

    // ---- phase 4: residual
    if (t < 108) {
        const int a = t >> 2, ic = t & 3;
        double r = 0.0;
        for (int q = 0; q < 27; ++q)
            for (int k = 0; k < 4; ++k) r += q2basis(q, a, k, s) * sQ[q][QRC + 4 * ic + k];
        A.rrec[108 * e + t] = r;
    }

    // ---- phase 5: record, entry ((27 a + b) 16 + 4 i + j)
    double *rec = A.em + (int64_t)e * (729 * 16);
    for (int at = 0; at < 7; ++at)
        for (int bt = 0; bt < 7; ++bt) {
            const int a = 4 * at + kk, b = 4 * bt + n4;
            if (a < 27 && b < 27) rec[(27 * a + b) * 16 + 4 * i + j4] = acc[at][bt];
        }
}

// residual of every node from the element records (its (element, node slot)
// entries in ascending order)
__global__ void k_q2_res_gather(const double *rrec, const int64_t *roff, const int32_t *rlist, int64_t n_nodes,
                                double *out) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= n_nodes) return;
    double r[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t c = roff[n]; c < roff[n + 1]; ++c) {
        const int64_t q = rlist[c];
        for (int k = 0; k < 4; ++k) r[k] += rrec[4 * q + k];
    }
    for (int k = 0; k < 4; ++k) out[4 * n + k] = r[k];
}

void launch_q2(hipStream_t s, const Q2Args &a) {
    if (a.n_el <= 0) return;
    hipLaunchKernelGGL(k_q2, dim3((unsigned)a.n_el), dim3(256), 0, s, a);
}

void launch_q2_res_gather(hipStream_t s, const double *rrec, const int64_t *roff, const int32_t *rlist,
                          int64_t n_nodes, double *out) {
    if (n_nodes <= 0) return;
    hipLaunchKernelGGL(k_q2_res_gather, dim3((unsigned)((n_nodes + 255) / 256)), dim3(256), 0, s, rrec, roff,
                       rlist, n_nodes, out);
}

}  // namespace vmsk

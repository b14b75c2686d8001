// Internal interface between the host API of libvms and its HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vmsk {

// Surface on the device. Triangles are packed as 9 doubles (a, b, c) plus an
// axis-aligned box (6 doubles: min xyz, max xyz). Rays along +x are served by
// a 2D grid of bins over (y, z); bin(v) = clamp(floor((v - v0) * inv), 0, n-1)
// is evaluated identically when bins are filled (host) and queried (device).
struct SurfDev {
    int32_t n_tri;
    int32_t nby, nbz;
    int32_t pad;
    const double *tv;    // [n_tri][9]
    const double *tbox;  // [n_tri][6]
    double lo[3], hi[3];
    double y0, z0, iny, inz;
    const int32_t *bin_off;  // [nby*nbz + 1]
    const int32_t *bin_tri;
};

struct GeoArgs {
    double origin[3];
    double root_len;
    int32_t max_level;
    int32_t depth;
};

// Exact labels of points given by integer coordinates at max-level resolution.
void launch_vertex_labels(hipStream_t s, const SurfDev &S, const GeoArgs &g, int64_t n,
                          const int32_t *ix, const int32_t *iy, const int32_t *iz, uint8_t *lab,
                          unsigned long long *ndeg);
// Exact labels of arbitrary points.
void launch_point_labels(hipStream_t s, const SurfDev &S, int64_t n, const double *px,
                         const double *py, const double *pz, uint8_t *lab,
                         unsigned long long *ndeg);
// Exact labels of the points whose index is listed (learned-filter fallback).
void launch_point_labels_list(hipStream_t s, const SurfDev &S, const int64_t *idx,
                              const unsigned long long *count, int64_t cap, const double *px,
                              const double *py, const double *pz, uint8_t *lab,
                              unsigned long long *ndeg);

// Learned in-out filter (signed-distance network) as the kernels see it.
// Parameters (float): W1 (64x64, out x in), b1, W2, b2, W3, b3, w4 (64), b4 (1).
struct Net {
    const float *theta;      // FP32 parameters (null: no network)
    const _Float16 *w16;     // FP16 copies of W1, W2, W3 (3 x 64 x 64)
    const float *B;          // 32 x 3 Fourier matrix
    float lo[3], inv[3];     // xh = 2 (x - lo) * inv - 1 with inv = 1 / (hi - lo)
    double blo[3], bhi[3];   // the box itself
};

// Per-cell margins over the network box (m == nullptr: the scalar margin)
struct MarginGrid {
    const float *m;
    int n[3];
    double lo[3], inv[3];  // cell of x along k: floor((x - lo) inv), clamped
};

// The network in front of the exact test of the sub-cell quadrature: used on
// the elements with at least min_bt background triangles.
struct LearnedArgs {
    Net net;
    MarginGrid grid;
    float margin;
    int32_t min_bt;
};

// Adaptive sub-cell quadrature of INTERCEPTED elements. pass 0 counts kept
// points per element into cnt; pass 1 writes the sorted entries
// (key << 2 | level) at off[i]. Per element i of the list: element id,
// anchor/level, corner labels, and background triangles bt_ids[bt_off[i] ..).
struct SubqArgs {
    int64_t n;
    const int32_t *el;
    const int32_t *ax, *ay, *az;
    const uint8_t *level;
    const uint8_t *corner_lab;  // [n][8]
    const int64_t *bt_off;
    const int32_t *bt_ids;
    int32_t *cnt;
    const int64_t *off;
    uint32_t *entries;
    unsigned long long *nlabel;
    unsigned long long *ndeg;
    unsigned int *flag;  // bit 0: a relabelled element changed its point count
    unsigned long long *nexact;  // pass 1: points labelled by the exact test (added to)
    LearnedArgs learned; // learned.net.theta null: exact labels only
    const int32_t *order;  // non-null: only the n_order elements order[..] of the list
    int64_t n_order;
    // certified normal-based filter (normal != 0, pass 1): per background
    // triangle of an element the local index (0..7) of its body among the
    // element's bodies, per element the mask of its bodies (0: filter off there)
    int32_t normal;
    const uint8_t *bt_lc;
    const uint8_t *nmask;
};
// wg_per_cu > 0: the relabel pass (pass 1) gets dynamic LDS so that at most
// that many workgroups share a CU
void launch_subquad(hipStream_t s, const SurfDev &S, const GeoArgs &g, const SubqArgs &a, int pass,
                    int wg_per_cu = 0);
// resident workgroups per CU of the exact relabel kernel
int subquad_per_cu();
// bad[e] = 1 when vertex corner[e] of triangle t2[e] lies strictly outside the
// plane of triangle t1[e] (exact orientation): the surface is not convex at
// that edge
void launch_edge_convex(hipStream_t s, const SurfDev &S, const int32_t *t1, const int32_t *t2,
                        const int8_t *corner, int64_t n, uint8_t *bad);
void launch_zero_u64(hipStream_t s, unsigned long long *c);

// Assembly.
struct AsmArgs {
    // element data (indexed by element id)
    const int32_t *masters;   // [E][8]
    const uint32_t *ccode;    // [E][4]
    const uint8_t *has_hang;  // [E]
    const uint8_t *level;     // [E]
    // work list
    int64_t n_items;
    const int32_t *items;     // element ids
    const int64_t *pt_off;    // SUB: first entry of the item's points
    const int32_t *pt_cnt;    // SUB: number of points
    const uint32_t *entries;  // SUB: key << 2 | level
    int32_t depth;
    // fields
    const double *f[7];       // ux uy uz p ux0 uy0 uz0
    // parameters: rho, mu, theta, the root edge, and derived by set_params:
    // 1/dt, 1/rho, 2/root_len and the two terms of
    // tau_M^-2 = c_t/dt^2 + c_i nu^2 G:G = tau_a + tau_b g^2 for G = g I, g = (2/h)^2
    double rho, mu, theta, root_len;
    double idt, irho, two_over_root, tau_a, tau_b;
    // outputs: element-matrix records (1024 entries per work item, record
    // slot0 + item) and residual records (32 doubles per work item at the
    // same record index: entry 4 a + i for master slot a, component i); the
    // CSR values and the residual are summed from them in a fixed order
    double *rrec;
    void *em;
    int64_t slot0;
    // atomic scatter (vals non-null): the element matrix is added straight
    // into the CSR values (double for FP64, else float) with hardware atomics
    // instead of being written as a record; entry (i, j) of slot pair (s, t)
    // goes to 16 nrow_ptr[m_s] + 4 el_kk[64 e + 8 s + t] + 4 i deg(m_s) + j
    void *vals;
    const int64_t *nrow_ptr;  // [n_nodes + 1] block rows
    const uint16_t *el_kk;    // [E][8][8] block column of m_t within row m_s
};
inline void set_params(AsmArgs &a, double rho, double mu, double dt, double theta, double c_t,
                       double c_i, double root_len) {
    const double nu = mu / rho;
    a.rho = rho;
    a.mu = mu;
    a.theta = theta;
    a.root_len = root_len;
    a.idt = 1.0 / dt;
    a.irho = 1.0 / rho;
    a.two_over_root = 2.0 / root_len;
    a.tau_a = c_t / (dt * dt);
    a.tau_b = 3.0 * c_i * nu * nu;
}
// wg_per_cu > 0 (sub-cell items only): dynamic LDS so that at most that many
// workgroups share a CU, leaving the rest of its waves to another stream's
// kernel
void launch_assemble_f64(hipStream_t s, const AsmArgs &a, bool sub, bool mat, int wg_per_cu = 0);

// one unit of the persistent batched assembly: items [first, first + count) of
// tree `tree`'s OUT-element list (sub = 0) or sub-cell work-item list (sub = 1)
struct BatchUnit {
    int32_t tree;
    int32_t sub;
    int64_t first;
    int32_t count;
    int32_t pad;
};
// one persistent launch of n_groups workgroups over all units, in list order;
// counter: a device counter (reset by the launch sequence)
void launch_assemble_batch(hipStream_t s, int precision, const AsmArgs *std_args,
                           const AsmArgs *sub_args, const BatchUnit *units, int64_t n_units,
                           unsigned long long *counter, int n_groups);
void launch_assemble_mixed(hipStream_t s, const AsmArgs &a, bool sub, bool mat, int fp16, int wg_per_cu = 0);
// resident workgroups per CU of the sub-cell item kernel of a precision form
// (0 FP64, 1 BF16x3, 2 FP16x2; with the matrix), from its registers and LDS
int sub_items_per_cu(int precision);
// dynamic LDS that holds a kernel to at most wg_per_cu resident workgroups per CU
size_t lds_for_cap(const void *kernel, int wg_per_cu);

// CSR values from element-matrix records (see k_gather). A block whose
// stride carries VS_LATE (a positive stride only) has records of sub-cell or
// surface items; skip_late leaves those blocks to launch_gather_list, so that
// the rest can be summed as soon as the OUT-element records exist.
constexpr int32_t VS_LATE = 1 << 30;
void launch_gather_f64(hipStream_t s, const double *em, const int64_t *cb_off, const int32_t *contrib,
                       const int64_t *vbase, const int32_t *vstride, int64_t nb, double *vals,
                       bool skip_late = false);
void launch_gather_f32(hipStream_t s, const float *em, const int64_t *cb_off, const int32_t *contrib,
                       const int64_t *vbase, const int32_t *vstride, int64_t nb, float *vals,
                       bool skip_late = false);
// the same for the n listed blocks only (list: DEVICE, block indices)
void launch_gather_list(hipStream_t s, bool fp64, const void *em, const int64_t *cb_off, const int32_t *contrib,
                        const int64_t *vbase, const int32_t *vstride, const int64_t *list, int64_t n,
                        void *vals);
void launch_fill_f64(hipStream_t s, double *p, int64_t n, double v);
void launch_fill_f32(hipStream_t s, float *p, int64_t n, float v);
// Triquadratic (27-node) elements of a uniform octree, FP64: element node
// lists, fields, the (uniform) element side and the parameters as in AsmArgs;
// outputs the element-matrix records ([E][27 x 27 node pairs][16]) and the
// residual records ([E][27][4]).
struct Q2Args {
    int64_t n_el;
    const int32_t *el_node;   // [E][27]
    const double *f[7];       // ux uy uz p ux0 uy0 uz0
    double h;
    double rho, mu, theta, idt, irho, tau_a, tau_b;
    double *em;
    double *rrec;
};
void launch_q2(hipStream_t s, const Q2Args &a);
void launch_q2_res_gather(hipStream_t s, const double *rrec, const int64_t *roff, const int32_t *rlist,
                          int64_t n_nodes, double *out);

// One tree's summation lists and outputs, for the batched gathers.
struct GatherTab {
    const void *em;           // element-matrix records (double or float)
    const int64_t *cb_off;
    const int32_t *contrib;
    const int64_t *vbase;
    const int32_t *vstride;
    void *vals;
    const double *rrec;
    const int64_t *roff;
    const int32_t *rlist;
    double *resid;            // null: no residual for this tree
};
// CSR values (identity blocks of inactive nodes included) and residuals of
// every tree: blk_prefix / node_prefix [n_trees + 1] are the trees' first
// blocks / nodes in the concatenation; n_blocks / n_nodes their totals
void launch_gather_batch(hipStream_t s, int precision, const GatherTab *tabs, const int64_t *blk_prefix,
                         int64_t n_blocks, const int64_t *node_prefix, int64_t n_nodes, int n_trees);
// rows of the listed nodes -> identity rows (diag_pos: block index of the
// diagonal in each node row), their residual entries (if resid) -> 0
void launch_dirichlet_rows_f64(hipStream_t s, double *vals, const int64_t *nrow_ptr, const int32_t *diag_pos,
                               const int32_t *nodes, int64_t n, double *resid);
void launch_dirichlet_rows_f32(hipStream_t s, float *vals, const int64_t *nrow_ptr, const int32_t *diag_pos,
                               const int32_t *nodes, int64_t n, double *resid);
// sum of squares, FP64, into out[0] (zeroed by the caller)
void launch_norm2(hipStream_t s, const double *v, int64_t n, double *out);
// Weak (Nitsche) boundary terms at surface points: items [0, n_items), item
// k = element items[k] with points [pt_off[k], pt_off[k+1]) (reference
// coordinates xi, area weights w, unit normals n of the fluid domain), tau_B
// per item; records at slot0 + k (block-major like the volume records)
struct SurfArgs {
    const int32_t *masters;
    const uint32_t *ccode;
    const uint8_t *has_hang;
    const uint8_t *level;
    int64_t n_items;
    const int32_t *items;
    const int64_t *pt_off;
    const double *xi, *w, *n, *tau;
    const double *f[7];
    double rho, mu, theta, root_len, g[3];
    double *rrec;  // residual records, as in AsmArgs
    void *em;
    int64_t slot0;
};
// mode 0: records (+ residual records if rrec), 1: residual records only, 2:
// Jacobian action along x into the residual records; fp64 selects FP64
// element-matrix records (else FP32)
void launch_surface(hipStream_t s, const SurfArgs &a, int mode, bool fp64, const double *x);
// Jacobian action along x: FP64 point work if fp64, else FP32; the residual
// records receive the element contributions to y
void launch_jacobian_action(hipStream_t s, const AsmArgs &a, bool sub, bool fp64, const double *x);
// residual (or Jacobian action) from the residual records: out[4 n + i] = sum,
// over node n's entries rlist[roff[n] .. roff[n + 1]) (8 record + slot,
// ascending), of rrec[32 record + 4 slot + i]; 0 for a node without entries
void launch_res_gather(hipStream_t s, const double *rrec, const int64_t *roff, const int32_t *rlist,
                       int64_t n_nodes, double *out);
// y[4 n + c] = x[4 n + c] for the listed nodes (identity rows)
void launch_copy_rows(hipStream_t s, const double *x, double *y, const int32_t *nodes, int64_t n);
// y = A x for the CSR of 4x4 node blocks: node row n has blocks
// [nrow_ptr[n], nrow_ptr[n + 1]) with node columns ncol[b]; its four dof rows
// are stored one after the other from 16 nrow_ptr[n], 4 deg entries each
void launch_bspmv_f64(hipStream_t s, const int64_t *nrow_ptr, const int32_t *ncol, const double *vals,
                      const double *x, double *y, int64_t n_nodes);
void launch_bspmv_f32(hipStream_t s, const int64_t *nrow_ptr, const int32_t *ncol, const float *vals,
                      const double *x, double *y, int64_t n_nodes);

// Krylov vector kernels (krylov.hip). dinv: 16 doubles per node, the inverse
// of the node's diagonal 4x4 block (diag_pos[n] = its block index in the node
// row); *bad is or-ed with 1 where a block is singular.
void launch_bjac_invert_f64(hipStream_t s, const double *vals, const int64_t *nrow_ptr,
                            const int32_t *diag_pos, int64_t n_nodes, double *dinv, int *bad);
void launch_bjac_invert_f32(hipStream_t s, const float *vals, const int64_t *nrow_ptr,
                            const int32_t *diag_pos, int64_t n_nodes, double *dinv, int *bad);
void launch_bjac_apply(hipStream_t s, const double *dinv, const double *x, double *y, int64_t n_nodes);
// out[k] = V_k . w for k < nk (V_k = V + k ldv), deterministic; partial holds
// nk * multidot_blocks(n) doubles
int multidot_blocks(int64_t n);
void launch_multidot(hipStream_t s, const double *V, int64_t ldv, int nk, const double *w, int64_t n,
                     double *partial, double *out);
// mode 0: w -= sum_k c[k] V_k; mode 1: w = sum_k c[k] V_k (c: device, nk entries)
void launch_combine(hipStream_t s, const double *V, int64_t ldv, int nk, const double *c, double *w,
                    int64_t n, int mode);
// out = a x + b y
void launch_axpby(hipStream_t s, double a, const double *x, double b, const double *y, double *out,
                  int64_t n);
// out = a x + b y + c z
void launch_axpbypcz(hipStream_t s, double a, const double *x, double b, const double *y, double c,
                     const double *z, double *out, int64_t n);

}  // namespace vmsk

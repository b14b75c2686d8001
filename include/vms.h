/*
 * libvms — C-ABI of the MI355X VMS assembly and in-out hot path.
 *
 * The method is the immersogeometric variational-multiscale (VMS) finite
 * element assembly of Saurabh et al., "Industrial scale large eddy
 * simulations with adaptive octree meshes using immersogeometric analysis"
 * (arXiv 2009.00706):
 *   - residual of the VMS weak form, eq. (vms), with the fine scales u' and p'
 *     of eqs. (uprime) and (pprime), and its Jacobian (matrix assembly,
 *     Alg. 2 and Alg. 6), for trilinear hexahedral octants, 2x2x2 Gauss points;
 *   - hanging-node constraints M_e of Alg. 3, scattered into a global CSR;
 *   - element markers IN / OUT / INTERCEPTED (Alg. 4) and exact in-out tests
 *     of quadrature points (the ground truth that Alg. 5 and ray tracing
 *     approximate);
 *   - adaptive sub-cell quadrature of INTERCEPTED elements (Section
 *     "Adaptive Quadrature" and the caption of its Gauss-point figure).
 *
 * Conventions shared by every entry point:
 *   - every function returns an int status (VMS_OK or a negative code) and
 *     never throws; vms_last_error() gives a message;
 *   - "host" pointers are read during the call only; "device" pointers are
 *     HIP device memory owned by the caller (the library never frees them);
 *   - dof numbering: dof = 4*node + c, c in (ux, uy, uz, p); independent nodes
 *     are numbered by the Morton key of their integer coordinates at
 *     resolution 2^max_level (x in the lowest bit); hanging vertices are not
 *     nodes;
 *   - CSR: rows ascending, columns ascending within a row, full 4x4 blocks
 *     for every node pair coupled by a non-IN element, plus every node's
 *     diagonal block; row_ptr is int64, col_idx int32;
 *   - signs: R = B^VMS - F^VMS with F = 0 (eq. ALE-VMS-form); J = dR/dU at the
 *     new time level, with tau_M, tau_C and taubar frozen at the current state;
 *   - nodes that receive no contribution from a non-IN element get an
 *     identity diagonal block and a zero residual; no boundary condition is
 *     imposed otherwise;
 *   - calls enqueue work on the context's stream and return; outputs are
 *     valid once the caller synchronises that stream. A context is bound to
 *     one stream and is not thread-safe.
 */
#ifndef VMS_H
#define VMS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vms_ctx vms_ctx; /* opaque */

/* status codes */
enum {
    VMS_OK = 0,
    VMS_EINVAL = -1,      /* bad argument (null pointer, size, NaN parameter, dt <= 0) */
    VMS_EMESH = -2,       /* octree not 2:1 balanced, chained constraint, surface not watertight */
    VMS_EHIP = -3,        /* a HIP runtime call failed */
    VMS_ENOMEM = -4,      /* device allocation failed */
    VMS_EOVERFLOW = -5,   /* a device-side capacity was exceeded */
    VMS_EUNSUPPORTED = -6 /* option outside what this build implements */
};

/* arithmetic of the element contractions (vms_params.precision) */
enum {
    VMS_FP64 = 0,       /* everything FP64; CSR values are double */
    VMS_MIXED_BF16 = 1, /* B^T D B on BF16 MFMA, FP32 accumulate; CSR values are float */
    VMS_MIXED_FP16 = 2  /* B^T D B on FP16 MFMA, FP32 accumulate; CSR values are float */
};

/* in-out test of quadrature points (inout_classify mode; vms_params.inout_mode) */
enum {
    VMS_INOUT_EXACT = 0,   /* exact segment parity with exact orientation predicates */
    VMS_INOUT_LEARNED = 1, /* learned signed-distance filter, exact test inside the margin */
    VMS_INOUT_NORMAL = 2   /* the normal-based test of Alg. 5 as a certified filter in front
                              of the exact test (sub-cell quadrature only; see vms_set_inout) */
};

/* scatter of the element matrices into the CSR values (vms_set_scatter) */
enum {
    VMS_SCATTER_RECORDS = 0, /* records summed per CSR block in a fixed order (default) */
    VMS_SCATTER_ATOMIC = 1   /* hardware atomic adds into the values (order not fixed) */
};

/* vms_assemble flags */
enum {
    VMS_RELABEL = 1u  /* recompute sub-cell quadrature points and their labels first */
};

/* vms_export selectors (all written to HOST memory, sizes from vms_sizes) */
enum {
    VMS_EXPORT_NODE_XYZ = 1,   /* int32 [3][n_nodes] integer coordinates (SoA) */
    VMS_EXPORT_ROW_PTR = 2,    /* int64 [n_rows + 1] */
    VMS_EXPORT_COL_IDX = 3,    /* int32 [nnz] */
    VMS_EXPORT_MARKERS = 4,    /* uint8 [n_oct]: 0 OUT, 1 IN, 2 INTERCEPTED */
    VMS_EXPORT_VERTEX_LAB = 5, /* uint8 [n_oct][8]: label of each element corner (0 OUT, 1 IN) */
    VMS_EXPORT_SUBGP = 6,      /* int64 [n_subgp] element, int32 [n_subgp] key, uint8 [n_subgp]
                                  level, double [n_subgp][3] xyz; canonical order (elements
                                  ascending, depth-first, children and Gauss points x fastest) */
    VMS_EXPORT_MASTERS = 7,    /* int32 [n_oct][8] master nodes per element slot (-1 unused) */
    VMS_EXPORT_SURFGP = 8,     /* surface points of the weak boundary terms, n = stats[6]:
                                  int64 [n] element, double [n][3] reference coordinates,
                                  double [n] weight, double [n][3] unit normal of the fluid */
    VMS_EXPORT_NODE_ROW_PTR = 9, /* int64 [n_nodes + 1]: the CSR at node level (4x4 blocks),
                                    block-row offsets; nnz / 16 blocks in all */
    VMS_EXPORT_NODE_COL = 10     /* int32 [nnz / 16]: block columns (column nodes), ascending
                                    within each block row; dof row 4 n + i holds the columns
                                    4 m + j (j = 0..3) of the block columns m of node row n */
};

/* Linear octree leaves, HOST pointers (copied at vms_create). A leaf at level L
 * has anchor (ax, ay, az) in units of 2^-max_level of the root side and side
 * 2^(max_level - L) units; physical x = origin + root_len * (integer / 2^max_level).
 * Leaves must not overlap and must be 2:1 balanced across faces, edges and
 * vertices (Section "Octree based Mesh Generation"). max_level <= 20. */
typedef struct {
    int64_t n_oct;
    const int32_t *ax, *ay, *az;
    const uint8_t *level;
    int32_t max_level;
    int32_t pad;
    double origin[3];
    double root_len;
} vms_octree;

/* Closed, watertight, consistently outward-oriented triangle surface, HOST
 * pointers: verts [n_vert][3] interleaved, tri [n_tri][3] (counter-clockwise
 * seen from outside), body_id [n_tri] (nullable) the body each triangle
 * belongs to. The bodies (components) are the body_id groups, or without
 * body_id the connected pieces of the triangle mesh (triangles joined by an
 * edge); bodies are disjoint and none lies inside another (vms_surface_components). */
typedef struct {
    int32_t n_vert, n_tri;
    const double *verts;
    const int32_t *tri;
    const int32_t *body_id;
} vms_surface;

/* Physical and discretisation parameters. theta = 1/2 is Crank-Nicolson (the
 * paper's remark on time stepping); tau_M = (c_t/dt^2 + u.G.u + c_i nu^2 G:G)^-1/2,
 * tau_C = 1/(tau_M tr G), taubar = (u'.G.u')^-1/2 with G = (2/h)^2 I.
 * quad_depth is the maximum split level of the adaptive quadrature (0..3). */
typedef struct {
    double rho, mu, dt, theta, c_t, c_i;
    int32_t quad_depth;
    uint32_t precision;      /* VMS_FP64 | VMS_MIXED_BF16 | VMS_MIXED_FP16 */
    uint32_t inout_mode;     /* in-out test of the sub-cell quadrature points on relabel:
                                VMS_INOUT_EXACT, VMS_INOUT_LEARNED (the network given by
                                vms_set_inout decides where |prediction| >= margin) or
                                VMS_INOUT_NORMAL (certified normal-based filter) */
    int32_t learned_min_bt;  /* LEARNED: the network is used on INTERCEPTED elements with at
                                least this many background triangles, the exact test alone
                                on the others */
} vms_params;

/* Nodal fields, DEVICE pointers, SoA over independent nodes (length n_nodes):
 * new-level velocity and pressure, previous-level velocity. */
typedef struct {
    const double *ux, *uy, *uz, *p, *ux0, *uy0, *uz0;
} vms_fields;

/* Create a context: derives vertices, hanging constraints (Alg. 3) and nodes on
 * the host; if surf is non-null, labels every corner exactly and sets element
 * markers (Alg. 4), gathers the background triangles of each INTERCEPTED
 * element and generates its adaptive sub-cell quadrature points (device);
 * builds the CSR pattern. stream is a hipStream_t (0 = null stream).
 * Errors: VMS_EINVAL, VMS_EMESH (unbalanced tree, chained constraint, surface
 * not watertight), VMS_EUNSUPPORTED (quad_depth > 3, max_level > 20),
 * VMS_ENOMEM, VMS_EHIP. On error *out is null. */
int vms_create(vms_ctx **out, const vms_octree *tree, const vms_surface *surf,
               const vms_params *prm, void *stream);

/* Sizes of the derived mesh: independent nodes, rows (= 4 n_nodes), nonzeros,
 * kept sub-cell quadrature points. Any pointer may be null. Synchronises the
 * stream; reports VMS_EOVERFLOW if a device-side capacity was exceeded. */
int vms_sizes(vms_ctx *ctx, int64_t *n_nodes, int64_t *n_rows, int64_t *nnz, int64_t *n_subgp);

/* Copy a derived quantity to HOST memory dst (see VMS_EXPORT_*). For
 * VMS_EXPORT_SUBGP dst must hold n_subgp * (8 + 4 + 1 + 24) bytes, laid out
 * as the four arrays one after the other. */
int vms_export(vms_ctx *ctx, uint32_t what, void *dst);

/* Matrix and vector assembly (Alg. 1 element loop, Alg. 2, Alg. 6):
 * csr_vals (DEVICE, nnz entries, double for VMS_FP64 else float) receives the
 * Jacobian, resid (DEVICE, n_rows doubles, nullable) the residual. Both are
 * overwritten; every entry is the sum of its element contributions in a fixed
 * order (element records summed by a gather, no atomics), so repeated calls on
 * the same input give the same bits. OUT elements use the 2x2x2 Gauss points,
 * INTERCEPTED elements their kept sub-cell points, IN elements nothing. */
int vms_assemble(vms_ctx *ctx, const vms_fields *f, void *csr_vals, double *resid,
                 uint32_t flags);

/* Vector assembly only: resid (DEVICE, n_rows doubles) is overwritten. If
 * norm2 (HOST) is non-null the call synchronises and stores ||resid||_2,
 * reduced in FP64 on the device. */
int vms_apply(vms_ctx *ctx, const vms_fields *f, double *resid, double *norm2);

/* Matrix-free Jacobian action: the product a Newton-Krylov solver asks for
 * when no matrix is assembled (the matrix-free route of the introduction's
 * matrix-assembly bullet, the footnote to the elemental matrix assembly of
 * §"Matrix Assembly on Distributed Octrees", and the conclusion).
 * y = J(U) x with J the Jacobian that vms_assemble writes at the fields f
 * (tau_M, tau_C and taubar frozen at f): at every quadrature point the
 * residual integrand of eq. (vms) with eq. (uprime) and eq. (pprime) is
 * differentiated along x, then contracted with the basis like the residual;
 * no element matrix and no CSR value is formed. x, y: DEVICE, n_rows doubles
 * (dof 4 node + c), y overwritten; rows of inactive nodes get y = x (their
 * identity blocks). FP64 contexts evaluate in FP64, mixed ones in FP32 with
 * FP64 accumulation of y. Timing (vms_last_timing): relabel 0, zeroing, OUT
 * elements, INTERCEPTED elements, identity rows. Errors: VMS_EINVAL (null
 * argument), VMS_EHIP. */
int vms_apply_jacobian(vms_ctx *ctx, const vms_fields *f, const double *x, double *y);

/* y = A x with A the matrix of the context's CSR pattern (layouts of
 * vms_export) and csr_vals its values (DEVICE, nnz entries, double for
 * VMS_FP64 contexts else float, e.g. from vms_assemble); x, y DEVICE, n_rows
 * doubles, y overwritten, FP64 accumulation in a fixed order (bitwise
 * reproducible). The Krylov product with the assembled Jacobian of
 * Alg. 2. Errors: VMS_EINVAL (null argument), VMS_EHIP. */
int vms_spmv(vms_ctx *ctx, const void *csr_vals, const double *x, double *y);

/* Dirichlet conditions of the solution procedure: the CG nodes of IN elements
 * (Section "Algorithms", where elements are labelled: no integration on IN
 * elements and Dirichlet conditions on their nodes) are the element corners
 * that are independent vertices (a hanging corner constrains nothing).
 * vms_dirichlet_nodes: count into *n (HOST) and, if nodes is not NULL, the
 * sorted node ids (HOST, *n int32). vms_dirichlet_in_nodes: every row of those
 * nodes in csr_vals (DEVICE, the context's precision) becomes an identity row
 * (all other entries of the row zero) and, if resid is not NULL (DEVICE),
 * their residual entries become zero (the iterate holds the prescribed
 * values, so Newton's update vanishes there). Without it an INTERCEPTED
 * element whose sub-cell points are all IN leaves its IN nodes with empty
 * rows. Errors: VMS_EINVAL (null argument), VMS_ENOMEM, VMS_EHIP. */
int vms_dirichlet_nodes(vms_ctx *ctx, int64_t *n, int32_t *nodes);
int vms_dirichlet_in_nodes(vms_ctx *ctx, void *csr_vals, double *resid);

/* Krylov method of vms_solve */
enum {
    VMS_KSP_BCGS = 0, /* BiCGStab, the paper's Krylov method (appendix "Details of solver selection") */
    VMS_KSP_GMRES = 1 /* restarted GMRES(restart) */
};
/* vms_solve flags */
enum {
    VMS_SOLVE_DIRICHLET = 1u /* the matrix-free operator takes identity rows at the Dirichlet
                                nodes too (use with values that had vms_dirichlet_in_nodes) */
};

/* Newton's linear step A dx = b, the solve the paper hands to its Krylov
 * solver between Jacobian and residual assemblies (Alg. 2 feeds it; the
 * paper's runs use BiCGStab with an additive Schwarz preconditioner, here
 * block Jacobi on the 4x4 node blocks, its one-block-per-node form without
 * overlap). Right preconditioning by the inverses of the diagonal node blocks
 * of csr_vals, so the monitored residual is the true one; FP64 vectors and
 * deterministic inner products. method: VMS_KSP_BCGS or VMS_KSP_GMRES (Arnoldi
 * by classical Gram-Schmidt with one reorthogonalisation, restart in
 * [1, 200]; ignored for BiCGStab). A is the assembled matrix (fields = NULL)
 * or the matrix-free Jacobian action at the given fields (vms_apply_jacobian);
 * the preconditioner always comes from csr_vals (DEVICE, nnz values of the
 * context's precision, e.g. from vms_assemble). b, x: DEVICE, n_rows doubles;
 * x holds the initial guess on entry and the iterate on return. Stops when
 * ||b - A x|| <= rtol ||b|| (true residual, recomputed at every restart of
 * the recurrence), after max_iter steps (a BiCGStab step has two products
 * with A), or at a breakdown that a restart cannot cure. flags: 0 or
 * VMS_SOLVE_DIRICHLET. iters, rel_res: HOST
 * outputs (nullable): steps taken and the final true relative residual (the
 * caller compares it with rtol). Device workspace (max(restart + 1, 8) + 3
 * vectors of n_rows doubles and 16 doubles per node) is allocated by the first
 * call and kept by the context; synchronises the context stream. Errors:
 * VMS_EINVAL (null argument, unknown method or flag, restart outside [1, 200],
 * negative max_iter, non-positive rtol, singular diagonal block), VMS_ENOMEM,
 * VMS_EHIP. */
int vms_solve(vms_ctx *ctx, const void *csr_vals, const vms_fields *fields, const double *b, double *x,
              int method, int restart, int max_iter, double rtol, uint32_t flags, int *iters,
              double *rel_res);

/* Weak (Nitsche) enforcement of u = g on the immersed surface, eq. (weakbc)
 * with the remark after it (§"Weak Enforcement of Boundary Conditions"): once
 * enabled, vms_assemble, vms_apply and vms_apply_jacobian add the surface
 * integrals (consistency, adjoint consistency with the sign of eq. (weakbc),
 * inflow term on u . n < 0, tangential and normal penalties) to the residual
 * and the Jacobian. Surface quadrature: three points per triangle
 * (barycentric 2/3, 1/6, 1/6 and permutations, a third of the area each),
 * each in the leaf octant that contains it (half-open boxes at the finest
 * resolution; points in IN octants dropped); n is the unit normal of the fluid
 * domain (minus the body's outward normal); velocity terms at u_theta, the
 * pressure at the new step. tau_T = tau_N = c_b mu / h_b per element, h_b the
 * largest exact distance from the element's OUT corners to the surface, at
 * least h/100. g: HOST double[3], the prescribed surface velocity (0 for no
 * slip). The Jacobian freezes tau_B and the inflow indicator. Builds the
 * surface points, h_b and the record lists on the first call (allocates;
 * synchronises the stream); enable = 0 switches the terms off. Contexts with
 * the terms on cannot join a vms_batch, and a batch whose context has them
 * switched on later refuses to assemble (VMS_EUNSUPPORTED, before any launch).
 * Errors: VMS_EINVAL (no surface, c_b < 0
 * or non-finite values), VMS_ENOMEM, VMS_EHIP. */
int vms_set_weak_bc(vms_ctx *ctx, int enable, double c_b, const double *g);

/* Element weights of eq. (Wpart) (§"Estimation of Weight for the INTERCEPTED
 * Elements"): w[e] = n_Vgp(e)/n_Tgp + ts_over_tv n_Sgp(e)/n_Tgp with n_Tgp = 8
 * (trilinear elements), n_Vgp the element's volume quadrature points (8 for
 * OUT, its kept sub-cell points for INTERCEPTED, 0 for IN) and n_Sgp its
 * surface points of the weak boundary terms (0 while they are off). OUT
 * elements weigh 1, IN elements 0. ts_over_tv is the measured ratio of the
 * cost of a surface point to that of a volume point. w: HOST, n_oct doubles,
 * octree order. Errors: VMS_EINVAL (null argument, negative ratio). */
int vms_element_weights(vms_ctx *ctx, double ts_over_tv, double *w);

/* Exact in-out labels of n points against a surface (Alg. 5's question,
 * answered exactly): px, py, pz DEVICE arrays of n doubles, labels DEVICE
 * uint8 (1 IN or on the surface, 0 OUT). mode VMS_INOUT_EXACT, or
 * VMS_INOUT_LEARNED with mlp a vms_mlp handle (points whose |prediction| >=
 * its margin take the network's sign, the rest the exact test).
 * The surface's acceleration structure is built on the host at each call
 * unless a context-free cache handle is used (see inout_prepare).
 * stream is a hipStream_t. */
int inout_classify(const vms_surface *surf, const double *px, const double *py, const double *pz,
                   int64_t n, uint8_t *labels, uint32_t mode, const void *mlp, void *stream);

/* Reusable in-out handle: the surface's acceleration structure built once
 * (host pointers read during the call; device memory owned by the handle);
 * the handle is bound to stream. inout_classify_prepared has the semantics of
 * inout_classify. In VMS_INOUT_EXACT mode it allocates nothing. In
 * VMS_INOUT_LEARNED mode it uses 20 bytes of handle-owned scratch per point
 * (network outputs, the indices sent to the exact test, their count):
 * inout_reserve(h, n) allocates it for up to n points beforehand, so that
 * later calls of at most n points allocate nothing; a call with more points
 * than reserved grows it (allocates, synchronising). */
typedef struct inout_handle inout_handle;
int inout_prepare(const vms_surface *surf, void *stream, inout_handle **out);
int inout_reserve(inout_handle *h, int64_t n);
int inout_classify_prepared(inout_handle *h, const double *px, const double *py, const double *pz,
                            int64_t n, uint8_t *labels, uint32_t mode, const void *mlp);
void inout_release(inout_handle *h);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the exact
 * labels of inout_classify (mode VMS_INOUT_EXACT) with the surface's staging
 * (packed triangles, their boxes and the (y, z) bin grid, about 120 bytes per
 * triangle plus the bins) in a static device array of VMS_STATIC_SCRATCH_MIB
 * MiB that each GPU holds from the first call on it until the process ends.
 * Allocates no device memory. surf: HOST arrays (read during the call);
 * px, py, pz, labels: DEVICE arrays of n entries on the current device;
 * stream: a hipStream_t of the current device. The staging is copied in on
 * stream and the call synchronises stream before returning. All calls on one
 * GPU share the array and each overwrites it: calls that overlap on one GPU
 * (other threads) race. Errors: VMS_EINVAL (null argument, negative n,
 * invalid surface), VMS_EMESH (surface not closed / not consistently
 * oriented), VMS_EOVERFLOW (staging larger than the array; nothing is
 * launched), VMS_EHIP. Message: inout_static_last_error(). */
#define VMS_STATIC_SCRATCH_MIB 32
int inout_classify_static(const vms_surface *surf, const double *px, const double *py,
                          const double *pz, int64_t n, uint8_t *labels, void *stream);
const char *inout_static_last_error(void);

/* Triquadratic (Q2, 27-node) elements on a uniform octree: the quadratic
 * basis of the paper's matrix-assembly comparison (the table of assembly
 * times for linear and quadratic bases on a uniform mesh) with the basis
 * tabulated at the (bf+1)^d = 27 Gauss points (App. A). Every leaf must be on
 * one level (no hanging nodes; VMS_EMESH otherwise), max_level <= 19, no
 * immersed body, precision VMS_FP64 (VMS_EUNSUPPORTED otherwise). The
 * integrand is that of vms_assemble (eq. (vms), (uprime), (pprime); taus
 * frozen for the Jacobian) integrated with the 3-point Gauss rule per axis.
 * Nodes: positions on the grid of half the element side (vms_q2_export
 * VMS_EXPORT_NODE_XYZ gives these integers, physical x = origin + root_len
 * (integer / 2^(max_level + 1))), numbered by Morton key; element node a is
 * (a % 3, a / 3 % 3, a / 9) of its 3 x 3 x 3 node grid. CSR (VMS_EXPORT_ROW_PTR,
 * VMS_EXPORT_COL_IDX): full 4x4 blocks for every node pair that shares an
 * element, columns ascending, dof = 4 node + c. vms_q2_assemble: fields
 * DEVICE arrays over the nodes, csr_vals DEVICE nnz doubles, resid DEVICE
 * (nullable) 4 n_nodes doubles; both overwritten with sums of element records
 * in a fixed order; enqueued on the context's stream. Set-up allocates; the
 * assembly does not. Errors: VMS_EINVAL, VMS_EMESH, VMS_EUNSUPPORTED,
 * VMS_ENOMEM, VMS_EHIP; message from vms_q2_last_error (null: last failed
 * create). */
typedef struct vms_q2 vms_q2;
int vms_q2_create(vms_q2 **out, const vms_octree *tree, const vms_params *prm, void *stream);
int vms_q2_sizes(vms_q2 *q, int64_t *n_nodes, int64_t *n_rows, int64_t *nnz);
int vms_q2_export(vms_q2 *q, uint32_t what, void *dst);
int vms_q2_assemble(vms_q2 *q, const vms_fields *fields, double *csr_vals, double *resid);
/* HOST ms[2]: element kernel and gathers of the last vms_q2_assemble
 * (synchronises on it; VMS_EINVAL if there was none). */
int vms_q2_last_timing(vms_q2 *q, float *ms);
const char *vms_q2_last_error(vms_q2 *q);
void vms_q2_destroy(vms_q2 *q);

/* Host-only mesh derivation (no device involved): the node numbering,
 * hanging constraints and CSR pattern that vms_create derives, for checks on
 * machines without a GPU. markers (HOST, nullable) excludes IN elements
 * (marker 1) from the pattern. vms_mesh_export accepts VMS_EXPORT_NODE_XYZ,
 * _ROW_PTR, _COL_IDX and _MASTERS with the layouts of vms_export. */
typedef struct vms_mesh vms_mesh;
int vms_mesh_create(vms_mesh **out, const vms_octree *tree, const uint8_t *markers);
int vms_mesh_sizes(vms_mesh *h, int64_t *n_nodes, int64_t *nnz, int64_t *n_hanging);
int vms_mesh_export(vms_mesh *h, uint32_t what, void *dst);
void vms_mesh_destroy(vms_mesh *h);

/* Per-stage timing with HIP events recorded on the context stream (off by
 * default). vms_last_timing synchronises on the last recorded event and
 * writes HOST ms[5]: relabelling (sub-cell quadrature and in-out tests),
 * host set-up of the kernel arguments (no kernel), OUT-element assembly
 * kernel, INTERCEPTED-element assembly kernel (and surface terms), summation
 * of the element records into the CSR values (with identity rows) and the
 * residual, of the last vms_assemble / vms_apply. After an overlapped
 * vms_assemble (vms_set_overlap) ms[0] and ms[3] are measured on the second
 * stream and ran beside ms[4], which spans from the end of the OUT elements to
 * the end of the call: the device time of the call is ms[1] + ms[2] + ms[4]
 * there, the sum of all five otherwise. */
int vms_set_timing(vms_ctx *ctx, int on);
int vms_last_timing(vms_ctx *ctx, float *ms);

/* Schedule of vms_assemble (on = 1, the default, or 0). The element records
 * of OUT elements are complete once their kernel ends, and most CSR blocks
 * (those of nodes away from the surface) receive no other records. With
 * overlap on, a call that assembles the matrix and has INTERCEPTED items (or
 * weak boundary terms) runs the relabel, the INTERCEPTED items and the surface
 * terms on a second stream that the context owns (created on first use, on the
 * current device, default priority), started by an event after the OUT
 * kernel, while the context stream sums the blocks without late records; the
 * context stream then waits for the second stream and sums the late blocks.
 * When the relabel and the INTERCEPTED items are estimated to take well under
 * the gather, fewer of their workgroups share a CU (extra LDS requested at
 * their launch), which leaves the HBM-bound gather more waves; the estimate
 * uses the numbers of labels and sub-cell points and the gather's bytes at
 * rates measured on MI355X.
 * All of the call's work is ordered before later work on the context stream,
 * and the outputs are bit for bit those of the in-order schedule (same
 * records, same per-block summation order). Off: every stage in order on the
 * context stream (isolated stage times). Errors: VMS_EINVAL (null context). */
int vms_set_overlap(vms_ctx *ctx, int on);

/* Scatter of the element matrices in vms_assemble. VMS_SCATTER_RECORDS (the
 * default): every work item writes a 1024-entry record and a gather sums each
 * CSR block from its records in a fixed order (repeatable bits). Scatter
 * alternative measured beside it, VMS_SCATTER_ATOMIC: the values are zeroed,
 * then each element kernel adds its entries with hardware atomic adds (FP64
 * for VMS_FP64, FP32 otherwise) at their CSR places, and the identity blocks of
 * inactive nodes are written last; no record and no gather, but the order of
 * the additions, and so the last bits of the values, may change from call to
 * call. The residual is summed from records in both modes. The first switch to
 * the atomic mode copies each element's block columns to the device (128
 * bytes per element). Batches (vms_batch_*) keep the records. Errors:
 * VMS_EINVAL (null context, unknown mode), VMS_EUNSUPPORTED (atomic mode with
 * the weak boundary terms on; vms_set_weak_bc refuses them in the atomic
 * mode), VMS_ENOMEM. */
int vms_set_scatter(vms_ctx *ctx, uint32_t mode);

/* Learned in-out filter (signed-distance network; negative inside):
 * xh = 2 (x - lo)/(hi - lo) - 1, phi = [sin 2 pi B xh; cos 2 pi B xh] with
 * B (32 x 3, HOST float, row-major), three hidden SiLU layers of width 64, a
 * linear output; theta (HOST float[12545]): W1 (64x64 row-major, out x in),
 * b1, W2, b2, W3, b3, w4 (64), b4. Training regresses the signed distance
 * clamped to [-trunc, trunc] (loss: mean of squared error / 2) with Adam.
 * The handle owns its device memory and is bound to stream. Callers that use
 * it for classification: points with |prediction| >= margin take its sign, the
 * rest the exact test (the margin is the caller's calibration, default +inf).
 * The box must contain the surface's box: a point outside it is reported as
 * far outside (prediction +inf), which is exact. */
typedef struct vms_mlp vms_mlp;
int vms_mlp_create(vms_mlp **out, const double *lo, const double *hi, const float *theta,
                   const float *B, float trunc, void *stream);
int vms_mlp_get_params(vms_mlp *m, float *theta /* HOST */);
int vms_mlp_set_margin(vms_mlp *m, float margin);
/* Per-cell margins: margins HOST float[nx*ny*nz] (x fastest) over a uniform
 * grid of the network box; a point uses the margin of its cell (+inf: never
 * decided by the network). nx = ny = nz = 0 removes the grid (the scalar
 * margin applies again). VMS_EINVAL for negative or NaN margins. */
int vms_mlp_set_margin_grid(vms_mlp *m, int nx, int ny, int nz, const float *margins);
/* Loss and gradient over n samples (DEVICE points, DEVICE exact signed
 * distances); grad DEVICE float[12545] (nullable), loss HOST (nullable). */
int vms_mlp_grad(vms_mlp *m, const double *px, const double *py, const double *pz, const double *sdf,
                 int64_t n, float *grad, double *loss);
/* steps Adam updates (beta 0.9, 0.999, eps 1e-8) over consecutive batches of
 * the n samples (wrapping around); last_loss HOST (nullable): loss of the last batch. */
int vms_mlp_train(vms_mlp *m, const double *px, const double *py, const double *pz, const double *sdf,
                  int64_t n, int steps, int batch, float lr, double *last_loss);
/* One Adam update with a given DEVICE gradient. */
int vms_mlp_adam_step(vms_mlp *m, const float *grad, float lr);
/* Network outputs of n DEVICE points into DEVICE float pred (FP16 MFMA inference). */
int vms_mlp_predict(vms_mlp *m, const double *px, const double *py, const double *pz, int64_t n,
                    float *pred);
const char *vms_mlp_last_error(void);
void vms_mlp_destroy(vms_mlp *m);

/* Exact signed distance of n DEVICE points to the handle's surface, clamped to
 * [-trunc, trunc] (negative inside; sign from the exact in-out test), into
 * DEVICE sdf. Synchronises the handle's stream. */
int vms_sdf_sample(inout_handle *h, const double *px, const double *py, const double *pz, int64_t n,
                   double trunc, double *sdf);

/* Batched assembly of many contexts (independent octrees, one precision) in
 * one persistent launch: workgroups take units of work from a device counter
 * until the queue is empty. A unit is a run of OUT elements or of sub-cell
 * work items of one tree, cut at about `tile` element weights of eq. (Wpart)
 * (§"Estimation of Weight for the INTERCEPTED Elements": an OUT element weighs
 * 1, an INTERCEPTED element's work item its points over 8), and the queue
 * holds the units heaviest first, so that it ends on light units (the load
 * balance that the paper's weighted partition gives across processes).
 * vms_batch_set_order(b, 0) selects the fixed order instead (every sub-cell
 * item a unit of its own, all of them first, then runs of `tile` OUT
 * elements). After the persistent launch one batched gather sums every
 * tree's CSR values (identity rows of inactive nodes included) and one its
 * residual. fields/vals/resid are arrays with one entry per context (resid
 * entries nullable), with the meaning of vms_assemble (labels are not
 * recomputed). vms_batch_autotune times every (tile, workgroups per CU)
 * candidate on the given buffers and keeps the fastest. With
 * vms_batch_use_graph(b, 1) the launch sequence (counter reset, persistent
 * assembly, gathers) is captured into a HIP graph at the first call and
 * replayed while the buffer pointers stay the same. Every call re-checks its
 * contexts: one whose record buffers were rebuilt since (weak boundary terms
 * switched on and off again) is re-read and the captured graph dropped; one
 * with weak boundary terms on makes the call return VMS_EUNSUPPORTED before
 * any launch. vms_batch_last_timing writes HOST ms[3] (an empty interval
 * before the kernels, persistent assembly kernel, gathers) of the last eager
 * (not graph-replayed) vms_batch_assemble, synchronising on it; VMS_EINVAL if
 * there was none. */
typedef struct vms_batch vms_batch;
int vms_batch_create(vms_batch **out, vms_ctx *const *ctxs, int n, void *stream);
int vms_batch_set_config(vms_batch *b, int tile, int groups_per_cu);
int vms_batch_set_order(vms_batch *b, int by_weight);
int vms_batch_get_config(vms_batch *b, int *tile, int *groups_per_cu, int64_t *n_units);
int vms_batch_use_graph(vms_batch *b, int on);
int vms_batch_assemble(vms_batch *b, const vms_fields *fields, void *const *vals,
                       double *const *resid);
int vms_batch_autotune(vms_batch *b, const vms_fields *fields, void *const *vals,
                       double *const *resid, float *ms);
int vms_batch_last_timing(vms_batch *b, float *ms);
void vms_batch_destroy(vms_batch *b);

/* In-out test of the sub-cell quadrature on relabel (§"Adaptive Quadrature";
 * Alg. 5's question answered with a learned filter in front of the exact
 * test): mode VMS_INOUT_EXACT, or VMS_INOUT_LEARNED with mlp a trained and
 * calibrated vms_mlp handle (kept by reference: it must outlive its use by
 * the context). On INTERCEPTED elements with at least min_bt background
 * triangles each candidate point goes through the network first; a point
 * whose |prediction| reaches its margin takes the network's sign, every other
 * point the exact test. Labels equal the exact ones wherever the margin
 * exceeds the network's error; a relabel whose kept-point count of an
 * element differs from the set-up's exact count reports VMS_EOVERFLOW at the
 * next vms_sizes. Errors: VMS_EINVAL. vms_relabel_stats writes HOST out[2]:
 * candidate points of the sub-cell quadrature (set-up pass) and those
 * labelled by the exact test in the last relabel (synchronises). */
int vms_set_inout(vms_ctx *ctx, uint32_t mode, const vms_mlp *mlp, int32_t min_bt);
int vms_relabel_stats(vms_ctx *ctx, int64_t *out);

/* VMS_INOUT_NORMAL (vms_set_inout with mlp null, min_bt 0, or inout_mode in
 * vms_params): the paper's normal-based test (Alg. 5 and the text after it)
 * used only where it is certain. A body is convex when at every edge the far
 * vertex of one adjacent triangle is not strictly outside the plane of the
 * other (checked with exact predicates at vms_create); a point strictly
 * outside the plane of one of a convex body's triangles (the sign of the
 * exact orientation of the triangle and the point, i.e. of (P - centroid) . n)
 * is outside that body. A candidate point of an INTERCEPTED element is labelled
 * OUT when, for every body with triangles among the element's background
 * triangles, it is strictly outside one of those triangles' planes and the
 * body is convex (a body with no background triangle cannot contain a point
 * of an element it does not cut, bodies being disjoint and not nested); every
 * other point (inside all planes, on one, a non-convex body, more than 8
 * bodies or more than 64 background triangles at the element) takes the exact
 * test. Labels are therefore exact; vms_relabel_stats counts the points the
 * exact test labelled. vms_components writes HOST n_comp and, if convex is
 * non-null, convex[n_comp] (1 convex, 0 not) for the context's surface. */
int vms_components(vms_ctx *ctx, int32_t *n_comp, uint8_t *convex);

/* Host-only: the bodies of a surface (the body_id groups, or the connected
 * pieces of the mesh), comp (HOST [n_tri], nullable) the body index of each
 * triangle, 0 .. n_comp - 1 in order of first appearance. Errors: VMS_EINVAL
 * (invalid surface, or body_id differing across an edge), VMS_EMESH (not
 * closed / not consistently oriented). */
int vms_surface_components(const vms_surface *surf, int32_t *comp, int32_t *n_comp);

/* Counters of a context (HOST out[7]): OUT elements, INTERCEPTED elements,
 * points labelled by the last sub-cell quadrature, degenerate directions
 * abandoned, hanging vertices, kept sub-cell points, surface points of the
 * weak boundary terms (0 while they are off). */
int vms_stats(vms_ctx *ctx, int64_t *out);

/* Message of the last error on ctx (or of the last failed vms_create /
 * inout_classify when ctx is null). Never null. */
const char *vms_last_error(vms_ctx *ctx);

/* Free the context's device memory. Accepts null. */
void vms_destroy(vms_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* VMS_H */

// C-ABI of libvms: context creation (host mesh derivation, device setup of
// labels, markers and sub-cell quadrature), assembly launches, exports.
#include "../../include/vms.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "geom.h"
#include "kernels.h"
#include "mesh.h"
#include "par.h"
#include "mlp.h"
#include "surface_pack.h"

using vmsk::SurfDev;

int vmsm_sdf(hipStream_t s, const vmsk::SurfDev &S, const std::vector<double> &tv, const double *lo,
             const double *hi, const double *px, const double *py, const double *pz, int64_t n,
             double trunc, double *out);

// sub-cell points per assembly work item (longer items: fewer element-matrix
// records and item set-ups; shorter items: finer load balance)
#ifndef VMS_ITEM_PTS
#define VMS_ITEM_PTS 128
#endif

namespace vms {

// Watertightness and orientation: every directed edge appears once and its
// reverse appears too.
int check_watertight(const vms_surface *s, std::string &err) {
    const int64_t nt = s->n_tri;
    std::vector<uint64_t> fwd;
    fwd.reserve(3 * nt);
    for (int64_t t = 0; t < nt; ++t)
        for (int k = 0; k < 3; ++k) {
            int64_t a = s->tri[3 * t + k], b = s->tri[3 * t + (k + 1) % 3];
            if (a < 0 || b < 0 || a >= s->n_vert || b >= s->n_vert || a == b) {
                err = "triangle with an invalid vertex index";
                return VMS_EINVAL;
            }
            fwd.push_back(((uint64_t)a << 32) | (uint64_t)b);
        }
    std::sort(fwd.begin(), fwd.end());
    for (size_t i = 1; i < fwd.size(); ++i)
        if (fwd[i] == fwd[i - 1]) { err = "surface not consistently oriented (repeated edge)"; return VMS_EMESH; }
    for (uint64_t e : fwd) {
        uint64_t r = ((e & 0xffffffffull) << 32) | (e >> 32);
        if (!std::binary_search(fwd.begin(), fwd.end(), r)) {
            err = "surface not watertight (edge without its opposite)";
            return VMS_EMESH;
        }
    }
    return VMS_OK;
}

// Bodies of a closed surface: the body_id groups, or the connected pieces
// (triangles joined by an edge, union-find), numbered by first appearance.
// edges (nullable) receives every edge once as (t1, t2, corner of t2 opposite
// the edge) for the convexity test. The surface must have passed
// check_watertight: every undirected edge has exactly two triangles.
int surface_components(const vms_surface *s, std::vector<int32_t> &comp, int32_t &n_comp,
                       std::vector<int32_t> *et1, std::vector<int32_t> *et2, std::vector<int8_t> *ecorner,
                       std::string &err) {
    const int64_t nt = s->n_tri;
    struct E { uint64_t key; int32_t t; int8_t k; };
    std::vector<E> ed;
    ed.reserve(3 * nt);
    for (int64_t t = 0; t < nt; ++t)
        for (int k = 0; k < 3; ++k) {
            const uint64_t a = (uint32_t)s->tri[3 * t + k], b = (uint32_t)s->tri[3 * t + (k + 1) % 3];
            ed.push_back({(std::min(a, b) << 32) | std::max(a, b), (int32_t)t, (int8_t)k});
        }
    std::sort(ed.begin(), ed.end(), [](const E &x, const E &y) { return x.key != y.key ? x.key < y.key : x.t < y.t; });
    std::vector<int32_t> par(nt);
    for (int64_t t = 0; t < nt; ++t) par[t] = (int32_t)t;
    auto find = [&](int32_t x) {
        while (par[x] != x) x = par[x] = par[par[x]];
        return x;
    };
    if (s->body_id)
        for (int64_t t = 0; t < nt; ++t)
            if (s->body_id[t] < 0) { err = "negative body id"; return VMS_EINVAL; }
    for (size_t i = 0; i + 1 < ed.size(); i += 2) {
        if (ed[i].key != ed[i + 1].key) { err = "surface edge without exactly two triangles"; return VMS_EMESH; }
        const int32_t t1 = ed[i].t, t2 = ed[i + 1].t;
        if (s->body_id && s->body_id[t1] != s->body_id[t2]) { err = "body id differs across an edge"; return VMS_EINVAL; }
        const int32_t r1 = find(t1), r2 = find(t2);
        if (r1 != r2) par[std::max(r1, r2)] = std::min(r1, r2);
        if (et1) {
            et1->push_back(t1);
            et2->push_back(t2);
            ecorner->push_back((int8_t)((ed[i + 1].k + 2) % 3));
        }
    }
    comp.assign(nt, -1);
    std::vector<int64_t> ids(nt);
    for (int64_t t = 0; t < nt; ++t) ids[t] = s->body_id ? (int64_t)s->body_id[t] : (int64_t)find((int32_t)t);
    std::vector<int64_t> order(ids);
    std::sort(order.begin(), order.end());
    order.erase(std::unique(order.begin(), order.end()), order.end());
    std::vector<int32_t> num(order.size(), -1);
    n_comp = 0;
    for (int64_t t = 0; t < nt; ++t) {
        const size_t j = std::lower_bound(order.begin(), order.end(), ids[t]) - order.begin();
        if (num[j] < 0) num[j] = n_comp++;
        comp[t] = num[j];
    }
    return VMS_OK;
}

// bin index, the same arithmetic as the device query
static inline int host_bin(double v, double v0, double inv, int n) {
    volatile double d = v - v0;
    volatile double t = d * inv;
    int b = (int)std::floor(t);
    return b < 0 ? 0 : (b >= n ? n - 1 : b);
}

int pack_surface(const vms_surface *s, SurfacePack &P, std::string &err) {
    if (!s || s->n_tri <= 0 || s->n_vert <= 0 || !s->verts || !s->tri) {
        err = "empty or null surface";
        return VMS_EINVAL;
    }
    int rc = check_watertight(s, err);
    if (rc) return rc;
    const int64_t nt = s->n_tri;
    if (nt > INT32_MAX) { err = "too many triangles"; return VMS_EINVAL; }
    P.tv.resize(9 * nt);
    P.tbox.resize(6 * nt);
    SurfDev &S = P.S;
    S = SurfDev{};
    for (int k = 0; k < 3; ++k) { S.lo[k] = INFINITY; S.hi[k] = -INFINITY; }
    for (int64_t v = 0; v < s->n_vert; ++v)
        for (int k = 0; k < 3; ++k) {
            double x = s->verts[3 * v + k];
            if (!std::isfinite(x)) { err = "non-finite surface vertex"; return VMS_EINVAL; }
            S.lo[k] = std::min(S.lo[k], x);
            S.hi[k] = std::max(S.hi[k], x);
        }
    for (int64_t t = 0; t < nt; ++t) {
        for (int c = 0; c < 3; ++c)
            for (int k = 0; k < 3; ++k) P.tv[9 * t + 3 * c + k] = s->verts[3 * s->tri[3 * t + c] + k];
        for (int k = 0; k < 3; ++k) {
            double a = P.tv[9 * t + k], b = P.tv[9 * t + 3 + k], c = P.tv[9 * t + 6 + k];
            P.tbox[6 * t + k] = std::min(a, std::min(b, c));
            P.tbox[6 * t + 3 + k] = std::max(a, std::max(b, c));
        }
    }
    // (y, z) bins for rays along +x or -x
    int nb = (int)std::ceil(std::sqrt((double)nt));
    nb = std::max(1, std::min(nb, 1024));
    S.n_tri = (int32_t)nt;
    S.nby = S.nbz = nb;
    S.y0 = S.lo[1];
    S.z0 = S.lo[2];
    double wy = S.hi[1] - S.lo[1], wz = S.hi[2] - S.lo[2];
    S.iny = wy > 0 ? nb / wy : 0.0;
    S.inz = wz > 0 ? nb / wz : 0.0;
    P.off.assign((size_t)nb * nb + 1, 0);
    auto range = [&](int64_t t, int &y0, int &y1, int &z0, int &z1) {
        y0 = host_bin(P.tbox[6 * t + 1], S.y0, S.iny, nb);
        y1 = host_bin(P.tbox[6 * t + 4], S.y0, S.iny, nb);
        z0 = host_bin(P.tbox[6 * t + 2], S.z0, S.inz, nb);
        z1 = host_bin(P.tbox[6 * t + 5], S.z0, S.inz, nb);
    };
    for (int64_t t = 0; t < nt; ++t) {
        int y0, y1, z0, z1;
        range(t, y0, y1, z0, z1);
        for (int z = z0; z <= z1; ++z)
            for (int y = y0; y <= y1; ++y) P.off[(size_t)z * nb + y + 1]++;
    }
    for (size_t i = 1; i < P.off.size(); ++i) P.off[i] += P.off[i - 1];
    P.ids.assign(P.off.back(), 0);
    std::vector<int32_t> fillp(P.off.begin(), P.off.end() - 1);
    for (int64_t t = 0; t < nt; ++t) {
        int y0, y1, z0, z1;
        range(t, y0, y1, z0, z1);
        for (int z = z0; z <= z1; ++z)
            for (int y = y0; y <= y1; ++y) P.ids[fillp[(size_t)z * nb + y]++] = (int32_t)t;
    }
    return VMS_OK;
}

}  // namespace vms

using vms::check_watertight;
using vms::host_bin;

namespace {

std::mutex g_err_mu;
std::string g_err = "no error";

void set_global_err(const std::string &s) {
    std::lock_guard<std::mutex> lk(g_err_mu);
    g_err = s;
}

struct DevBuf {
    std::vector<void *> ptrs;
    ~DevBuf() { release(); }
    void release() {
        for (void *p : ptrs) (void)hipFree(p);
        ptrs.clear();
    }
    void free(void *p) {
        if (!p) return;
        for (size_t i = 0; i < ptrs.size(); ++i)
            if (ptrs[i] == p) {
                (void)hipFree(p);
                ptrs.erase(ptrs.begin() + (long)i);
                return;
            }
    }
    template <typename T>
    hipError_t alloc(T **p, size_t n) {
        *p = nullptr;
        if (n == 0) n = 1;
        hipError_t e = hipMalloc((void **)p, n * sizeof(T));
        if (e == hipSuccess) ptrs.push_back(*p);
        return e;
    }
};

// Surface on the device plus its host-side description.
struct SurfaceHost {
    SurfDev S{};
    DevBuf buf;
    std::vector<double> tv, tbox;  // host copies (background-triangle gathering)
    double lo[3], hi[3];
};

int build_surface(const vms_surface *s, hipStream_t st, SurfaceHost &H, std::string &err) {
    vms::SurfacePack P;
    int rc = vms::pack_surface(s, P, err);
    if (rc) return rc;
    H.S = P.S;
    for (int k = 0; k < 3; ++k) { H.lo[k] = P.S.lo[k]; H.hi[k] = P.S.hi[k]; }
    double *dtv, *dtb;
    int32_t *doff, *dids;
    if (H.buf.alloc(&dtv, P.tv.size()) || H.buf.alloc(&dtb, P.tbox.size()) ||
        H.buf.alloc(&doff, P.off.size()) || H.buf.alloc(&dids, P.ids.size())) {
        err = "device allocation failed (surface)";
        return VMS_ENOMEM;
    }
    if (hipMemcpyAsync(dtv, P.tv.data(), P.tv.size() * 8, hipMemcpyHostToDevice, st) ||
        hipMemcpyAsync(dtb, P.tbox.data(), P.tbox.size() * 8, hipMemcpyHostToDevice, st) ||
        hipMemcpyAsync(doff, P.off.data(), P.off.size() * 4, hipMemcpyHostToDevice, st) ||
        (P.ids.size() && hipMemcpyAsync(dids, P.ids.data(), P.ids.size() * 4, hipMemcpyHostToDevice, st)) ||
        hipStreamSynchronize(st)) {
        err = "device copy failed (surface)";
        return VMS_EHIP;
    }
    H.S.tv = dtv;
    H.S.tbox = dtb;
    H.S.bin_off = doff;
    H.S.bin_tri = dids;
    H.tv = std::move(P.tv);
    H.tbox = std::move(P.tbox);
    return VMS_OK;
}

}  // namespace

struct vms_ctx {
    hipStream_t stream = nullptr;
    std::string err = "no error";
    vms_params prm{};
    double origin[3] = {0, 0, 0};
    double root_len = 1.0;
    int max_level = 0;
    vms::MeshHost mesh;
    std::vector<int32_t> ax, ay, az;
    std::vector<uint8_t> level, markers, corner_lab;
    bool has_surf = false;
    SurfaceHost surf;
    DevBuf buf;
    // element data
    int32_t *d_masters = nullptr;
    uint32_t *d_ccode = nullptr;
    uint8_t *d_hang = nullptr, *d_level = nullptr;
    int64_t n_std = 0;
    int32_t *d_std = nullptr;
    // intercepted elements and their sub-cell points
    int64_t n_sq = 0;
    std::vector<int32_t> sq_el;
    std::vector<int32_t> sq_cnt;
    std::vector<int64_t> sq_off;
    int32_t *d_sq_el = nullptr, *d_sq_ax = nullptr, *d_sq_ay = nullptr, *d_sq_az = nullptr;
    uint8_t *d_sq_level = nullptr, *d_sq_clab = nullptr;
    int64_t *d_bt_off = nullptr;
    std::vector<int32_t> sq_nbt;  // background triangles of each INTERCEPTED element (host)
    // bodies of the surface and their convexity; per background-triangle entry
    // the local index of its body at the element, per element the body mask
    // (0: the normal-based filter is off there)
    std::vector<int32_t> comp;
    std::vector<uint8_t> comp_convex;
    int32_t n_comp = 0;
    uint8_t *d_bt_lc = nullptr, *d_sq_nmask = nullptr;
    // learned mode: the INTERCEPTED elements (list positions) at or above the
    // threshold on the background-triangle count, and the others
    int32_t split_bt = -1;
    int sub_cap = -1, rel_cap = 0;  // workgroups per CU beside the gather (side_caps; -1: not yet set)
    int64_t n_sq_net = 0, n_sq_exact = 0;
    int32_t *d_sq_net = nullptr, *d_sq_exact = nullptr;
    int32_t *d_bt_ids = nullptr;
    int32_t *d_sq_cnt = nullptr;
    int64_t *d_sq_off = nullptr;
    uint32_t *d_entries = nullptr;
    int64_t n_subgp = 0;
    // assembly work items over the sub-cell points: at most ITEM_PTS points each
    int64_t n_sub_items = 0;
    std::vector<int32_t> sub_item_el;  // element of each item (host copy)
    std::vector<int32_t> sub_item_cnt; // points of each item (host copy)
    int32_t *d_sub_el = nullptr, *d_sub_cnt = nullptr;
    int64_t *d_sub_off = nullptr;
    std::vector<int32_t> std_el;  // host copy of the OUT-element list
    // weak boundary terms (eq. weakbc): surface Gauss points, one item per
    // element holding points (records after the sub-cell items)
    bool wbc = false;
    double wbc_g[3] = {0, 0, 0};
    int64_t n_surf_items = 0, n_surfgp = 0;
    std::vector<int32_t> surf_item_el;
    std::vector<int64_t> surf_pt_el;  // element of each point (export)
    std::vector<double> surf_xi, surf_w, surf_n;
    int32_t *d_surf_el = nullptr;
    int64_t *d_surf_off = nullptr;
    double *d_surf_xi = nullptr, *d_surf_w = nullptr, *d_surf_n = nullptr, *d_surf_tau = nullptr;
    // inactive nodes (no non-IN element): identity rows
    int64_t n_inact = 0;
    int32_t *d_inact = nullptr;
    // node-level CSR (block rows, block columns) for the product with the matrix
    int64_t *d_nrow_ptr = nullptr;
    int32_t *d_ncol = nullptr;
    // GMRES workspace, allocated by the first solve and grown with the restart
    // length: Krylov basis V ((m + 1) vectors), work vectors, block-Jacobi
    // inverses, multi-dot partial sums and coefficients
    // Dirichlet nodes: CG nodes that are corners of IN elements (host list;
    // device copy made by the first vms_dirichlet_in_nodes)
    std::vector<int32_t> dir_nodes;
    int32_t *d_dir_nodes = nullptr;
    int gm_m = 0;
    double *d_gm_V = nullptr, *d_gm_w = nullptr, *d_gm_z = nullptr, *d_gm_r = nullptr;
    double *d_gm_part = nullptr, *d_gm_h = nullptr, *d_gm_dinv = nullptr;
    int32_t *d_diag_pos = nullptr;
    int *d_gm_bad = nullptr;
    // element-matrix records (one per work item: OUT elements first, then the
    // sub-cell items) and, per CSR block, the list of record blocks summed into it
    int64_t n_slots = 0, n_blocks = 0;
    void *d_em = nullptr;
    // residual records (32 doubles per record) and each node's list of
    // (record, slot) entries, 8 record + slot, ascending
    double *d_rrec = nullptr;
    int64_t *d_roff = nullptr;
    int32_t *d_rlist = nullptr;
    int64_t *d_cb_off = nullptr, *d_vbase = nullptr;
    int32_t *d_contrib = nullptr, *d_vstride = nullptr;
    // the late blocks (records of sub-cell or surface items; flagged VS_LATE
    // in their stride), ascending
    int64_t n_late = 0;
    int64_t *d_late = nullptr;
    // overlapped schedule of the matrix assembly: a second stream of the
    // context (default priority) runs the relabel, the INTERCEPTED items and the
    // surface terms beside the summation of the other blocks; fork / join order
    // it after the OUT elements and before the late blocks
    bool overlap = true, last_split = false;
    // scatter of the element matrices (vms_set_scatter); the atomic mode needs
    // each element's block columns on the device
    uint32_t scatter = VMS_SCATTER_RECORDS;
    uint16_t *d_el_kk = nullptr;
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    // bumped whenever the record buffers and gather lists are rebuilt, so that
    // a batch holding this context re-reads them (and drops a captured graph)
    uint64_t gen = 0;
    // 0: labelled points (set-up pass), 1: degenerate directions, 2: points
    // labelled by the exact test in the last relabel
    unsigned long long *d_counters = nullptr;
    // learned in-out filter of the sub-cell quadrature (prm.inout_mode)
    const vmsm::MlpHandle *mlp = nullptr;
    unsigned int *d_flag = nullptr;            // device-side overflow flag
    double *d_norm = nullptr;
    // optional per-stage timing with events on the context stream (ev[6..8]
    // on the second stream in the overlapped schedule)
    bool timing = false;
    hipEvent_t ev[9] = {};
    uint64_t n_labelled = 0, n_degenerate = 0;
};

namespace {

int fail(vms_ctx *c, int code, const std::string &msg) {
    if (c) c->err = msg;
    set_global_err(msg);
    return code;
}

#define HIPCHK(ctx, expr)                                                                    \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(ctx, VMS_EHIP, std::string("HIP error: ") + hipGetErrorString(e_) + \
                                           " at " #expr);                                    \
    } while (0)

template <typename T>
int upload(vms_ctx *c, T **dst, const std::vector<T> &src) {
    if (c->buf.alloc(dst, src.size())) return fail(c, VMS_ENOMEM, "device allocation failed");
    if (!src.empty())
        HIPCHK(c, hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice,
                                 c->stream));
    return VMS_OK;
}

bool params_ok(const vms_params *p, std::string &why) {
    const double v[6] = {p->rho, p->mu, p->dt, p->theta, p->c_t, p->c_i};
    for (double x : v)
        if (!std::isfinite(x)) { why = "non-finite parameter"; return false; }
    if (p->rho <= 0 || p->dt <= 0 || p->mu < 0 || p->c_t <= 0 || p->c_i < 0 || p->theta < 0 ||
        p->theta > 1) {
        why = "parameter out of range (rho > 0, dt > 0, mu >= 0, c_t > 0, c_i >= 0, 0 <= theta <= 1)";
        return false;
    }
    if (p->inout_mode != VMS_INOUT_EXACT && p->inout_mode != VMS_INOUT_LEARNED &&
        p->inout_mode != VMS_INOUT_NORMAL) {
        why = "unknown in-out mode";
        return false;
    }
    if (p->learned_min_bt < 0) {
        why = "learned_min_bt must be >= 0";
        return false;
    }
    return true;
}

// background triangles of the listed elements: every triangle whose box meets
// the closed element box (same coordinate formula as the device)
void gather_bt(vms_ctx *c, std::vector<int64_t> &off, std::vector<int32_t> &ids) {
    const SurfaceHost &H = c->surf;
    const int64_t nt = H.S.n_tri;
    const int nb = std::max(1, std::min(256, (int)std::ceil(std::cbrt((double)nt) * 2)));
    double inv[3];
    for (int k = 0; k < 3; ++k) {
        double w = H.hi[k] - H.lo[k];
        inv[k] = w > 0 ? nb / w : 0.0;
    }
    auto bin = [&](double v, int k) { return host_bin(v, H.lo[k], inv[k], nb); };
    std::vector<int32_t> cnt((size_t)nb * nb * nb + 1, 0);
    for (int pass = 0; pass < 2; ++pass) {
        static thread_local std::vector<int32_t> fillp;
        if (pass == 1) fillp.assign(cnt.begin(), cnt.end() - 1);
        static thread_local std::vector<int32_t> cell_ids;
        if (pass == 1) cell_ids.assign(cnt.back(), 0);
        for (int64_t t = 0; t < nt; ++t) {
            int r0[3], r1[3];
            for (int k = 0; k < 3; ++k) { r0[k] = bin(H.tbox[6 * t + k], k); r1[k] = bin(H.tbox[6 * t + 3 + k], k); }
            for (int z = r0[2]; z <= r1[2]; ++z)
                for (int y = r0[1]; y <= r1[1]; ++y)
                    for (int x = r0[0]; x <= r1[0]; ++x) {
                        size_t cell = ((size_t)z * nb + y) * nb + x;
                        if (pass == 0) cnt[cell + 1]++;
                        else cell_ids[fillp[cell]++] = (int32_t)t;
                    }
        }
        if (pass == 0) {
            for (size_t i = 1; i < cnt.size(); ++i) cnt[i] += cnt[i - 1];
            continue;
        }
        const int M = c->max_level;
        const double sc = std::ldexp(1.0, -M);
        off.assign(c->n_sq + 1, 0);
        ids.clear();
        std::vector<int32_t> cand;
        for (int64_t i = 0; i < c->n_sq; ++i) {
            const int e = c->sq_el[i];
            const int64_t s = (int64_t)1 << (M - c->level[e]);
            const int64_t A[3] = {c->ax[e], c->ay[e], c->az[e]};
            double lo[3], hi[3];
            for (int k = 0; k < 3; ++k) {
                lo[k] = vmsd::point_coord(c->origin[k], c->root_len, sc, A[k], 0, 0.0);
                hi[k] = vmsd::point_coord(c->origin[k], c->root_len, sc, A[k] + s, 0, 0.0);
            }
            int r0[3], r1[3];
            bool outside = false;
            for (int k = 0; k < 3; ++k) {
                if (hi[k] < H.lo[k] || lo[k] > H.hi[k]) outside = true;
                r0[k] = bin(lo[k], k);
                r1[k] = bin(hi[k], k);
            }
            cand.clear();
            if (!outside)
                for (int z = r0[2]; z <= r1[2]; ++z)
                    for (int y = r0[1]; y <= r1[1]; ++y)
                        for (int x = r0[0]; x <= r1[0]; ++x) {
                            size_t cell = ((size_t)z * nb + y) * nb + x;
                            for (int32_t j = cnt[cell]; j < cnt[cell + 1]; ++j) cand.push_back(cell_ids[j]);
                        }
            std::sort(cand.begin(), cand.end());
            cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
            for (int32_t t : cand) {
                bool meet = true;
                for (int k = 0; k < 3 && meet; ++k)
                    if (H.tbox[6 * t + 3 + k] < lo[k] || H.tbox[6 * t + k] > hi[k]) meet = false;
                if (meet) ids.push_back(t);
            }
            off[i + 1] = (int64_t)ids.size();
        }
    }
}

// sub-cell quadrature on the device, on stream st. At creation: count pass,
// offsets on the host, fill pass. On relabelling: the fill pass alone, which
// recomputes every label and verifies each element's point count on the device
// (a mismatch sets the overflow flag, reported by vms_sizes); no host
// synchronisation.
int run_subquad(vms_ctx *c, bool first, hipStream_t st, int wg_per_cu = 0) {
    if (c->n_sq == 0) return VMS_OK;
    vmsk::GeoArgs g{};
    for (int k = 0; k < 3; ++k) g.origin[k] = c->origin[k];
    g.root_len = c->root_len;
    g.max_level = c->max_level;
    g.depth = c->prm.quad_depth;
    vmsk::SubqArgs a{};
    a.n = c->n_sq;
    a.el = c->d_sq_el;
    a.ax = c->d_sq_ax; a.ay = c->d_sq_ay; a.az = c->d_sq_az;
    a.level = c->d_sq_level;
    a.corner_lab = c->d_sq_clab;
    a.bt_off = c->d_bt_off;
    a.bt_ids = c->d_bt_ids;
    a.cnt = c->d_sq_cnt;
    a.nlabel = c->d_counters;
    a.ndeg = c->d_counters + 1;
    a.flag = c->d_flag;
    if (first) {
        HIPCHK(c, hipMemsetAsync(c->d_counters, 0, 2 * sizeof(unsigned long long), st));
        vmsk::launch_subquad(st, c->surf.S, g, a, 0);
        HIPCHK(c, hipGetLastError());
        std::vector<int32_t> cnt(c->n_sq);
        HIPCHK(c, hipMemcpyAsync(cnt.data(), c->d_sq_cnt, c->n_sq * 4, hipMemcpyDeviceToHost, st));
        unsigned long long ctr[2];
        HIPCHK(c, hipMemcpyAsync(ctr, c->d_counters, sizeof ctr, hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        c->n_labelled = ctr[0];
        c->n_degenerate = ctr[1];
        std::vector<int64_t> off(c->n_sq + 1, 0);
        for (int64_t i = 0; i < c->n_sq; ++i) off[i + 1] = off[i] + cnt[i];
        c->sq_cnt = cnt;
        c->sq_off = off;
        c->n_subgp = off.back();
        if (upload(c, &c->d_sq_off, off)) return VMS_ENOMEM;
        if (c->buf.alloc(&c->d_entries, (size_t)std::max<int64_t>(1, c->n_subgp)))
            return fail(c, VMS_ENOMEM, "device allocation failed (sub-cell points)");
    }
    a.off = c->d_sq_off;
    a.entries = c->d_entries;
    a.nexact = c->d_counters + 2;
    a.normal = (!first && c->prm.inout_mode == VMS_INOUT_NORMAL) ? 1 : 0;
    a.bt_lc = c->d_bt_lc;
    a.nmask = c->d_sq_nmask;
    vmsk::launch_zero_u64(st, a.nexact);
    // the set-up pass is exact; relabels use the learned filter in LEARNED
    // mode on the elements at or above the threshold (their own launch), the
    // exact kernel on the others
    if (!first && c->prm.inout_mode == VMS_INOUT_LEARNED) {
        if (!c->mlp) return fail(c, VMS_EINVAL, "learned in-out mode needs a network (vms_set_inout)");
        if (c->split_bt != c->prm.learned_min_bt) {
            // New element lists. Relabels still in flight on either stream read
            // the old ones, and upload() copies on the context stream while the
            // kernels below may run on the second stream (overlapped schedule,
            // whose fork precedes these copies): wait for both streams before
            // freeing, and for the copies before launching.
            HIPCHK(c, hipStreamSynchronize(c->stream));
            if (st != c->stream) HIPCHK(c, hipStreamSynchronize(st));
            std::vector<int32_t> net, ex;
            for (int64_t i = 0; i < c->n_sq; ++i)
                (c->sq_nbt[i] >= c->prm.learned_min_bt ? net : ex).push_back((int32_t)i);
            c->buf.free(c->d_sq_net);
            c->buf.free(c->d_sq_exact);
            c->d_sq_net = c->d_sq_exact = nullptr;
            if ((net.size() && upload(c, &c->d_sq_net, net)) || (ex.size() && upload(c, &c->d_sq_exact, ex)))
                return fail(c, VMS_ENOMEM, "device allocation failed (element lists)");
            c->n_sq_net = (int64_t)net.size();
            c->n_sq_exact = (int64_t)ex.size();
            c->split_bt = c->prm.learned_min_bt;
            HIPCHK(c, hipStreamSynchronize(c->stream));
        }
        vmsk::SubqArgs ae = a, an = a;
        ae.order = c->d_sq_exact;
        ae.n_order = c->n_sq_exact;
        an.order = c->d_sq_net;
        an.n_order = c->n_sq_net;
        an.learned.net = vmsm::mlp_net(c->mlp);
        an.learned.grid = vmsm::mlp_grid(c->mlp);
        an.learned.margin = vmsm::mlp_margin(c->mlp);
        an.learned.min_bt = 0;
        if (ae.n_order) vmsk::launch_subquad(st, c->surf.S, g, ae, 1, wg_per_cu);
        if (an.n_order) vmsk::launch_subquad(st, c->surf.S, g, an, 1, wg_per_cu);
    } else {
        vmsk::launch_subquad(st, c->surf.S, g, a, 1, wg_per_cu);
    }
    HIPCHK(c, hipGetLastError());
    return VMS_OK;
}

// element data and parameters of the assembly kernels (no work list, no fields)
vmsk::AsmArgs base_args(vms_ctx *c) {
    vmsk::AsmArgs a{};
    a.masters = c->d_masters;
    a.ccode = c->d_ccode;
    a.has_hang = c->d_hang;
    a.level = c->d_level;
    a.depth = c->prm.quad_depth;
    vmsk::set_params(a, c->prm.rho, c->prm.mu, c->prm.dt, c->prm.theta, c->prm.c_t, c->prm.c_i,
                     c->root_len);
    return a;
}

}  // namespace

// Per CSR block, the element-matrix record blocks that sum into it, in
// ascending record order (record r = work item slot * 64 + 8 s + t for master
// slots s, t; slots: OUT elements in list order, then the sub-cell items).
static int build_gather(vms_ctx *c, const std::vector<int32_t> &stdl) {
    const vms::MeshHost &m = c->mesh;
    const std::vector<int32_t> &sub_el = c->sub_item_el;
    const std::vector<int32_t> &surf_el = c->surf_item_el;
    const int64_t n_surf = c->wbc ? c->n_surf_items : 0;
    c->n_slots = c->n_std + c->n_sub_items + n_surf;
    c->n_blocks = m.nrow_ptr[m.n_nodes];
    if (c->n_slots * 64 > INT32_MAX) return fail(c, VMS_EUNSUPPORTED, "too many element-matrix records");
    auto el_of = [&](int64_t slot) {
        return slot < c->n_std ? stdl[slot]
               : (slot < c->n_std + c->n_sub_items ? sub_el[slot - c->n_std]
                                                   : surf_el[slot - c->n_std - c->n_sub_items]);
    };
    // counted and filled on worker threads; each block's list is then sorted,
    // which gives the ascending record order of a serial fill
    std::vector<int64_t> off(c->n_blocks + 1, 0);
    vms::parallel_for(c->n_slots, [&](int64_t b, int64_t f, int) {
        for (int64_t sl = b; sl < f; ++sl) {
            const int64_t e = el_of(sl);
            for (int s = 0; s < 8; ++s) {
                const int ms = m.masters[8 * e + s];
                if (ms < 0) continue;
                for (int t = 0; t < 8; ++t)
                    if (m.masters[8 * e + t] >= 0)
                        __atomic_fetch_add(&off[m.nrow_ptr[ms] + m.el_kk[64 * e + 8 * s + t] + 1], 1,
                                           __ATOMIC_RELAXED);
            }
        }
    });
    for (int64_t b = 0; b < c->n_blocks; ++b) off[b + 1] += off[b];
    std::vector<int32_t> contrib(off[c->n_blocks]);
    {
        std::vector<int64_t> pos(off.begin(), off.end() - 1);
        vms::parallel_for(c->n_slots, [&](int64_t b, int64_t f, int) {
            for (int64_t sl = b; sl < f; ++sl) {
                const int64_t e = el_of(sl);
                for (int s = 0; s < 8; ++s) {
                    const int ms = m.masters[8 * e + s];
                    if (ms < 0) continue;
                    for (int t = 0; t < 8; ++t)
                        if (m.masters[8 * e + t] >= 0) {
                            const int64_t at = __atomic_fetch_add(
                                &pos[m.nrow_ptr[ms] + m.el_kk[64 * e + 8 * s + t]], 1, __ATOMIC_RELAXED);
                            contrib[at] = (int32_t)(sl * 64 + 8 * s + t);
                        }
                }
            }
        });
    }
    vms::parallel_for(c->n_blocks, [&](int64_t b, int64_t f, int) {
        for (int64_t k = b; k < f; ++k)
            if (off[k + 1] - off[k] > 1) std::sort(contrib.begin() + off[k], contrib.begin() + off[k + 1]);
    });
    // CSR place of entry (i, j) of block b in node row n: 16 nrow_ptr[n] + 4 (b - nrow_ptr[n])
    // + i 4 deg(n) + j
    std::vector<int64_t> vbase(c->n_blocks);
    std::vector<int32_t> vstride(c->n_blocks);
    vms::parallel_for(m.n_nodes, [&](int64_t nb, int64_t nf, int) {
        for (int64_t n = nb; n < nf; ++n) {
            const int64_t b0 = m.nrow_ptr[n], deg = m.nrow_ptr[n + 1] - b0;
            for (int64_t b = b0; b < m.nrow_ptr[n + 1]; ++b) {
                vbase[b] = 16 * b0 + 4 * (b - b0);
                vstride[b] = (int32_t)(4 * deg);
            }
            // the diagonal block of a node of no non-IN element (its only
            // block, with no records): the gather writes an identity block
            if (!m.node_active[n]) vstride[b0 + m.diag_pos[n]] = -(int32_t)(4 * deg);
        }
    });
    // late blocks: the last (largest) record of the block's list is not an OUT
    // element's
    const int64_t std_recs = 64 * c->n_std;
    std::vector<int64_t> late;
    {
        const int nt = vms::host_threads();
        std::vector<std::vector<int64_t>> part(nt);
        vms::parallel_for(c->n_blocks, [&](int64_t b, int64_t f, int t) {
            for (int64_t k = b; k < f; ++k)
                if (off[k + 1] > off[k] && contrib[off[k + 1] - 1] >= std_recs) {
                    vstride[k] |= vmsk::VS_LATE;
                    part[t].push_back(k);
                }
        });
        for (auto &v : part) late.insert(late.end(), v.begin(), v.end());  // ranges in order: ascending
    }
    // residual lists: node n receives slot s of every record whose element has
    // master n at slot s (counted, filled, then sorted like the block lists)
    std::vector<int64_t> roff(m.n_nodes + 1, 0);
    vms::parallel_for(c->n_slots, [&](int64_t b, int64_t f, int) {
        for (int64_t sl = b; sl < f; ++sl) {
            const int64_t e = el_of(sl);
            for (int s = 0; s < 8; ++s) {
                const int ms = m.masters[8 * e + s];
                if (ms >= 0) __atomic_fetch_add(&roff[ms + 1], 1, __ATOMIC_RELAXED);
            }
        }
    });
    for (int64_t n = 0; n < m.n_nodes; ++n) roff[n + 1] += roff[n];
    std::vector<int32_t> rlist(roff[m.n_nodes]);
    {
        std::vector<int64_t> pos(roff.begin(), roff.end() - 1);
        vms::parallel_for(c->n_slots, [&](int64_t b, int64_t f, int) {
            for (int64_t sl = b; sl < f; ++sl) {
                const int64_t e = el_of(sl);
                for (int s = 0; s < 8; ++s) {
                    const int ms = m.masters[8 * e + s];
                    if (ms >= 0) rlist[__atomic_fetch_add(&pos[ms], 1, __ATOMIC_RELAXED)] = (int32_t)(8 * sl + s);
                }
            }
        });
    }
    vms::parallel_for(m.n_nodes, [&](int64_t b, int64_t f, int) {
        for (int64_t n = b; n < f; ++n)
            if (roff[n + 1] - roff[n] > 1) std::sort(rlist.begin() + roff[n], rlist.begin() + roff[n + 1]);
    });
    const size_t esz = c->prm.precision == VMS_FP64 ? 8 : 4;
    char *em = nullptr;
    double *rrec = nullptr;
    // a rebuild (weak boundary terms switched) replaces the previous lists
    c->buf.free(c->d_cb_off);
    c->buf.free(c->d_contrib);
    c->buf.free(c->d_vbase);
    c->buf.free(c->d_vstride);
    c->buf.free(c->d_late);
    c->d_late = nullptr;
    c->n_late = (int64_t)late.size();
    c->buf.free(c->d_em);
    c->buf.free(c->d_rrec);
    c->buf.free(c->d_roff);
    c->buf.free(c->d_rlist);
    c->d_em = nullptr;
    c->d_rrec = nullptr;
    if (upload(c, &c->d_cb_off, off) || upload(c, &c->d_contrib, contrib) ||
        upload(c, &c->d_vbase, vbase) || upload(c, &c->d_vstride, vstride) ||
        upload(c, &c->d_roff, roff) || upload(c, &c->d_rlist, rlist) ||
        (c->n_late && upload(c, &c->d_late, late)) ||
        c->buf.alloc(&em, (size_t)std::max<int64_t>(c->n_slots, 1) * 1024 * esz) ||
        c->buf.alloc(&rrec, (size_t)std::max<int64_t>(c->n_slots, 1) * 32 * sizeof(double)))
        return fail(c, VMS_ENOMEM, "device allocation failed (element-matrix records)");
    c->d_em = em;
    c->d_rrec = rrec;
    ++c->gen;
    return VMS_OK;
}

// Surface Gauss points of the weak boundary terms (eq. weakbc): three per
// triangle at barycentric (2/3, 1/6, 1/6) and permutations, a third of the
// area each; each point belongs to the leaf octant that contains it (half-open
// boxes at the finest resolution), points in IN octants are dropped; the
// normal is that of the fluid domain (minus the body's outward normal).
// tau_B = c_b mu / h_b per element, h_b the largest distance from the
// element's OUT corners to the surface, at least h/100 (the remark after the
// equation). Host arithmetic in a fixed order (no contraction) so that points,
// weights and reference coordinates are reproducible bit for bit.
#pragma clang fp contract(off)
static int build_weak_bc(vms_ctx *c, double c_b) {
    const SurfaceHost &H = c->surf;
    const int64_t nt = (int64_t)H.tv.size() / 9, E = (int64_t)c->level.size();
    const int M = c->max_level;
    const double sc = std::ldexp(1.0, M) / c->root_len;
    // leaves of each level, sorted by packed integer corner
    std::vector<std::vector<std::pair<int64_t, int32_t>>> lv(32);
    for (int64_t e = 0; e < E; ++e)
        lv[c->level[e]].push_back({(int64_t)c->ax[e] | ((int64_t)c->ay[e] << 21) | ((int64_t)c->az[e] << 42),
                                   (int32_t)e});
    for (auto &v : lv) std::sort(v.begin(), v.end());
    struct SP { int32_t e; double xi[3], w, n[3]; };
    std::vector<SP> pts;
    pts.reserve(3 * nt);
    const double bary[3][3] = {{2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0}, {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0},
                               {1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0}};
    for (int64_t t = 0; t < nt; ++t) {
        const double *A = &H.tv[9 * t], *B = A + 3, *Cc = A + 6;
        double e1[3], e2[3];
        for (int d = 0; d < 3; ++d) {
            e1[d] = B[d] - A[d];
            e2[d] = Cc[d] - A[d];
        }
        const double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                              e1[0] * e2[1] - e1[1] * e2[0]};
        const double ln = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
        const double w = 0.5 * ln / 3.0;
        for (int k = 0; k < 3; ++k) {
            double x[3];
            int64_t q[3];
            bool inside = true;
            for (int d = 0; d < 3; ++d) {
                const double s0 = bary[k][0] * A[d];
                const double s1 = bary[k][1] * B[d];
                const double s2 = bary[k][2] * Cc[d];
                x[d] = (s0 + s1) + s2;
                q[d] = (int64_t)std::floor((x[d] - c->origin[d]) * sc);
                inside = inside && q[d] >= 0 && q[d] < ((int64_t)1 << M);
            }
            if (!inside) continue;
            int32_t e = -1;
            for (int L = 0; L <= M && e < 0; ++L) {
                const auto &v = lv[L];
                if (v.empty()) continue;
                const int sh = M - L;
                const int64_t key = ((q[0] >> sh) << sh) | (((q[1] >> sh) << sh) << 21) |
                                    (((q[2] >> sh) << sh) << 42);
                auto it = std::lower_bound(v.begin(), v.end(), std::make_pair(key, (int32_t)-1));
                if (it != v.end() && it->first == key) e = it->second;
            }
            if (e < 0 || c->markers[e] == 1) continue;
            SP p;
            p.e = e;
            const double h = c->root_len * ((double)((int64_t)1 << (M - c->level[e])) / (double)((int64_t)1 << M));
            const int32_t Ae[3] = {c->ax[e], c->ay[e], c->az[e]};
            for (int d = 0; d < 3; ++d) {
                const double lo = c->origin[d] + c->root_len * ((double)Ae[d] / (double)((int64_t)1 << M));
                p.xi[d] = 2.0 * (x[d] - lo) / h - 1.0;
                p.n[d] = -cr[d] / ln;
            }
            p.w = w;
            pts.push_back(p);
        }
    }
    std::stable_sort(pts.begin(), pts.end(), [](const SP &a, const SP &b) { return a.e < b.e; });
    // items and h_b from the exact distance of the OUT corners
    std::vector<int32_t> item_el;
    std::vector<int64_t> off;
    for (size_t i = 0; i < pts.size(); ++i)
        if (i == 0 || pts[i].e != pts[i - 1].e) {
            item_el.push_back(pts[i].e);
            off.push_back((int64_t)i);
        }
    off.push_back((int64_t)pts.size());
    const int64_t ni = (int64_t)item_el.size(), np = (int64_t)pts.size();
    std::vector<double> cx, cy, cz;
    std::vector<int64_t> citem;
    for (int64_t k = 0; k < ni; ++k) {
        const int32_t e = item_el[k];
        const double h = c->root_len * ((double)((int64_t)1 << (M - c->level[e])) / (double)((int64_t)1 << M));
        const int32_t Ae[3] = {c->ax[e], c->ay[e], c->az[e]};
        for (int v = 0; v < 8; ++v) {
            if (c->corner_lab[8 * (int64_t)e + v] != 0) continue;
            double p[3];
            for (int d = 0; d < 3; ++d) {
                const double lo = c->origin[d] + c->root_len * ((double)Ae[d] / (double)((int64_t)1 << M));
                p[d] = lo + h * (double)((v >> d) & 1);
            }
            cx.push_back(p[0]);
            cy.push_back(p[1]);
            cz.push_back(p[2]);
            citem.push_back(k);
        }
    }
    std::vector<double> dist(cx.size(), 0.0), hmax(ni, 0.0);
    for (int64_t k = 0; k < ni; ++k)
        hmax[k] = c->root_len * ((double)((int64_t)1 << (M - c->level[item_el[k]])) / (double)((int64_t)1 << M));
    if (!cx.empty()) {
        double trunc = 0.0;
        for (double v : hmax) trunc = std::max(trunc, 4.0 * v);
        DevBuf tmp;
        double *dx, *dy, *dz, *dd;
        const int64_t n = (int64_t)cx.size();
        if (tmp.alloc(&dx, n) || tmp.alloc(&dy, n) || tmp.alloc(&dz, n) || tmp.alloc(&dd, n))
            return fail(c, VMS_ENOMEM, "device allocation failed (surface distances)");
        if (hipMemcpyAsync(dx, cx.data(), n * 8, hipMemcpyHostToDevice, c->stream) ||
            hipMemcpyAsync(dy, cy.data(), n * 8, hipMemcpyHostToDevice, c->stream) ||
            hipMemcpyAsync(dz, cz.data(), n * 8, hipMemcpyHostToDevice, c->stream))
            return fail(c, VMS_EHIP, "device copy failed (surface distances)");
        int rc = vmsm_sdf(c->stream, H.S, H.tv, H.lo, H.hi, dx, dy, dz, n, trunc, dd);
        if (rc) return fail(c, rc, "surface distance kernel failed");
        if (hipMemcpyAsync(dist.data(), dd, n * 8, hipMemcpyDeviceToHost, c->stream) ||
            hipStreamSynchronize(c->stream))
            return fail(c, VMS_EHIP, "device copy failed (surface distances)");
    }
    std::vector<double> hb(ni, 0.0), tau(ni);
    for (size_t i = 0; i < dist.size(); ++i) hb[citem[i]] = std::max(hb[citem[i]], std::fabs(dist[i]));
    for (int64_t k = 0; k < ni; ++k) tau[k] = c_b * c->prm.mu / std::max(hb[k], 0.01 * hmax[k]);
    c->n_surf_items = ni;
    c->n_surfgp = np;
    c->surf_item_el = item_el;
    c->surf_pt_el.resize(np);
    c->surf_xi.resize(3 * np);
    c->surf_w.resize(np);
    c->surf_n.resize(3 * np);
    for (int64_t i = 0; i < np; ++i) {
        c->surf_pt_el[i] = pts[i].e;
        c->surf_w[i] = pts[i].w;
        for (int d = 0; d < 3; ++d) {
            c->surf_xi[3 * i + d] = pts[i].xi[d];
            c->surf_n[3 * i + d] = pts[i].n[d];
        }
    }
    for (void *p : {(void *)c->d_surf_el, (void *)c->d_surf_off, (void *)c->d_surf_xi, (void *)c->d_surf_w,
                    (void *)c->d_surf_n, (void *)c->d_surf_tau})
        c->buf.free(p);
    if (upload(c, &c->d_surf_el, item_el) || upload(c, &c->d_surf_off, off) ||
        upload(c, &c->d_surf_xi, c->surf_xi) || upload(c, &c->d_surf_w, c->surf_w) ||
        upload(c, &c->d_surf_n, c->surf_n) || upload(c, &c->d_surf_tau, tau))
        return VMS_ENOMEM;
    return VMS_OK;
}
#pragma clang fp contract(on)

static vmsk::SurfArgs surf_args(vms_ctx *c, const double *const fp[7], double *resid) {
    vmsk::SurfArgs s{};
    s.masters = c->d_masters;
    s.ccode = c->d_ccode;
    s.has_hang = c->d_hang;
    s.level = c->d_level;
    s.n_items = c->n_surf_items;
    s.items = c->d_surf_el;
    s.pt_off = c->d_surf_off;
    s.xi = c->d_surf_xi;
    s.w = c->d_surf_w;
    s.n = c->d_surf_n;
    s.tau = c->d_surf_tau;
    for (int k = 0; k < 7; ++k) s.f[k] = fp[k];
    s.rho = c->prm.rho;
    s.mu = c->prm.mu;
    s.theta = c->prm.theta;
    s.root_len = c->root_len;
    for (int k = 0; k < 3; ++k) s.g[k] = c->wbc_g[k];
    s.rrec = resid ? c->d_rrec : nullptr;
    s.em = c->d_em;
    s.slot0 = c->n_std + c->n_sub_items;
    return s;
}

// residual (or Jacobian action) = sums of the residual records by node
static void gather_resid(vms_ctx *c, hipStream_t st, double *out) {
    vmsk::launch_res_gather(st, c->d_rrec, c->d_roff, c->d_rlist, c->mesh.n_nodes, out);
}

// CSR values = sums of the element-matrix records; the identity blocks of
// inactive nodes are written by the same gather
static void gather_csr(vms_ctx *c, hipStream_t st, void *vals) {
    if (c->prm.precision == VMS_FP64)
        vmsk::launch_gather_f64(st, (const double *)c->d_em, c->d_cb_off, c->d_contrib, c->d_vbase,
                                c->d_vstride, c->n_blocks, (double *)vals);
    else
        vmsk::launch_gather_f32(st, (const float *)c->d_em, c->d_cb_off, c->d_contrib, c->d_vbase,
                                c->d_vstride, c->n_blocks, (float *)vals);
}

extern "C" {

const char *vms_last_error(vms_ctx *ctx) {
    if (ctx) return ctx->err.c_str();
    std::lock_guard<std::mutex> lk(g_err_mu);
    return g_err.c_str();
}

void vms_destroy(vms_ctx *ctx) {
    if (!ctx) return;
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    if (ctx->side) {
        (void)hipStreamSynchronize(ctx->side);
        (void)hipStreamDestroy(ctx->side);
    }
    for (hipEvent_t e : {ctx->fork, ctx->join})
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t &e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    delete ctx;
}

// Set-up stage times on stderr when the environment sets VMS_SETUP_LOG (the
// host mesh work of a 10^7-octant tree takes tens of seconds).
struct StageLog {
    bool on = std::getenv("VMS_SETUP_LOG") != nullptr;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now(), t = t0;
    void operator()(const char *what) {
        if (!on) return;
        const auto n = std::chrono::steady_clock::now();
        std::fprintf(stderr, "[vms setup] %-28s %8.2f s (total %8.2f s)\n", what,
                     std::chrono::duration<double>(n - t).count(), std::chrono::duration<double>(n - t0).count());
        std::fflush(stderr);
        t = n;
    }
};

int vms_create(vms_ctx **out, const vms_octree *tree, const vms_surface *surf,
               const vms_params *prm, void *stream) {
    if (!out) return fail(nullptr, VMS_EINVAL, "null output pointer");
    *out = nullptr;
    if (!tree || !prm || !tree->ax || !tree->ay || !tree->az || !tree->level || tree->n_oct <= 0)
        return fail(nullptr, VMS_EINVAL, "null or empty octree");
    if (tree->max_level < 0 || tree->max_level > 20)
        return fail(nullptr, VMS_EUNSUPPORTED, "max_level must be in [0, 20]");
    if (tree->n_oct >= ((int64_t)1 << 31)) return fail(nullptr, VMS_EUNSUPPORTED, "more than 2^31 octants");
    std::string why;
    if (!params_ok(prm, why)) return fail(nullptr, VMS_EINVAL, why);
    if (prm->quad_depth < 0 || prm->quad_depth > 3)
        return fail(nullptr, VMS_EUNSUPPORTED, "quad_depth must be in [0, 3]");
    if (prm->precision > VMS_MIXED_FP16) return fail(nullptr, VMS_EUNSUPPORTED, "unknown precision");
    if (!std::isfinite(tree->root_len) || tree->root_len <= 0)
        return fail(nullptr, VMS_EINVAL, "root_len must be positive");

    vms_ctx *c = new vms_ctx();
    c->stream = (hipStream_t)stream;
    c->prm = *prm;
    for (int k = 0; k < 3; ++k) c->origin[k] = tree->origin[k];
    c->root_len = tree->root_len;
    c->max_level = tree->max_level;
    const int64_t E = tree->n_oct;
    c->ax.assign(tree->ax, tree->ax + E);
    c->ay.assign(tree->ay, tree->ay + E);
    c->az.assign(tree->az, tree->az + E);
    c->level.assign(tree->level, tree->level + E);
    auto bail = [&](int code) {
        set_global_err(c->err);
        delete c;
        return code;
    };

    std::string err;
    int rc;
    if (surf) {  // host-side validation first: no device work for a bad surface
        if (surf->n_tri <= 0 || surf->n_vert <= 0 || !surf->verts || !surf->tri) {
            c->err = "empty or null surface";
            return bail(VMS_EINVAL);
        }
        rc = check_watertight(surf, err);
        if (rc) { c->err = err; return bail(rc); }
    }
    StageLog stage;
    vms::TreeIn ti{E, c->ax.data(), c->ay.data(), c->az.data(), c->level.data(), tree->max_level};
    rc = vms::derive_mesh(ti, c->mesh, err);
    stage("nodes and constraints");
    if (rc) { c->err = err; return bail(rc == -2 ? VMS_EMESH : VMS_EINVAL); }
    vms::MeshHost &m = c->mesh;
    if (c->buf.alloc(&c->d_counters, 4) || c->buf.alloc(&c->d_norm, 1) ||
        c->buf.alloc(&c->d_flag, 1) || hipMemsetAsync(c->d_flag, 0, 4, c->stream) != hipSuccess) {
        c->err = "device allocation failed";
        return bail(VMS_ENOMEM);
    }

    // ---- markers (Alg. 4) from exact corner labels
    c->markers.assign(E, 0);
    c->corner_lab.assign((size_t)E * 8, 0);
    if (surf) {
        rc = build_surface(surf, c->stream, c->surf, err);
        if (rc) { c->err = err; return bail(rc); }
        c->has_surf = true;
        // bodies and their convexity (exact orientation of every edge's far vertex)
        {
            std::vector<int32_t> t1, t2;
            std::vector<int8_t> cor;
            rc = vms::surface_components(surf, c->comp, c->n_comp, &t1, &t2, &cor, err);
            if (rc) { c->err = err; return bail(rc); }
            const int64_t ne = (int64_t)t1.size();
            DevBuf eb;
            int32_t *d1, *d2;
            int8_t *dc;
            uint8_t *dbad;
            std::vector<uint8_t> bad(ne);
            if (eb.alloc(&d1, std::max<int64_t>(ne, 1)) || eb.alloc(&d2, std::max<int64_t>(ne, 1)) ||
                eb.alloc(&dc, std::max<int64_t>(ne, 1)) || eb.alloc(&dbad, std::max<int64_t>(ne, 1))) {
                c->err = "device allocation failed (convexity)";
                return bail(VMS_ENOMEM);
            }
            if (ne && (hipMemcpyAsync(d1, t1.data(), ne * 4, hipMemcpyHostToDevice, c->stream) ||
                       hipMemcpyAsync(d2, t2.data(), ne * 4, hipMemcpyHostToDevice, c->stream) ||
                       hipMemcpyAsync(dc, cor.data(), ne, hipMemcpyHostToDevice, c->stream))) {
                c->err = "device copy failed (convexity)";
                return bail(VMS_EHIP);
            }
            vmsk::launch_edge_convex(c->stream, c->surf.S, d1, d2, dc, ne, dbad);
            if (hipGetLastError() != hipSuccess ||
                (ne && hipMemcpyAsync(bad.data(), dbad, ne, hipMemcpyDeviceToHost, c->stream)) ||
                hipStreamSynchronize(c->stream)) {
                c->err = "convexity kernel failed";
                return bail(VMS_EHIP);
            }
            c->comp_convex.assign(c->n_comp, 1);
            for (int64_t e = 0; e < ne; ++e)
                if (bad[e]) c->comp_convex[c->comp[t1[e]]] = 0;
        }
        const int64_t NV = (int64_t)m.vert_key.size();
        std::vector<int32_t> ix(NV), iy(NV), iz(NV);
        for (int64_t v = 0; v < NV; ++v) {
            int64_t x, y, z;
            vms::unmorton3(m.vert_key[v], x, y, z);
            ix[v] = (int32_t)x; iy[v] = (int32_t)y; iz[v] = (int32_t)z;
        }
        DevBuf tmp;
        int32_t *dix, *diy, *diz;
        uint8_t *dlab;
        if (tmp.alloc(&dix, NV) || tmp.alloc(&diy, NV) || tmp.alloc(&diz, NV) || tmp.alloc(&dlab, NV)) {
            c->err = "device allocation failed (vertex labels)";
            return bail(VMS_ENOMEM);
        }
        std::vector<uint8_t> vlab(NV);
        vmsk::GeoArgs g{};
        for (int k = 0; k < 3; ++k) g.origin[k] = c->origin[k];
        g.root_len = c->root_len;
        g.max_level = c->max_level;
        g.depth = prm->quad_depth;
        if (hipMemcpyAsync(dix, ix.data(), NV * 4, hipMemcpyHostToDevice, c->stream) ||
            hipMemcpyAsync(diy, iy.data(), NV * 4, hipMemcpyHostToDevice, c->stream) ||
            hipMemcpyAsync(diz, iz.data(), NV * 4, hipMemcpyHostToDevice, c->stream) ||
            hipMemsetAsync(c->d_counters, 0, 32, c->stream)) {
            c->err = "device copy failed (vertex labels)";
            return bail(VMS_EHIP);
        }
        vmsk::launch_vertex_labels(c->stream, c->surf.S, g, NV, dix, diy, diz, dlab, c->d_counters + 1);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(vlab.data(), dlab, NV, hipMemcpyDeviceToHost, c->stream) ||
            hipStreamSynchronize(c->stream)) {
            c->err = "vertex label kernel failed";
            return bail(VMS_EHIP);
        }
        for (int64_t e = 0; e < E; ++e) {
            int nin = 0;
            for (int a = 0; a < 8; ++a) {
                uint8_t l = vlab[m.elem_vert[8 * e + a]];
                c->corner_lab[8 * e + a] = l;
                nin += l;
            }
            c->markers[e] = nin == 8 ? 1 : (nin == 0 ? 0 : 2);
        }
    }

    // Dirichlet nodes: independent vertices among the corners of IN elements
    for (int64_t e = 0; e < E; ++e) {
        if (c->markers[e] != 1) continue;
        for (int a = 0; a < 8; ++a) {
            const int32_t v = m.elem_vert[8 * e + a];
            if (m.vert_type[v] != 1) continue;
            const auto it = std::lower_bound(m.node_key.begin(), m.node_key.end(), m.vert_key[v]);
            c->dir_nodes.push_back((int32_t)(it - m.node_key.begin()));
        }
    }
    std::sort(c->dir_nodes.begin(), c->dir_nodes.end());
    c->dir_nodes.erase(std::unique(c->dir_nodes.begin(), c->dir_nodes.end()), c->dir_nodes.end());
    stage("corner labels and markers");
    // ---- intercepted elements: background triangles, sub-cell quadrature
    for (int64_t e = 0; e < E; ++e)
        if (c->markers[e] == 2) c->sq_el.push_back((int32_t)e);
    c->n_sq = (int64_t)c->sq_el.size();
    if (c->n_sq) {
        std::vector<int64_t> bt_off;
        std::vector<int32_t> bt_ids;
        gather_bt(c, bt_off, bt_ids);
        c->sq_nbt.resize(c->n_sq);
        for (int64_t i = 0; i < c->n_sq; ++i) c->sq_nbt[i] = (int32_t)(bt_off[i + 1] - bt_off[i]);
        // bodies at each element for the normal-based filter: local index of
        // each background triangle's body (first appearance), mask of the
        // element's bodies; 0 (filter off) with a non-convex body or more than 8
        std::vector<uint8_t> bt_lc(std::max<size_t>(bt_ids.size(), 1), 0), nmask(c->n_sq, 0);
        for (int64_t i = 0; i < c->n_sq; ++i) {
            int32_t loc[8];
            int nl = 0;
            bool ok = true;
            for (int64_t j = bt_off[i]; j < bt_off[i + 1] && ok; ++j) {
                const int32_t cid = c->comp[bt_ids[j]];
                int k = 0;
                while (k < nl && loc[k] != cid) ++k;
                if (k == nl) {
                    if (nl == 8 || !c->comp_convex[cid]) ok = false;
                    else loc[nl++] = cid;
                }
                if (ok) bt_lc[j] = (uint8_t)k;
            }
            nmask[i] = ok && nl ? (uint8_t)((1u << nl) - 1u) : 0;
        }
        std::vector<int32_t> sax(c->n_sq), say(c->n_sq), saz(c->n_sq);
        std::vector<uint8_t> slev(c->n_sq), sclab(8 * c->n_sq);
        for (int64_t i = 0; i < c->n_sq; ++i) {
            int e = c->sq_el[i];
            sax[i] = c->ax[e]; say[i] = c->ay[e]; saz[i] = c->az[e]; slev[i] = c->level[e];
            for (int a = 0; a < 8; ++a) sclab[8 * i + a] = c->corner_lab[8 * e + a];
        }
        if (upload(c, &c->d_sq_el, c->sq_el) || upload(c, &c->d_sq_ax, sax) ||
            upload(c, &c->d_sq_ay, say) || upload(c, &c->d_sq_az, saz) ||
            upload(c, &c->d_sq_level, slev) || upload(c, &c->d_sq_clab, sclab) ||
            upload(c, &c->d_bt_off, bt_off) || upload(c, &c->d_bt_ids, bt_ids) ||
            upload(c, &c->d_bt_lc, bt_lc) || upload(c, &c->d_sq_nmask, nmask) ||
            c->buf.alloc(&c->d_sq_cnt, c->n_sq))
            return bail(VMS_ENOMEM);
        stage("background triangles");
        rc = run_subquad(c, true, c->stream);
        if (rc) return bail(rc);
        stage("sub-cell quadrature");
        // split every element's point list into work items of at most ITEM_PTS
        // points (each item writes its own record; the gathers sum them)
        const int ITEM_PTS = VMS_ITEM_PTS;
        std::vector<int32_t> iel, icnt;
        std::vector<int64_t> ioff;
        for (int64_t i = 0; i < c->n_sq; ++i)
            for (int64_t p = 0; p < c->sq_cnt[i]; p += ITEM_PTS) {
                iel.push_back(c->sq_el[i]);
                ioff.push_back(c->sq_off[i] + p);
                icnt.push_back((int32_t)std::min<int64_t>(ITEM_PTS, c->sq_cnt[i] - p));
            }
        c->n_sub_items = (int64_t)iel.size();
        c->sub_item_el = iel;
        c->sub_item_cnt = icnt;
        if (upload(c, &c->d_sub_el, iel) || upload(c, &c->d_sub_off, ioff) ||
            upload(c, &c->d_sub_cnt, icnt))
            return bail(VMS_ENOMEM);
    }

    // ---- CSR pattern over non-IN elements
    std::vector<uint8_t> active(E);
    for (int64_t e = 0; e < E; ++e) active[e] = c->markers[e] != 1;
    rc = vms::build_pattern(m, active, err);
    if (rc) { c->err = err; return bail(rc == -6 ? VMS_EUNSUPPORTED : VMS_EINVAL); }
    stage("CSR pattern");

    // ---- device element data and work lists
    std::vector<int32_t> stdl, cutl;
    for (int64_t e = 0; e < E; ++e)
        if (c->markers[e] == 0) stdl.push_back((int32_t)e);
    c->n_std = (int64_t)stdl.size();
    std::vector<int32_t> inact;
    for (int64_t n = 0; n < m.n_nodes; ++n)
        if (!m.node_active[n]) inact.push_back((int32_t)n);
    c->n_inact = (int64_t)inact.size();
    if (upload(c, &c->d_masters, m.masters) || upload(c, &c->d_ccode, m.ccode) ||
        upload(c, &c->d_hang, m.has_hang) || upload(c, &c->d_level, c->level) ||
        upload(c, &c->d_std, stdl) ||
        upload(c, &c->d_inact, inact) || upload(c, &c->d_nrow_ptr, m.nrow_ptr) ||
        upload(c, &c->d_ncol, m.ncol))
        return bail(VMS_ENOMEM);
    c->std_el = stdl;
    stage("element data upload");
    rc = build_gather(c, stdl);
    if (rc) return bail(rc);
    stage("record gather lists");
    if (hipStreamSynchronize(c->stream) != hipSuccess) {
        c->err = "device synchronisation failed at create";
        return bail(VMS_EHIP);
    }
    *out = c;
    return VMS_OK;
}

int vms_sizes(vms_ctx *c, int64_t *n_nodes, int64_t *n_rows, int64_t *nnz, int64_t *n_subgp) {
    if (!c) return fail(nullptr, VMS_EINVAL, "null context");
    unsigned int flag = 0;
    HIPCHK(c, hipMemcpyAsync(&flag, c->d_flag, 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (flag) return fail(c, VMS_EOVERFLOW, "relabelling changed the sub-cell point count of an element");
    if (n_nodes) *n_nodes = c->mesh.n_nodes;
    if (n_rows) *n_rows = 4 * c->mesh.n_nodes;
    if (nnz) *nnz = c->mesh.nnz;
    if (n_subgp) *n_subgp = c->n_subgp;
    return VMS_OK;
}

int vms_export(vms_ctx *c, uint32_t what, void *dst) {
    if (!c || !dst) return fail(c, VMS_EINVAL, "null context or destination");
    const vms::MeshHost &m = c->mesh;
    const int64_t E = m.n_el;
    switch (what) {
        case VMS_EXPORT_NODE_XYZ: {
            int32_t *d = (int32_t *)dst;
            for (int64_t n = 0; n < m.n_nodes; ++n) {
                int64_t x, y, z;
                vms::unmorton3(m.node_key[n], x, y, z);
                d[n] = (int32_t)x; d[m.n_nodes + n] = (int32_t)y; d[2 * m.n_nodes + n] = (int32_t)z;
            }
            return VMS_OK;
        }
        case VMS_EXPORT_ROW_PTR:
            std::memcpy(dst, m.row_ptr.data(), m.row_ptr.size() * 8);
            return VMS_OK;
        case VMS_EXPORT_COL_IDX:
            vms::fill_col_idx(m, (int32_t *)dst);
            return VMS_OK;
        case VMS_EXPORT_NODE_ROW_PTR:
            std::memcpy(dst, m.nrow_ptr.data(), m.nrow_ptr.size() * 8);
            return VMS_OK;
        case VMS_EXPORT_NODE_COL:
            std::memcpy(dst, m.ncol.data(), m.ncol.size() * 4);
            return VMS_OK;
        case VMS_EXPORT_MARKERS:
            std::memcpy(dst, c->markers.data(), E);
            return VMS_OK;
        case VMS_EXPORT_VERTEX_LAB:
            std::memcpy(dst, c->corner_lab.data(), 8 * E);
            return VMS_OK;
        case VMS_EXPORT_MASTERS:
            std::memcpy(dst, m.masters.data(), 8 * E * 4);
            return VMS_OK;
        case VMS_EXPORT_SURFGP: {
            // int64 element, 3 doubles xi, weight, 3 doubles normal per point
            const int64_t n = c->wbc ? c->n_surfgp : 0;
            char *o = (char *)dst;
            if (n) {
                std::memcpy(o, c->surf_pt_el.data(), 8 * n);
                std::memcpy(o + 8 * n, c->surf_xi.data(), 24 * n);
                std::memcpy(o + 32 * n, c->surf_w.data(), 8 * n);
                std::memcpy(o + 40 * n, c->surf_n.data(), 24 * n);
            }
            return VMS_OK;
        }
        case VMS_EXPORT_SUBGP: {
            const int64_t n = c->n_subgp;
            std::vector<uint32_t> ent(n);
            if (n) {
                HIPCHK(c, hipMemcpyAsync(ent.data(), c->d_entries, n * 4, hipMemcpyDeviceToHost, c->stream));
                HIPCHK(c, hipStreamSynchronize(c->stream));
            }
            int64_t *o_el = (int64_t *)dst;
            int32_t *o_key = (int32_t *)((char *)dst + 8 * n);
            uint8_t *o_lvl = (uint8_t *)((char *)dst + 12 * n);
            double *o_xyz = (double *)((char *)dst + 13 * n);
            const int D = c->prm.quad_depth, M = c->max_level;
            const double scF = std::ldexp(1.0, -(M + D));
            for (int64_t i = 0; i < c->n_sq; ++i) {
                const int e = c->sq_el[i];
                const int64_t SE = (int64_t)1 << (M - c->level[e] + D);
                const int64_t A0[3] = {(int64_t)c->ax[e] << D, (int64_t)c->ay[e] << D, (int64_t)c->az[e] << D};
                for (int64_t p = c->sq_off[i]; p < c->sq_off[i + 1]; ++p) {
                    uint32_t en = ent[p];
                    int l = en & 3;
                    uint32_t key = en >> 2;
                    int gp = (key >> (3 * (D - l))) & 7;
                    int64_t A[3] = {A0[0], A0[1], A0[2]};
                    for (int k = 1; k <= l; ++k) {
                        uint32_t dg = (key >> (3 * (D - k + 1))) & 7u;
                        for (int ax = 0; ax < 3; ++ax)
                            if ((dg >> ax) & 1u) A[ax] += SE >> k;
                    }
                    o_el[p] = e;
                    o_key[p] = (int32_t)key;
                    o_lvl[p] = (uint8_t)l;
                    double xyz[3];
                    for (int ax = 0; ax < 3; ++ax)
                        xyz[ax] = vmsd::point_coord(c->origin[ax], c->root_len, scF, A[ax], SE >> l,
                                                    ((gp >> ax) & 1) ? VMS_GP : VMS_GM);
                    std::memcpy(o_xyz + 3 * p, xyz, sizeof xyz);
                }
            }
            return VMS_OK;
        }
        default:
            return fail(c, VMS_EINVAL, "unknown export selector");
    }
}

static int ensure_diag_pos(vms_ctx *c);

// the second stream of the overlapped schedule and its events (made on first use)
static int ensure_side(vms_ctx *c) {
    if (!c->side) HIPCHK(c, hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
    if (!c->fork) HIPCHK(c, hipEventCreateWithFlags(&c->fork, hipEventDisableTiming));
    if (!c->join) HIPCHK(c, hipEventCreateWithFlags(&c->join, hipEventDisableTiming));
    return VMS_OK;
}

// One assembly. In order on the context stream: relabel (if asked), OUT
// elements, INTERCEPTED items, surface terms, CSR blocks, residual. With the
// matrix and any late work, the overlapped schedule instead forks the relabel,
// the INTERCEPTED items and the surface terms onto the second stream once the
// OUT elements are done, sums the blocks without late records meanwhile, joins,
// and sums the late blocks; every block is summed by the same code in the same
// order either way, so the outputs are identical.
// Workgroups per CU of the second stream's kernels (exact relabel, sub-cell
// items) while they run beside the CSR gather in the overlapped schedule. The
// gather is bound by HBM and needs many waves in flight; the second stream's
// kernels are latency-bound and lose little when fewer of their waves are
// resident. When their estimated work fits well inside the gather's (under
// 0.8 of it), the sub-cell items keep ceil(w/2) of their w waves per SIMD and
// the relabel a third of its workgroups per CU (the choices that measured
// best on MI355X); otherwise neither is limited. Estimates from rates measured
// on this GPU: 0.51 ns per sub-cell point over the whole GPU in FP64, 0.33 ns
// in the mixed forms, 1.5e10 exact labels per second in the relabel, the
// gather's bytes (records read, values written) at 4.7 TB/s (FP64 values) or
// 4.0 TB/s (FP32). 0 = no limit.
static void side_caps(vms_ctx *c, bool relabel, int &items_cap, int &relabel_cap) {
    items_cap = relabel_cap = 0;
    const bool fp64 = c->prm.precision == VMS_FP64;
    const double vb = fp64 ? 8.0 : 4.0;
    const double t_items = (double)c->n_subgp * (fp64 ? 0.51e-9 : 0.33e-9);
    const double t_rel = relabel ? (double)c->n_labelled / 1.5e10 : 0.0;
    const double recs = (double)(c->n_std + c->n_sub_items);
    const double t_gather = (recs * 1024.0 + (double)c->mesh.nnz) * vb / (fp64 ? 4.7e12 : 4.0e12);
    if (!(t_items + t_rel < 0.8 * t_gather)) return;
    if (c->sub_cap < 0) {
        const int per_cu = vmsk::sub_items_per_cu(fp64 ? 0 : (c->prm.precision == VMS_MIXED_BF16 ? 1 : 2));
        const int w = per_cu / 4;  // waves per SIMD: one-wave workgroups, 4 SIMDs per CU
        c->sub_cap = w >= 2 ? 4 * ((w + 1) / 2) : 0;
        const int sq = vmsk::subquad_per_cu();
        // caps of 3 or more keep a capped workgroup within 64 KB of LDS
        c->rel_cap = sq >= 9 ? (sq + 2) / 3 : 0;
    }
    items_cap = c->sub_cap;
    relabel_cap = relabel ? c->rel_cap : 0;
}

static int assemble_impl(vms_ctx *c, const vms_fields *f, void *vals, double *resid, uint32_t flags,
                         bool mat) {
    if (!c || !f) return fail(c, VMS_EINVAL, "null context or fields");
    if (mat && !vals) return fail(c, VMS_EINVAL, "null csr_vals");
    if (!mat && !resid) return fail(c, VMS_EINVAL, "null resid");
    const double *fp[7] = {f->ux, f->uy, f->uz, f->p, f->ux0, f->uy0, f->uz0};
    for (const double *p : fp)
        if (!p) return fail(c, VMS_EINVAL, "null field pointer");
    const bool relabel = (flags & VMS_RELABEL) && c->has_surf;
    const bool late_work = c->n_sub_items > 0 || (c->wbc && c->n_surf_items > 0);
    const bool atomic = mat && c->scatter == VMS_SCATTER_ATOMIC;
    const bool split = mat && c->overlap && late_work && !atomic;
    if (split) {
        int rc = ensure_side(c);
        if (rc) return rc;
    }
    hipStream_t ms = c->stream, ls = split ? c->side : c->stream;
    c->last_split = split;
    int items_cap = 0, relabel_cap = 0;
    if (split) side_caps(c, relabel, items_cap, relabel_cap);
    if (c->timing) HIPCHK(c, hipEventRecord(c->ev[0], ms));
    if (relabel && !split) {
        int rc = run_subquad(c, false, ms);
        if (rc) return rc;
    }
    if (c->timing) HIPCHK(c, hipEventRecord(c->ev[1], ms));
    const bool fp64 = c->prm.precision == VMS_FP64;
    vmsk::AsmArgs a = base_args(c);
    for (int k = 0; k < 7; ++k) a.f[k] = fp[k];
    a.rrec = resid ? c->d_rrec : nullptr;
    a.em = c->d_em;
    a.slot0 = 0;
    if (atomic) {
        // the values start at zero; the kernels add every element matrix into them
        if (fp64) vmsk::launch_fill_f64(ms, (double *)vals, c->mesh.nrow_ptr[c->mesh.n_nodes] * 16, 0.0);
        else vmsk::launch_fill_f32(ms, (float *)vals, c->mesh.nrow_ptr[c->mesh.n_nodes] * 16, 0.0f);
        HIPCHK(c, hipGetLastError());
        a.vals = vals;
        a.nrow_ptr = c->d_nrow_ptr;
        a.el_kk = c->d_el_kk;
    }
    if (c->timing) HIPCHK(c, hipEventRecord(c->ev[2], ms));
    // OUT elements: 2x2x2 Gauss points
    a.n_items = c->n_std;
    a.items = c->d_std;
    if (fp64) vmsk::launch_assemble_f64(ms, a, false, mat);
    else vmsk::launch_assemble_mixed(ms, a, false, mat, c->prm.precision == VMS_MIXED_FP16);
    HIPCHK(c, hipGetLastError());
    if (c->timing) HIPCHK(c, hipEventRecord(c->ev[3], ms));
    int late_rc = VMS_OK;
    if (split) {
        HIPCHK(c, hipEventRecord(c->fork, ms));
        HIPCHK(c, hipStreamWaitEvent(ls, c->fork, 0));
        if (c->timing) HIPCHK(c, hipEventRecord(c->ev[6], ls));
        if (relabel) late_rc = run_subquad(c, false, ls, relabel_cap);
        if (c->timing) HIPCHK(c, hipEventRecord(c->ev[7], ls));
    }
    // INTERCEPTED elements: kept sub-cell points
    if (late_rc == VMS_OK && c->n_sub_items) {
        a.n_items = c->n_sub_items;
        a.items = c->d_sub_el;
        a.pt_off = c->d_sub_off;
        a.pt_cnt = c->d_sub_cnt;
        a.entries = c->d_entries;
        a.slot0 = c->n_std;
        if (fp64) vmsk::launch_assemble_f64(ls, a, true, mat, items_cap);
        else vmsk::launch_assemble_mixed(ls, a, true, mat, c->prm.precision == VMS_MIXED_FP16, items_cap);
        HIPCHK(c, hipGetLastError());
    }
    if (late_rc == VMS_OK && c->wbc && c->n_surf_items) {
        // weak boundary terms: records after the sub-cell items
        vmsk::launch_surface(ls, surf_args(c, fp, resid), mat ? 0 : 1, fp64, nullptr);
        HIPCHK(c, hipGetLastError());
    }
    const void *em = c->d_em;
    if (split) {
        if (c->timing) HIPCHK(c, hipEventRecord(c->ev[8], ls));
        HIPCHK(c, hipEventRecord(c->join, ls));
        if (late_rc == VMS_OK) {
            if (fp64)
                vmsk::launch_gather_f64(ms, (const double *)em, c->d_cb_off, c->d_contrib, c->d_vbase,
                                        c->d_vstride, c->n_blocks, (double *)vals, true);
            else
                vmsk::launch_gather_f32(ms, (const float *)em, c->d_cb_off, c->d_contrib, c->d_vbase,
                                        c->d_vstride, c->n_blocks, (float *)vals, true);
        }
        HIPCHK(c, hipStreamWaitEvent(ms, c->join, 0));
        if (late_rc) return late_rc;
        vmsk::launch_gather_list(ms, fp64, em, c->d_cb_off, c->d_contrib, c->d_vbase, c->d_vstride, c->d_late,
                                 c->n_late, vals);
    } else {
        if (c->timing) HIPCHK(c, hipEventRecord(c->ev[4], ms));
        if (atomic) {
            // identity blocks of the inactive nodes (no element adds to them)
            if (fp64)
                vmsk::launch_dirichlet_rows_f64(ms, (double *)vals, c->d_nrow_ptr, c->d_diag_pos, c->d_inact,
                                                c->n_inact, nullptr);
            else
                vmsk::launch_dirichlet_rows_f32(ms, (float *)vals, c->d_nrow_ptr, c->d_diag_pos, c->d_inact,
                                                c->n_inact, nullptr);
        } else if (mat) {
            gather_csr(c, ms, vals);
        }
    }
    if (resid) gather_resid(c, ms, resid);
    HIPCHK(c, hipGetLastError());
    if (c->timing) HIPCHK(c, hipEventRecord(c->ev[5], ms));
    return VMS_OK;
}

int vms_set_timing(vms_ctx *c, int on) {
    if (!c) return fail(nullptr, VMS_EINVAL, "null context");
    if (on)
        for (hipEvent_t &e : c->ev)
            if (!e) HIPCHK(c, hipEventCreate(&e));
    c->timing = on != 0;
    return VMS_OK;
}

int vms_last_timing(vms_ctx *c, float *ms) {
    if (!c || !ms) return fail(c, VMS_EINVAL, "null argument");
    if (!c->timing) return fail(c, VMS_EINVAL, "timing is off");
    HIPCHK(c, hipEventSynchronize(c->ev[5]));
    if (c->last_split) {
        // relabel and late items on the second stream; [4] from the end of the
        // OUT elements to the end of the call
        HIPCHK(c, hipEventElapsedTime(&ms[0], c->ev[6], c->ev[7]));
        HIPCHK(c, hipEventElapsedTime(&ms[1], c->ev[1], c->ev[2]));
        HIPCHK(c, hipEventElapsedTime(&ms[2], c->ev[2], c->ev[3]));
        HIPCHK(c, hipEventElapsedTime(&ms[3], c->ev[7], c->ev[8]));
        HIPCHK(c, hipEventElapsedTime(&ms[4], c->ev[3], c->ev[5]));
        return VMS_OK;
    }
    for (int k = 0; k < 5; ++k) HIPCHK(c, hipEventElapsedTime(&ms[k], c->ev[k], c->ev[k + 1]));
    return VMS_OK;
}

int vms_set_overlap(vms_ctx *c, int on) {
    if (!c) return fail(nullptr, VMS_EINVAL, "null context");
    c->overlap = on != 0;
    return VMS_OK;
}

int vms_set_scatter(vms_ctx *c, uint32_t mode) {
    if (!c) return fail(nullptr, VMS_EINVAL, "null context");
    if (mode != VMS_SCATTER_RECORDS && mode != VMS_SCATTER_ATOMIC) return fail(c, VMS_EINVAL, "unknown scatter mode");
    if (mode == VMS_SCATTER_ATOMIC) {
        if (c->wbc) return fail(c, VMS_EUNSUPPORTED, "the atomic scatter excludes the weak boundary terms");
        if (!c->d_el_kk && upload(c, &c->d_el_kk, c->mesh.el_kk))
            return fail(c, VMS_ENOMEM, "device allocation failed (element block columns)");
        int rc = ensure_diag_pos(c);
        if (rc) return rc;
    }
    c->scatter = mode;
    return VMS_OK;
}

int vms_assemble(vms_ctx *c, const vms_fields *f, void *csr_vals, double *resid, uint32_t flags) {
    return assemble_impl(c, f, csr_vals, resid, flags, true);
}

int vms_apply(vms_ctx *c, const vms_fields *f, double *resid, double *norm2) {
    int rc = assemble_impl(c, f, nullptr, resid, 0, false);
    if (rc) return rc;
    if (norm2) {
        HIPCHK(c, hipMemsetAsync(c->d_norm, 0, sizeof(double), c->stream));
        vmsk::launch_norm2(c->stream, resid, 4 * c->mesh.n_nodes, c->d_norm);
        double s = 0;
        HIPCHK(c, hipMemcpyAsync(&s, c->d_norm, sizeof s, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        *norm2 = std::sqrt(s);
    }
    return VMS_OK;
}

// y = J x without the matrix; stage events when timed and timing is on
static int jv_impl(vms_ctx *c, const double *const fp[7], const double *x, double *y, bool timed) {
    const bool tm = timed && c->timing;
    if (tm) c->last_split = false;
    if (tm) {
        HIPCHK(c, hipEventRecord(c->ev[0], c->stream));
        HIPCHK(c, hipEventRecord(c->ev[1], c->stream));
    }
    const bool fp64 = c->prm.precision == VMS_FP64;
    vmsk::AsmArgs a = base_args(c);
    for (int k = 0; k < 7; ++k) a.f[k] = fp[k];
    a.rrec = c->d_rrec;
    a.slot0 = 0;
    if (tm) HIPCHK(c, hipEventRecord(c->ev[2], c->stream));
    a.n_items = c->n_std;
    a.items = c->d_std;
    vmsk::launch_jacobian_action(c->stream, a, false, fp64, x);
    HIPCHK(c, hipGetLastError());
    if (tm) HIPCHK(c, hipEventRecord(c->ev[3], c->stream));
    if (c->n_sub_items) {
        a.n_items = c->n_sub_items;
        a.items = c->d_sub_el;
        a.pt_off = c->d_sub_off;
        a.pt_cnt = c->d_sub_cnt;
        a.entries = c->d_entries;
        a.slot0 = c->n_std;
        vmsk::launch_jacobian_action(c->stream, a, true, fp64, x);
        HIPCHK(c, hipGetLastError());
    }
    if (c->wbc && c->n_surf_items) {
        vmsk::launch_surface(c->stream, surf_args(c, fp, y), 2, true, x);
        HIPCHK(c, hipGetLastError());
    }
    if (tm) HIPCHK(c, hipEventRecord(c->ev[4], c->stream));
    gather_resid(c, c->stream, y);
    vmsk::launch_copy_rows(c->stream, x, y, c->d_inact, c->n_inact);
    HIPCHK(c, hipGetLastError());
    if (tm) HIPCHK(c, hipEventRecord(c->ev[5], c->stream));
    return VMS_OK;
}

int vms_apply_jacobian(vms_ctx *c, const vms_fields *f, const double *x, double *y) {
    if (!c || !f || !x || !y) return fail(c, VMS_EINVAL, "null argument");
    const double *fp[7] = {f->ux, f->uy, f->uz, f->p, f->ux0, f->uy0, f->uz0};
    for (const double *p : fp)
        if (!p) return fail(c, VMS_EINVAL, "null field pointer");
    return jv_impl(c, fp, x, y, true);
}

int vms_spmv(vms_ctx *c, const void *csr_vals, const double *x, double *y) {
    if (!c || !csr_vals || !x || !y) return fail(c, VMS_EINVAL, "null argument");
    if (c->prm.precision == VMS_FP64)
        vmsk::launch_bspmv_f64(c->stream, c->d_nrow_ptr, c->d_ncol, (const double *)csr_vals, x, y,
                               c->mesh.n_nodes);
    else
        vmsk::launch_bspmv_f32(c->stream, c->d_nrow_ptr, c->d_ncol, (const float *)csr_vals, x, y,
                               c->mesh.n_nodes);
    HIPCHK(c, hipGetLastError());
    return VMS_OK;
}

// device copy of each node's diagonal block position (first use)
static int ensure_diag_pos(vms_ctx *c) {
    if (c->d_diag_pos) return VMS_OK;
    std::vector<int32_t> dp(c->mesh.diag_pos.begin(), c->mesh.diag_pos.end());
    if (upload(c, &c->d_diag_pos, dp)) return fail(c, VMS_ENOMEM, "device allocation failed (diagonal map)");
    return VMS_OK;
}

int vms_dirichlet_nodes(vms_ctx *c, int64_t *n, int32_t *nodes) {
    if (!c || !n) return fail(c, VMS_EINVAL, "null argument");
    *n = (int64_t)c->dir_nodes.size();
    if (nodes) std::memcpy(nodes, c->dir_nodes.data(), c->dir_nodes.size() * sizeof(int32_t));
    return VMS_OK;
}

int vms_dirichlet_in_nodes(vms_ctx *c, void *csr_vals, double *resid) {
    if (!c || !csr_vals) return fail(c, VMS_EINVAL, "null argument");
    int rc = ensure_diag_pos(c);
    if (rc) return rc;
    const int64_t nd = (int64_t)c->dir_nodes.size();
    if (nd == 0) return VMS_OK;
    if (!c->d_dir_nodes && upload(c, &c->d_dir_nodes, c->dir_nodes))
        return fail(c, VMS_ENOMEM, "device allocation failed (Dirichlet nodes)");
    if (c->prm.precision == VMS_FP64)
        vmsk::launch_dirichlet_rows_f64(c->stream, (double *)csr_vals, c->d_nrow_ptr, c->d_diag_pos,
                                        c->d_dir_nodes, nd, resid);
    else
        vmsk::launch_dirichlet_rows_f32(c->stream, (float *)csr_vals, c->d_nrow_ptr, c->d_diag_pos,
                                        c->d_dir_nodes, nd, resid);
    HIPCHK(c, hipGetLastError());
    return VMS_OK;
}

// Krylov solve of A dx = b (Newton's linear step), right-preconditioned by
// the inverses of the 4x4 diagonal blocks of the assembled values, so the
// residual monitored is the true one of the unpreconditioned system. BiCGStab
// (the paper's Krylov method) or restarted GMRES(m) (Arnoldi with classical
// Gram-Schmidt and one reorthogonalisation pass; Givens rotations and the small
// triangular solve on the host). A = the assembled matrix, or the matrix-free
// Jacobian action at the given fields. Inner products are deterministic
// two-stage sums; every scalar decision is taken on the host in FP64.
int vms_solve(vms_ctx *c, const void *csr_vals, const vms_fields *f, const double *b, double *x,
              int method, int restart, int max_iter, double rtol, uint32_t flags, int *iters,
              double *rel_res) {
    if (!c || !csr_vals || !b || !x) return fail(c, VMS_EINVAL, "null argument");
    if (flags & ~(uint32_t)VMS_SOLVE_DIRICHLET) return fail(c, VMS_EINVAL, "unknown flags");
    if (method != VMS_KSP_BCGS && method != VMS_KSP_GMRES) return fail(c, VMS_EINVAL, "unknown method");
    if (method == VMS_KSP_GMRES && (restart < 1 || restart > 200))
        return fail(c, VMS_EINVAL, "restart must be in [1, 200]");
    if (max_iter < 0) return fail(c, VMS_EINVAL, "negative iteration limit");
    if (!(rtol > 0.0) || !std::isfinite(rtol)) return fail(c, VMS_EINVAL, "rtol must be positive");
    const double *fp[7] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    if (f) {
        const double *q[7] = {f->ux, f->uy, f->uz, f->p, f->ux0, f->uy0, f->uz0};
        for (int k = 0; k < 7; ++k) {
            if (!q[k]) return fail(c, VMS_EINVAL, "null field pointer");
            fp[k] = q[k];
        }
    }
    const hipStream_t st = c->stream;
    const int64_t N = c->mesh.n_nodes, n = 4 * N;
    // Krylov vectors: m + 1 for GMRES, 8 for BiCGStab
    const int m = method == VMS_KSP_GMRES ? restart : 7;
    // ---- workspace (kept by the context)
    if (c->gm_m < m) {
        for (double *p : {c->d_gm_V, c->d_gm_part, c->d_gm_h}) c->buf.free(p);
        c->d_gm_V = c->d_gm_part = c->d_gm_h = nullptr;
        c->gm_m = 0;
        if (c->buf.alloc(&c->d_gm_V, (size_t)(m + 1) * n) ||
            c->buf.alloc(&c->d_gm_part, (size_t)(m + 1) * vmsk::multidot_blocks(n)) ||
            c->buf.alloc(&c->d_gm_h, (size_t)m + 2))
            return fail(c, VMS_ENOMEM, "device allocation failed (Krylov vectors)");
        c->gm_m = m;
    }
    if (!c->d_gm_dinv) {
        int rc0 = ensure_diag_pos(c);
        if (rc0) return rc0;
        if (c->buf.alloc(&c->d_gm_w, n) || c->buf.alloc(&c->d_gm_z, n) || c->buf.alloc(&c->d_gm_r, n) ||
            c->buf.alloc(&c->d_gm_bad, 1) || c->buf.alloc(&c->d_gm_dinv, (size_t)16 * N))
            return fail(c, VMS_ENOMEM, "device allocation failed (preconditioner)");
    }
    double *V = c->d_gm_V, *w = c->d_gm_w, *z = c->d_gm_z, *r = c->d_gm_r, *dh = c->d_gm_h;
    // ---- block-Jacobi preconditioner from the current values
    HIPCHK(c, hipMemsetAsync(c->d_gm_bad, 0, sizeof(int), st));
    if (c->prm.precision == VMS_FP64)
        vmsk::launch_bjac_invert_f64(st, (const double *)csr_vals, c->d_nrow_ptr, c->d_diag_pos, N,
                                     c->d_gm_dinv, c->d_gm_bad);
    else
        vmsk::launch_bjac_invert_f32(st, (const float *)csr_vals, c->d_nrow_ptr, c->d_diag_pos, N,
                                     c->d_gm_dinv, c->d_gm_bad);
    HIPCHK(c, hipGetLastError());
    int bad = 0;
    HIPCHK(c, hipMemcpyAsync(&bad, c->d_gm_bad, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    if (bad) return fail(c, VMS_EINVAL, "singular diagonal block (assemble before solving)");
    const bool mf_dir = f && (flags & VMS_SOLVE_DIRICHLET) && !c->dir_nodes.empty();
    if (mf_dir && !c->d_dir_nodes && upload(c, &c->d_dir_nodes, c->dir_nodes))
        return fail(c, VMS_ENOMEM, "device allocation failed (Dirichlet nodes)");
    auto op = [&](const double *in, double *out) -> int {
        if (!f) return vms_spmv(c, csr_vals, in, out);
        int e = jv_impl(c, fp, in, out, false);
        if (e) return e;
        if (mf_dir) {  // identity rows at the Dirichlet nodes, as in the CSR values
            vmsk::launch_copy_rows(st, in, out, c->d_dir_nodes, (int64_t)c->dir_nodes.size());
            HIPCHK(c, hipGetLastError());
        }
        return VMS_OK;
    };
    auto prec = [&](const double *in, double *out) { vmsk::launch_bjac_apply(st, c->d_gm_dinv, in, out, N); };
    // host copies of nk inner products Vb_k . v (the coefficients stay in dh)
    std::vector<double> hv(m + 2);
    auto dots = [&](const double *Vb, int nk, const double *v) -> int {
        vmsk::launch_multidot(st, Vb, n, nk, v, n, c->d_gm_part, dh);
        HIPCHK(c, hipGetLastError());
        HIPCHK(c, hipMemcpyAsync(hv.data(), dh, sizeof(double) * nk, hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        return VMS_OK;
    };
    int rc;
    if ((rc = dots(b, 1, b))) return rc;
    const double bnorm = std::sqrt(hv[0]);
    if (bnorm == 0.0) {
        vmsk::launch_fill_f64(st, x, n, 0.0);
        HIPCHK(c, hipStreamSynchronize(st));
        if (iters) *iters = 0;
        if (rel_res) *rel_res = 0.0;
        return VMS_OK;
    }
    int it = 0;
    double res = 0.0;
    if (method == VMS_KSP_BCGS) {
        // vectors: r (residual), rh (shadow), p, v, ph = M^-1 p, s and t adjacent
        // (one multi-dot gives t.s and t.t), sh = M^-1 s
        double *rr = V, *rh = V + n, *pp = V + 2 * n, *vv = V + 3 * n, *ph = V + 4 * n, *ss = V + 5 * n,
               *tt = V + 6 * n, *sh = V + 7 * n;
        while (true) {
            // true residual; the recurrence restarts from it
            if ((rc = op(x, w))) return rc;
            vmsk::launch_axpby(st, 1.0, b, -1.0, w, rr, n);
            if ((rc = dots(rr, 1, rr))) return rc;
            res = std::sqrt(hv[0]) / bnorm;
            if (res <= rtol || it >= max_iter) break;
            vmsk::launch_axpby(st, 1.0, rr, 0.0, rr, rh, n);
            double rho_old = 1.0, alpha = 1.0, omega = 1.0;
            // rh . r of the next step: r . r at a restart (rh = r), else from the
            // same multi-dot as the end-of-step residual norm (r and rh adjacent)
            double rho_next = hv[0];
            const int it0 = it;
            for (int k = 0; it < max_iter; ++k) {
                const double rho = rho_next;
                if (rho == 0.0) break;
                if (k == 0) {
                    vmsk::launch_axpby(st, 1.0, rr, 0.0, rr, pp, n);
                } else {
                    const double beta = (rho / rho_old) * (alpha / omega);
                    vmsk::launch_axpbypcz(st, 1.0, rr, beta, pp, -beta * omega, vv, pp, n);
                }
                prec(pp, ph);
                if ((rc = op(ph, vv))) return rc;
                if ((rc = dots(rh, 1, vv))) return rc;
                if (hv[0] == 0.0) break;
                alpha = rho / hv[0];
                vmsk::launch_axpby(st, 1.0, rr, -alpha, vv, ss, n);
                ++it;
                if ((rc = dots(ss, 1, ss))) return rc;
                if (std::sqrt(hv[0]) <= rtol * bnorm) {  // confirmed by the true residual
                    vmsk::launch_axpby(st, 1.0, x, alpha, ph, x, n);
                    break;
                }
                prec(ss, sh);
                if ((rc = op(sh, tt))) return rc;
                if ((rc = dots(ss, 2, tt))) return rc;  // s.t, t.t
                if (hv[1] == 0.0) {
                    vmsk::launch_axpby(st, 1.0, x, alpha, ph, x, n);
                    break;
                }
                omega = hv[0] / hv[1];
                vmsk::launch_axpbypcz(st, 1.0, x, alpha, ph, omega, sh, x, n);
                vmsk::launch_axpby(st, 1.0, ss, -omega, tt, rr, n);
                if ((rc = dots(rr, 2, rr))) return rc;  // r . r, rh . r
                if (std::sqrt(hv[0]) <= rtol * bnorm || omega == 0.0) break;
                rho_next = hv[1];
                rho_old = rho;
            }
            if (it == it0) break;  // breakdown before any step: no progress from a restart
        }
    } else {
        std::vector<std::vector<double>> H(m + 1, std::vector<double>(m, 0.0));
        std::vector<double> cs(m), sn(m), g(m + 1), y(m), h(m + 1);
        while (true) {
            // true residual r = b - A x
            if ((rc = op(x, w))) return rc;
            vmsk::launch_axpby(st, 1.0, b, -1.0, w, r, n);
            if ((rc = dots(r, 1, r))) return rc;
            const double beta = std::sqrt(hv[0]);
            res = beta / bnorm;
            if (res <= rtol || it >= max_iter) break;
            vmsk::launch_axpby(st, 1.0 / beta, r, 0.0, r, V, n);
            std::fill(g.begin(), g.end(), 0.0);
            g[0] = beta;
            int j = 0;
            while (j < m && it < max_iter) {
                double *vj1 = V + (int64_t)(j + 1) * n;
                prec(V + (int64_t)j * n, z);
                if ((rc = op(z, w))) return rc;
                // two Gram-Schmidt passes against V_0 .. V_j
                if ((rc = dots(V, j + 1, w))) return rc;
                for (int i = 0; i <= j; ++i) h[i] = hv[i];
                vmsk::launch_combine(st, V, n, j + 1, dh, w, n, 0);
                if ((rc = dots(V, j + 1, w))) return rc;
                for (int i = 0; i <= j; ++i) h[i] += hv[i];
                vmsk::launch_combine(st, V, n, j + 1, dh, w, n, 0);
                if ((rc = dots(w, 1, w))) return rc;
                const double hn = std::sqrt(hv[0]);
                if (hn > 0.0) vmsk::launch_axpby(st, 1.0 / hn, w, 0.0, w, vj1, n);
                // Givens rotations
                for (int i = 0; i < j; ++i) {
                    const double t = cs[i] * h[i] + sn[i] * h[i + 1];
                    h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1];
                    h[i] = t;
                }
                const double den = std::hypot(h[j], hn);
                cs[j] = den > 0.0 ? h[j] / den : 1.0;
                sn[j] = den > 0.0 ? hn / den : 0.0;
                h[j] = den;
                for (int i = 0; i <= j; ++i) H[i][j] = h[i];
                g[j + 1] = -sn[j] * g[j];
                g[j] = cs[j] * g[j];
                ++j;
                ++it;
                if (std::fabs(g[j]) <= rtol * bnorm || hn == 0.0) break;
            }
            // y = H^-1 g (upper triangular j x j), x += M^-1 (V y)
            for (int i = j - 1; i >= 0; --i) {
                double sum = g[i];
                for (int k = i + 1; k < j; ++k) sum -= H[i][k] * y[k];
                y[i] = H[i][i] != 0.0 ? sum / H[i][i] : 0.0;
            }
            HIPCHK(c, hipMemcpyAsync(dh, y.data(), sizeof(double) * j, hipMemcpyHostToDevice, st));
            vmsk::launch_combine(st, V, n, j, dh, w, n, 1);
            prec(w, z);
            vmsk::launch_axpby(st, 1.0, x, 1.0, z, x, n);
            HIPCHK(c, hipGetLastError());
        }
    }
    HIPCHK(c, hipStreamSynchronize(st));
    if (iters) *iters = it;
    if (rel_res) *rel_res = res;
    return VMS_OK;
}

int vms_set_weak_bc(vms_ctx *c, int enable, double c_b, const double *g) {
    if (!c) return fail(nullptr, VMS_EINVAL, "null context");
    if (!enable) {
        if (!c->wbc) return VMS_OK;
        c->wbc = false;
        return build_gather(c, c->std_el);
    }
    if (!c->has_surf) return fail(c, VMS_EINVAL, "weak boundary terms need a surface");
    if (c->scatter == VMS_SCATTER_ATOMIC)
        return fail(c, VMS_EUNSUPPORTED, "the weak boundary terms need the record scatter");
    if (!g || !std::isfinite(c_b) || c_b < 0 || !std::isfinite(g[0]) || !std::isfinite(g[1]) ||
        !std::isfinite(g[2]))
        return fail(c, VMS_EINVAL, "bad weak-boundary parameters (c_b >= 0, finite g)");
    int rc = build_weak_bc(c, c_b);
    if (rc) return rc;
    for (int k = 0; k < 3; ++k) c->wbc_g[k] = g[k];
    c->wbc = true;
    return build_gather(c, c->std_el);
}

int vms_element_weights(vms_ctx *c, double ts_over_tv, double *w) {
    if (!c || !w) return fail(c, VMS_EINVAL, "null argument");
    if (!std::isfinite(ts_over_tv) || ts_over_tv < 0) return fail(c, VMS_EINVAL, "ts_over_tv must be >= 0");
    const int64_t E = (int64_t)c->markers.size();
    std::vector<int64_t> nv(E, 0), ns(E, 0);
    for (int64_t e = 0; e < E; ++e) nv[e] = c->markers[e] == 0 ? 8 : 0;
    for (int64_t i = 0; i < c->n_sq && i < (int64_t)c->sq_cnt.size(); ++i) nv[c->sq_el[i]] = c->sq_cnt[i];
    if (c->wbc)
        for (int64_t e : c->surf_pt_el) ++ns[e];
    for (int64_t e = 0; e < E; ++e) w[e] = (double)nv[e] / 8.0 + ts_over_tv * ((double)ns[e] / 8.0);
    return VMS_OK;
}

int vms_set_inout(vms_ctx *c, uint32_t mode, const vms_mlp *mlp, int32_t min_bt) {
    if (!c) return fail(nullptr, VMS_EINVAL, "null context");
    if (mode != VMS_INOUT_EXACT && mode != VMS_INOUT_LEARNED && mode != VMS_INOUT_NORMAL)
        return fail(c, VMS_EINVAL, "unknown in-out mode");
    if (mode == VMS_INOUT_LEARNED && !mlp) return fail(c, VMS_EINVAL, "learned in-out mode needs a network");
    if (min_bt < 0) return fail(c, VMS_EINVAL, "min_bt must be >= 0");
    c->prm.inout_mode = mode;
    c->prm.learned_min_bt = min_bt;
    c->mlp = (const vmsm::MlpHandle *)mlp;
    return VMS_OK;
}

int vms_components(vms_ctx *c, int32_t *n_comp, uint8_t *convex) {
    if (!c || !n_comp) return fail(c, VMS_EINVAL, "null argument");
    *n_comp = c->n_comp;
    if (convex && c->n_comp) std::memcpy(convex, c->comp_convex.data(), (size_t)c->n_comp);
    return VMS_OK;
}

int vms_surface_components(const vms_surface *surf, int32_t *comp, int32_t *n_comp) {
    if (!surf || !n_comp || surf->n_tri <= 0 || surf->n_vert <= 0 || !surf->verts || !surf->tri)
        return fail(nullptr, VMS_EINVAL, "null or empty surface");
    std::string err;
    int rc = vms::check_watertight(surf, err);
    if (rc) return fail(nullptr, rc, err);
    std::vector<int32_t> cc;
    int32_t nc = 0;
    rc = vms::surface_components(surf, cc, nc, nullptr, nullptr, nullptr, err);
    if (rc) return fail(nullptr, rc, err);
    *n_comp = nc;
    if (comp) std::memcpy(comp, cc.data(), cc.size() * sizeof(int32_t));
    return VMS_OK;
}

int vms_relabel_stats(vms_ctx *c, int64_t *out) {
    if (!c || !out) return fail(c, VMS_EINVAL, "null argument");
    unsigned long long v = 0;
    if (c->n_sq) {
        HIPCHK(c, hipMemcpyAsync(&v, c->d_counters + 2, sizeof v, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    out[0] = (int64_t)c->n_labelled;
    out[1] = (int64_t)v;
    return VMS_OK;
}

int vms_stats(vms_ctx *c, int64_t *out) {
    if (!c || !out) return fail(c, VMS_EINVAL, "null argument");
    out[0] = c->n_std;
    out[1] = c->n_sq;
    out[2] = (int64_t)c->n_labelled;
    out[3] = (int64_t)c->n_degenerate;
    out[4] = c->mesh.n_hanging;
    out[5] = c->n_subgp;
    out[6] = c->wbc ? c->n_surfgp : 0;
    return VMS_OK;
}

// ---------------------------------------------------------------------------
// in-out classification of arbitrary points
// ---------------------------------------------------------------------------

struct inout_handle {
    SurfaceHost surf;
    hipStream_t stream;
    unsigned long long *d_ndeg = nullptr;
    DevBuf buf;
    vmsm::Filter filter;
};

int inout_prepare(const vms_surface *s, void *stream, inout_handle **out) {
    if (!out) return fail(nullptr, VMS_EINVAL, "null output pointer");
    *out = nullptr;
    inout_handle *h = new inout_handle();
    h->stream = (hipStream_t)stream;
    std::string err;
    int rc = build_surface(s, h->stream, h->surf, err);
    if (rc) { set_global_err(err); delete h; return rc; }
    if (h->buf.alloc(&h->d_ndeg, 1)) { set_global_err("device allocation failed"); delete h; return VMS_ENOMEM; }
    *out = h;
    return VMS_OK;
}

int inout_reserve(inout_handle *h, int64_t n) {
    if (!h || n < 0) return fail(nullptr, VMS_EINVAL, "null handle or negative size");
    if (vmsm::reserve_filter(h->filter, n)) return fail(nullptr, VMS_ENOMEM, "device allocation failed");
    return VMS_OK;
}

void inout_release(inout_handle *h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    delete h;
}

int inout_classify_prepared(inout_handle *h, const double *px, const double *py, const double *pz,
                            int64_t n, uint8_t *labels, uint32_t mode, const void *mlp) {
    if (!h || (n > 0 && (!px || !py || !pz || !labels)) || n < 0)
        return fail(nullptr, VMS_EINVAL, "null argument or negative size");
    if (mode == VMS_INOUT_EXACT) {
        vmsk::launch_point_labels(h->stream, h->surf.S, n, px, py, pz, labels, nullptr);
    } else if (mode == VMS_INOUT_LEARNED) {
        if (!mlp) return fail(nullptr, VMS_EINVAL, "learned mode needs a network");
        int rc = vmsm::classify_learned(h->stream, h->filter, (const vmsm::MlpHandle *)mlp, h->surf.S, px,
                                        py, pz, n, labels);
        if (rc) return fail(nullptr, rc, "learned classification failed");
    } else {
        return fail(nullptr, VMS_EUNSUPPORTED, "unknown in-out mode");
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(nullptr, VMS_EHIP, hipGetErrorString(e));
    return VMS_OK;
}

int vms_sdf_sample(inout_handle *h, const double *px, const double *py, const double *pz, int64_t n,
                   double trunc, double *sdf) {
    if (!h || n < 0 || (n > 0 && (!px || !py || !pz || !sdf)) || !(trunc > 0))
        return fail(nullptr, VMS_EINVAL, "bad arguments");
    int rc = vmsm_sdf(h->stream, h->surf.S, h->surf.tv, h->surf.lo, h->surf.hi, px, py, pz, n, trunc, sdf);
    if (rc) return fail(nullptr, rc, "signed-distance sampling failed");
    return VMS_OK;
}

int inout_classify(const vms_surface *surf, const double *px, const double *py, const double *pz,
                   int64_t n, uint8_t *labels, uint32_t mode, const void *mlp, void *stream) {
    inout_handle *h = nullptr;
    int rc = inout_prepare(surf, stream, &h);
    if (rc) return rc;
    rc = inout_classify_prepared(h, px, py, pz, n, labels, mode, mlp);
    if (rc == VMS_OK && hipStreamSynchronize(h->stream) != hipSuccess) rc = VMS_EHIP;
    inout_release(h);
    return rc;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// host-only mesh derivation (no device involved)
// ---------------------------------------------------------------------------

struct vms_mesh {
    vms::MeshHost m;
    std::vector<int32_t> ax, ay, az;
    std::vector<uint8_t> level;
};

extern "C" {

int vms_mesh_create(vms_mesh **out, const vms_octree *tree, const uint8_t *markers) {
    if (!out) return fail(nullptr, VMS_EINVAL, "null output pointer");
    *out = nullptr;
    if (!tree || !tree->ax || !tree->ay || !tree->az || !tree->level || tree->n_oct <= 0)
        return fail(nullptr, VMS_EINVAL, "null or empty octree");
    if (tree->max_level < 0 || tree->max_level > 20)
        return fail(nullptr, VMS_EUNSUPPORTED, "max_level must be in [0, 20]");
    vms_mesh *h = new vms_mesh();
    const int64_t E = tree->n_oct;
    h->ax.assign(tree->ax, tree->ax + E);
    h->ay.assign(tree->ay, tree->ay + E);
    h->az.assign(tree->az, tree->az + E);
    h->level.assign(tree->level, tree->level + E);
    vms::TreeIn ti{E, h->ax.data(), h->ay.data(), h->az.data(), h->level.data(), tree->max_level};
    std::string err;
    int rc = vms::derive_mesh(ti, h->m, err);
    if (rc == 0) {
        std::vector<uint8_t> active(E, 1);
        if (markers)
            for (int64_t e = 0; e < E; ++e) active[e] = markers[e] != 1;
        rc = vms::build_pattern(h->m, active, err);
        if (rc) rc = rc == -6 ? VMS_EUNSUPPORTED : VMS_EINVAL;
    } else {
        rc = rc == -2 ? VMS_EMESH : VMS_EINVAL;
    }
    if (rc) {
        set_global_err(err);
        delete h;
        return rc;
    }
    *out = h;
    return VMS_OK;
}

int vms_mesh_sizes(vms_mesh *h, int64_t *n_nodes, int64_t *nnz, int64_t *n_hanging) {
    if (!h) return fail(nullptr, VMS_EINVAL, "null mesh");
    if (n_nodes) *n_nodes = h->m.n_nodes;
    if (nnz) *nnz = h->m.nnz;
    if (n_hanging) *n_hanging = h->m.n_hanging;
    return VMS_OK;
}

int vms_mesh_export(vms_mesh *h, uint32_t what, void *dst) {
    if (!h || !dst) return fail(nullptr, VMS_EINVAL, "null mesh or destination");
    const vms::MeshHost &m = h->m;
    switch (what) {
        case VMS_EXPORT_NODE_XYZ: {
            int32_t *d = (int32_t *)dst;
            for (int64_t n = 0; n < m.n_nodes; ++n) {
                int64_t x, y, z;
                vms::unmorton3(m.node_key[n], x, y, z);
                d[n] = (int32_t)x; d[m.n_nodes + n] = (int32_t)y; d[2 * m.n_nodes + n] = (int32_t)z;
            }
            return VMS_OK;
        }
        case VMS_EXPORT_ROW_PTR: std::memcpy(dst, m.row_ptr.data(), m.row_ptr.size() * 8); return VMS_OK;
        case VMS_EXPORT_COL_IDX: vms::fill_col_idx(m, (int32_t *)dst); return VMS_OK;
        case VMS_EXPORT_MASTERS: std::memcpy(dst, m.masters.data(), m.masters.size() * 4); return VMS_OK;
        default: return fail(nullptr, VMS_EINVAL, "unsupported export selector for a host mesh");
    }
}

void vms_mesh_destroy(vms_mesh *h) { delete h; }

}  // extern "C"

// ---------------------------------------------------------------------------
// batched assembly over many contexts: one persistent launch, device queue
// ---------------------------------------------------------------------------

struct vms_batch {
    hipStream_t stream = nullptr;
    std::vector<vms_ctx *> ctx;
    int precision = 0;
    int tile = 4, groups_per_cu = 8, n_cu = 256;
    bool by_weight = true;  // eq. (Wpart) units, heaviest first; else the fixed order
    std::vector<vmsk::AsmArgs> h_std, h_sub;
    std::vector<void *> h_vals;  // CSR values of each tree
    std::vector<double *> h_resid;  // residual of each tree (or null)
    vmsk::AsmArgs *d_std = nullptr, *d_sub = nullptr;
    vmsk::BatchUnit *d_units = nullptr;
    int64_t n_units = 0, units_cap = 0;
    double unit_weight_max = 0, unit_weight_sum = 0;
    unsigned long long *d_counter = nullptr;
    // batched gathers: per-tree lists, first block / node of each tree
    std::vector<vmsk::GatherTab> h_tabs;
    vmsk::GatherTab *d_tabs = nullptr;
    int64_t *d_blk_prefix = nullptr, *d_node_prefix = nullptr;
    int64_t tot_blocks = 0, tot_nodes = 0;
    DevBuf buf;
    // graph replay
    bool use_graph = false, captured = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<const void *> cap_ptrs;
    std::vector<uint64_t> gens;  // generation of each context's buffers when last read
    // timing of the last eager launch sequence
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    bool timed = false;
    std::string err = "no error";
    ~vms_batch() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

namespace {

int bfail(vms_batch *b, int code, const std::string &m) {
    if (b) b->err = m;
    set_global_err(m);
    return code;
}

int batch_units(vms_batch *b);

void drop_graph(vms_batch *b) {
    if (!b->captured) return;
    (void)hipGraphExecDestroy(b->exec);
    (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->captured = false;
}

// Every call re-checks its contexts: weak boundary terms switched on after
// the batch was made are refused, and rebuilt record buffers (a new
// generation) invalidate the unit list and any captured graph.
int batch_check(vms_batch *b) {
    for (vms_ctx *c : b->ctx)
        if (c->wbc) return bfail(b, VMS_EUNSUPPORTED, "the batched form has no weak boundary terms");
    bool stale = false;
    for (size_t t = 0; t < b->ctx.size(); ++t) stale |= b->ctx[t]->gen != b->gens[t];
    if (!stale) return VMS_OK;
    drop_graph(b);
    int rc = batch_units(b);
    if (rc) return rc;
    for (size_t t = 0; t < b->ctx.size(); ++t) b->gens[t] = b->ctx[t]->gen;
    return VMS_OK;
}

int batch_units(vms_batch *b) {
    // Units of about `tile` element weights of eq. (Wpart): an OUT element
    // weighs n_Vgp / n_Tgp = 1, a sub-cell work item its points / 8 (the
    // batch has no surface terms). Runs of consecutive items of one kind and
    // one tree are cut when they reach the target weight; the list is ordered
    // by decreasing weight (longest first) so that the queue ends on light
    // units.
    // Fixed order (by_weight false): every sub-cell work item a unit of its
    // own, all of them first, then runs of `tile` OUT elements.
    const double target = b->by_weight ? (double)b->tile : 0.0;
    std::vector<vmsk::BatchUnit> u;
    std::vector<double> w;
    for (size_t t = 0; t < b->ctx.size(); ++t) {
        const vms_ctx *c = b->ctx[t];
        int64_t first = 0;
        double acc = 0;
        for (int64_t i = 0; i < c->n_sub_items; ++i) {
            acc += c->sub_item_cnt[i] / 8.0;
            if (acc >= target || i + 1 == c->n_sub_items) {
                u.push_back({(int32_t)t, 1, first, (int32_t)(i + 1 - first), 0});
                w.push_back(acc);
                first = i + 1;
                acc = 0;
            }
        }
        for (int64_t i = 0; i < c->n_std; i += b->tile) {
            const int64_t n = std::min<int64_t>(b->tile, c->n_std - i);
            u.push_back({(int32_t)t, 0, i, (int32_t)n, 0});
            w.push_back((double)n);
        }
    }
    std::vector<int64_t> ord(u.size());
    for (size_t k = 0; k < ord.size(); ++k) ord[k] = (int64_t)k;
    if (b->by_weight)
        std::stable_sort(ord.begin(), ord.end(), [&](int64_t x, int64_t y) { return w[x] > w[y]; });
    else
        std::stable_partition(ord.begin(), ord.end(), [&](int64_t x) { return u[x].sub != 0; });
    std::vector<vmsk::BatchUnit> us(u.size());
    b->unit_weight_max = 0;
    b->unit_weight_sum = 0;
    for (size_t k = 0; k < ord.size(); ++k) {
        us[k] = u[ord[k]];
        b->unit_weight_max = std::max(b->unit_weight_max, w[ord[k]]);
        b->unit_weight_sum += w[ord[k]];
    }
    b->n_units = (int64_t)us.size();
    if (b->n_units > b->units_cap) {
        b->buf.free(b->d_units);
        if (b->buf.alloc(&b->d_units, (size_t)b->n_units)) return bfail(b, VMS_ENOMEM, "device allocation failed");
        b->units_cap = b->n_units;
    }
    if (b->n_units && (hipMemcpyAsync(b->d_units, us.data(), us.size() * sizeof(vmsk::BatchUnit),
                                      hipMemcpyHostToDevice, b->stream) ||
                       hipStreamSynchronize(b->stream)))
        return bfail(b, VMS_EHIP, "device copy failed (units)");
    return VMS_OK;
}

int batch_tables(vms_batch *b, const vms_fields *f, void *const *vals, double *const *resid) {
    const size_t n = b->ctx.size();
    for (size_t t = 0; t < n; ++t) {
        vms_ctx *c = b->ctx[t];
        const double *fp[7] = {f[t].ux, f[t].uy, f[t].uz, f[t].p, f[t].ux0, f[t].uy0, f[t].uz0};
        for (const double *p : fp)
            if (!p) return bfail(b, VMS_EINVAL, "null field pointer");
        if (!vals[t]) return bfail(b, VMS_EINVAL, "null csr_vals");
        vmsk::AsmArgs a = base_args(c);
        for (int k = 0; k < 7; ++k) a.f[k] = fp[k];
        b->h_vals[t] = vals[t];
        b->h_resid[t] = resid ? resid[t] : nullptr;
        a.rrec = resid ? c->d_rrec : nullptr;
        a.em = c->d_em;
        a.slot0 = 0;
        a.n_items = c->n_std;
        a.items = c->d_std;
        b->h_std[t] = a;
        a.n_items = c->n_sub_items;
        a.items = c->d_sub_el;
        a.pt_off = c->d_sub_off;
        a.pt_cnt = c->d_sub_cnt;
        a.entries = c->d_entries;
        a.slot0 = c->n_std;
        b->h_sub[t] = a;
        vmsk::GatherTab &G = b->h_tabs[t];
        G.em = c->d_em;
        G.cb_off = c->d_cb_off;
        G.contrib = c->d_contrib;
        G.vbase = c->d_vbase;
        G.vstride = c->d_vstride;
        G.vals = vals[t];
        G.rrec = c->d_rrec;
        G.roff = c->d_roff;
        G.rlist = c->d_rlist;
        G.resid = resid ? resid[t] : nullptr;
    }
    std::vector<int64_t> bp(n + 1, 0), np(n + 1, 0);
    for (size_t t = 0; t < n; ++t) {
        bp[t + 1] = bp[t] + b->ctx[t]->n_blocks;
        np[t + 1] = np[t] + b->ctx[t]->mesh.n_nodes;
    }
    b->tot_blocks = bp[n];
    b->tot_nodes = np[n];
    if (hipMemcpyAsync(b->d_std, b->h_std.data(), n * sizeof(vmsk::AsmArgs), hipMemcpyHostToDevice, b->stream) ||
        hipMemcpyAsync(b->d_sub, b->h_sub.data(), n * sizeof(vmsk::AsmArgs), hipMemcpyHostToDevice, b->stream) ||
        hipMemcpyAsync(b->d_tabs, b->h_tabs.data(), n * sizeof(vmsk::GatherTab), hipMemcpyHostToDevice,
                       b->stream) ||
        hipMemcpyAsync(b->d_blk_prefix, bp.data(), bp.size() * 8, hipMemcpyHostToDevice, b->stream) ||
        hipMemcpyAsync(b->d_node_prefix, np.data(), np.size() * 8, hipMemcpyHostToDevice, b->stream) ||
        hipStreamSynchronize(b->stream))
        return bfail(b, VMS_EHIP, "device copy failed (tables)");
    return VMS_OK;
}

// persistent assembly, then each tree's CSR values (with identity rows) and
// residual summed from its records (all kernels; no memset). With timed set,
// events bracket the persistent kernel and the summations.
void batch_enqueue(vms_batch *b, bool timed) {
    if (timed) (void)hipEventRecord(b->ev[0], b->stream);
    if (timed) (void)hipEventRecord(b->ev[1], b->stream);
    vmsk::launch_assemble_batch(b->stream, b->precision, b->d_std, b->d_sub, b->d_units, b->n_units,
                                b->d_counter, b->n_cu * b->groups_per_cu);
    if (timed) (void)hipEventRecord(b->ev[2], b->stream);
    vmsk::launch_gather_batch(b->stream, b->precision, b->d_tabs, b->d_blk_prefix, b->tot_blocks,
                              b->d_node_prefix, b->tot_nodes, (int)b->ctx.size());
    if (timed) (void)hipEventRecord(b->ev[3], b->stream);
    b->timed = timed;
}

}  // namespace

extern "C" {

int vms_batch_create(vms_batch **out, vms_ctx *const *ctxs, int n, void *stream) {
    if (!out || !ctxs || n <= 0) return bfail(nullptr, VMS_EINVAL, "bad arguments");
    *out = nullptr;
    vms_batch *b = new vms_batch();
    b->stream = (hipStream_t)stream;
    for (int i = 0; i < n; ++i) {
        if (!ctxs[i]) { delete b; return bfail(nullptr, VMS_EINVAL, "null context"); }
        b->ctx.push_back(ctxs[i]);
    }
    b->precision = (int)ctxs[0]->prm.precision;
    for (vms_ctx *c : b->ctx)
        if (c->wbc) {
            delete b;
            return bfail(nullptr, VMS_EUNSUPPORTED, "the batched form has no weak boundary terms");
        }
    for (vms_ctx *c : b->ctx)
        if ((int)c->prm.precision != b->precision) {
            delete b;
            return bfail(nullptr, VMS_EINVAL, "contexts of a batch must share one precision");
        }
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
        b->n_cu = cus;
    for (hipEvent_t &e : b->ev)
        if (hipEventCreate(&e) != hipSuccess) {
            delete b;
            return bfail(nullptr, VMS_EHIP, "event creation failed");
        }
    b->h_std.resize(n);
    b->h_sub.resize(n);
    b->h_vals.assign(n, nullptr);
    b->h_resid.assign(n, nullptr);
    b->h_tabs.assign(n, vmsk::GatherTab{});
    if (b->buf.alloc(&b->d_std, (size_t)n) || b->buf.alloc(&b->d_sub, (size_t)n) ||
        b->buf.alloc(&b->d_counter, 2) || b->buf.alloc(&b->d_tabs, (size_t)n) ||
        b->buf.alloc(&b->d_blk_prefix, (size_t)n + 1) || b->buf.alloc(&b->d_node_prefix, (size_t)n + 1)) {
        delete b;
        return bfail(nullptr, VMS_ENOMEM, "device allocation failed");
    }
    int rc = batch_units(b);
    if (rc) { delete b; return rc; }
    for (vms_ctx *c : b->ctx) b->gens.push_back(c->gen);
    *out = b;
    return VMS_OK;
}

int vms_batch_set_config(vms_batch *b, int tile, int groups_per_cu) {
    if (!b || tile <= 0 || groups_per_cu <= 0) return bfail(b, VMS_EINVAL, "bad configuration");
    b->groups_per_cu = groups_per_cu;
    if (tile != b->tile) {
        b->tile = tile;
        drop_graph(b);  // the captured graph refers to the old unit list
        return batch_units(b);
    }
    return VMS_OK;
}

int vms_batch_set_order(vms_batch *b, int by_weight) {
    if (!b) return bfail(nullptr, VMS_EINVAL, "null batch");
    if ((by_weight != 0) == b->by_weight) return VMS_OK;
    b->by_weight = by_weight != 0;
    drop_graph(b);
    return batch_units(b);
}

int vms_batch_get_config(vms_batch *b, int *tile, int *groups_per_cu, int64_t *n_units) {
    if (!b) return bfail(nullptr, VMS_EINVAL, "null batch");
    if (tile) *tile = b->tile;
    if (groups_per_cu) *groups_per_cu = b->groups_per_cu;
    if (n_units) *n_units = b->n_units;
    return VMS_OK;
}

int vms_batch_use_graph(vms_batch *b, int on) {
    if (!b) return bfail(nullptr, VMS_EINVAL, "null batch");
    b->use_graph = on != 0;
    return VMS_OK;
}

int vms_batch_assemble(vms_batch *b, const vms_fields *f, void *const *vals, double *const *resid) {
    if (!b || !f || !vals) return bfail(b, VMS_EINVAL, "null argument");
    int rc0 = batch_check(b);
    if (rc0) return rc0;
    const size_t n = b->ctx.size();
    std::vector<const void *> ptrs;
    for (size_t t = 0; t < n; ++t) {
        const double *fp[7] = {f[t].ux, f[t].uy, f[t].uz, f[t].p, f[t].ux0, f[t].uy0, f[t].uz0};
        for (const double *p : fp) ptrs.push_back(p);
        ptrs.push_back(vals[t]);
        ptrs.push_back(resid ? resid[t] : nullptr);
    }
    if (b->use_graph && b->captured && ptrs == b->cap_ptrs) {
        if (hipGraphLaunch(b->exec, b->stream) != hipSuccess) return bfail(b, VMS_EHIP, "graph launch failed");
        return VMS_OK;
    }
    int rc = batch_tables(b, f, vals, resid);
    if (rc) return rc;
    if (!b->use_graph) {
        batch_enqueue(b, true);
        if (hipGetLastError() != hipSuccess) return bfail(b, VMS_EHIP, "launch failed");
        return VMS_OK;
    }
    drop_graph(b);
    if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return bfail(b, VMS_EHIP, "stream capture failed to start");
    batch_enqueue(b, false);
    if (hipStreamEndCapture(b->stream, &b->graph) != hipSuccess ||
        hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess)
        return bfail(b, VMS_EHIP, "graph capture failed");
    b->captured = true;
    b->cap_ptrs = ptrs;
    if (hipGraphLaunch(b->exec, b->stream) != hipSuccess) return bfail(b, VMS_EHIP, "graph launch failed");
    return VMS_OK;
}

// Time every (tile, groups per CU) candidate on the given buffers and keep the
// fastest. ms (HOST, nullable) receives the best time of one assembly.
int vms_batch_autotune(vms_batch *b, const vms_fields *f, void *const *vals, double *const *resid,
                       float *ms_out) {
    if (!b) return bfail(nullptr, VMS_EINVAL, "null batch");
    const int tiles[] = {1, 2, 4, 8, 16};
    const int gpcs[] = {4, 8, 16, 32};
    const bool g = b->use_graph;
    b->use_graph = false;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) || hipEventCreate(&e1)) return bfail(b, VMS_EHIP, "event creation failed");
    float best = INFINITY;
    int bt = b->tile, bg = b->groups_per_cu;
    int rc = VMS_OK;
    for (int tile : tiles) {
        for (int gpc : gpcs) {
            if ((rc = vms_batch_set_config(b, tile, gpc))) break;
            if ((rc = vms_batch_assemble(b, f, vals, resid))) break;  // warm-up
            float tmin = INFINITY;
            for (int r = 0; r < 3; ++r) {
                (void)hipEventRecord(e0, b->stream);
                if ((rc = vms_batch_assemble(b, f, vals, resid))) break;
                (void)hipEventRecord(e1, b->stream);
                float t = 0;
                if (hipEventSynchronize(e1) || hipEventElapsedTime(&t, e0, e1)) { rc = VMS_EHIP; break; }
                tmin = std::min(tmin, t);
            }
            if (rc) break;
            if (tmin < best) { best = tmin; bt = tile; bg = gpc; }
        }
        if (rc) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->use_graph = g;
    if (rc) return rc;
    if (ms_out) *ms_out = best;
    return vms_batch_set_config(b, bt, bg);
}

int vms_batch_last_timing(vms_batch *b, float *ms) {
    if (!b || !ms) return bfail(b, VMS_EINVAL, "null argument");
    if (!b->timed) return bfail(b, VMS_EINVAL, "no eager batched assembly to time");
    if (hipEventSynchronize(b->ev[3]) != hipSuccess ||
        hipEventElapsedTime(&ms[0], b->ev[0], b->ev[1]) != hipSuccess ||
        hipEventElapsedTime(&ms[1], b->ev[1], b->ev[2]) != hipSuccess ||
        hipEventElapsedTime(&ms[2], b->ev[2], b->ev[3]) != hipSuccess)
        return bfail(b, VMS_EHIP, "event timing failed");
    return VMS_OK;
}

void vms_batch_destroy(vms_batch *b) {
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    delete b;
}

}  // extern "C"

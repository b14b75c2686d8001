// Triquadratic (Q2, 27-node) elements of libvms: host set-up and C-ABI.
//
// A uniform octree (every leaf on one level: no hanging nodes) gets the nodes
// of the 27-node elements (positions on the grid of half the element side,
// numbered by Morton key, x in the lowest bit), the CSR pattern of the node
// pairs that share an element (full 4x4 blocks, columns ascending), and the
// lists that sum each CSR block's element records and each node's residual
// entries in ascending record order (the same record-and-gather scheme as the
// trilinear elements: no atomics, reproducible bits).
#include "../../include/vms.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "kernels.h"
#include "mesh.h"
#include "par.h"

struct vms_q2 {
    hipStream_t stream = nullptr;
    std::string err = "no error";
    vms_params prm{};
    int32_t max_level = 0;
    int64_t E = 0, n_nodes = 0, nnz = 0, n_blocks = 0;
    double h = 0;
    std::vector<uint64_t> node_key;
    std::vector<int32_t> el_node;  // [E][27]
    std::vector<int64_t> nrow_ptr, row_ptr;
    std::vector<int32_t> ncol;
    std::vector<void *> dev;
    int32_t *d_el_node = nullptr, *d_contrib = nullptr, *d_vstride = nullptr, *d_rlist = nullptr;
    int64_t *d_cb_off = nullptr, *d_vbase = nullptr, *d_roff = nullptr;
    double *d_em = nullptr, *d_rrec = nullptr;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};  // element kernel, gathers
    bool timed = false;
    ~vms_q2() {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
        for (void *p : dev) (void)hipFree(p);
    }
    template <typename T>
    bool alloc(T **p, size_t n) {
        *p = nullptr;
        if (hipMalloc((void **)p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) return false;
        dev.push_back(*p);
        return true;
    }
    template <typename T>
    bool upload(T **p, const std::vector<T> &v) {
        return alloc(p, v.size()) &&
               (v.empty() || hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) == hipSuccess);
    }
};

namespace {

std::string g_q2_err = "no error";

int qfail(vms_q2 *q, int code, const std::string &m) {
    if (q) q->err = m;
    g_q2_err = m;
    return code;
}

}  // namespace

extern "C" {

int vms_q2_create(vms_q2 **out, const vms_octree *tree, const vms_params *prm, void *stream) {
    if (!out || !tree || !prm) return qfail(nullptr, VMS_EINVAL, "null argument");
    *out = nullptr;
    const int64_t E = tree->n_oct;
    if (E <= 0 || !tree->ax || !tree->ay || !tree->az || !tree->level)
        return qfail(nullptr, VMS_EINVAL, "empty or null octree");
    if (tree->max_level < 0 || tree->max_level > 19)
        return qfail(nullptr, VMS_EUNSUPPORTED, "Q2 elements need max_level <= 19");
    if (prm->precision != VMS_FP64) return qfail(nullptr, VMS_EUNSUPPORTED, "Q2 elements are FP64 only");
    if (!(prm->rho > 0) || !(prm->dt > 0) || !(prm->mu >= 0) || !(prm->theta >= 0) || prm->theta > 1)
        return qfail(nullptr, VMS_EINVAL, "parameter out of range");
    const int L = tree->level[0];
    for (int64_t e = 0; e < E; ++e)
        if (tree->level[e] != L || L > tree->max_level)
            return qfail(nullptr, VMS_EMESH, "Q2 elements need every leaf on one level (no hanging nodes)");
    const int64_t side = (int64_t)1 << (tree->max_level - L);
    for (int64_t e = 0; e < E; ++e)
        if (tree->ax[e] < 0 || tree->ay[e] < 0 || tree->az[e] < 0 || tree->ax[e] % side || tree->ay[e] % side ||
            tree->az[e] % side || tree->ax[e] + side > ((int64_t)1 << tree->max_level) ||
            tree->ay[e] + side > ((int64_t)1 << tree->max_level) ||
            tree->az[e] + side > ((int64_t)1 << tree->max_level))
            return qfail(nullptr, VMS_EMESH, "leaf outside the root or not aligned to its side");
    vms_q2 *q = new vms_q2();
    q->stream = (hipStream_t)stream;
    q->prm = *prm;
    q->max_level = tree->max_level;
    q->E = E;
    q->h = tree->root_len * (double)side / (double)((int64_t)1 << tree->max_level);

    // nodes: 2 anchor + s side on the half grid, s in {0, 1, 2} per axis
    std::vector<uint64_t> keys((size_t)E * 27);
    vms::parallel_for(E, [&](int64_t b, int64_t f, int) {
        for (int64_t e = b; e < f; ++e)
            for (int a = 0; a < 27; ++a)
                keys[27 * e + a] = vms::morton3(2 * (uint64_t)tree->ax[e] + (a % 3) * side,
                                                2 * (uint64_t)tree->ay[e] + ((a / 3) % 3) * side,
                                                2 * (uint64_t)tree->az[e] + (a / 9) * side);
    });
    q->node_key = keys;
    std::sort(q->node_key.begin(), q->node_key.end());
    q->node_key.erase(std::unique(q->node_key.begin(), q->node_key.end()), q->node_key.end());
    const int64_t N = (int64_t)q->node_key.size();
    q->n_nodes = N;
    if (E * 729 > INT32_MAX) { delete q; return qfail(nullptr, VMS_EUNSUPPORTED, "too many Q2 elements"); }
    q->el_node.resize((size_t)E * 27);
    vms::parallel_for(E * 27, [&](int64_t b, int64_t f, int) {
        for (int64_t k = b; k < f; ++k)
            q->el_node[k] = (int32_t)(std::lower_bound(q->node_key.begin(), q->node_key.end(), keys[k]) -
                                      q->node_key.begin());
    });
    // elements of each node
    std::vector<int64_t> ne_off(N + 1, 0);
    for (int64_t k = 0; k < E * 27; ++k) ne_off[q->el_node[k] + 1]++;
    for (int64_t n = 0; n < N; ++n) ne_off[n + 1] += ne_off[n];
    std::vector<int32_t> ne((size_t)E * 27);  // (element * 27 + slot), ascending per node
    {
        std::vector<int64_t> pos(ne_off.begin(), ne_off.end() - 1);
        for (int64_t k = 0; k < E * 27; ++k) ne[pos[q->el_node[k]]++] = (int32_t)k;
    }
    // node rows: the nodes of every element of the node
    std::vector<std::vector<int32_t>> rows(N);
    vms::parallel_for(N, [&](int64_t b, int64_t f, int) {
        for (int64_t n = b; n < f; ++n) {
            std::vector<int32_t> &r = rows[n];
            for (int64_t c = ne_off[n]; c < ne_off[n + 1]; ++c) {
                const int64_t e = ne[c] / 27;
                r.insert(r.end(), q->el_node.begin() + 27 * e, q->el_node.begin() + 27 * e + 27);
            }
            std::sort(r.begin(), r.end());
            r.erase(std::unique(r.begin(), r.end()), r.end());
        }
    });
    q->nrow_ptr.assign(N + 1, 0);
    for (int64_t n = 0; n < N; ++n) q->nrow_ptr[n + 1] = q->nrow_ptr[n] + (int64_t)rows[n].size();
    q->n_blocks = q->nrow_ptr[N];
    q->ncol.resize(q->n_blocks);
    for (int64_t n = 0; n < N; ++n) std::copy(rows[n].begin(), rows[n].end(), q->ncol.begin() + q->nrow_ptr[n]);
    rows.clear();
    q->row_ptr.assign(4 * N + 1, 0);
    for (int64_t n = 0; n < N; ++n) {
        const int64_t deg = q->nrow_ptr[n + 1] - q->nrow_ptr[n];
        for (int c = 0; c < 4; ++c) q->row_ptr[4 * n + c + 1] = q->row_ptr[4 * n + c] + 4 * deg;
    }
    q->nnz = q->row_ptr[4 * N];
    // block lists: record block (27 e + s) 27 + t of element e, node slots s
    // (test) and t (trial), summed into block (el_node[s], el_node[t]); the
    // elements are visited in ascending order, so each list is ascending
    std::vector<int64_t> cb_off(q->n_blocks + 1, 0);
    std::vector<int64_t> blk((size_t)E * 729);
    vms::parallel_for(E, [&](int64_t b, int64_t f, int) {
        for (int64_t e = b; e < f; ++e)
            for (int s = 0; s < 27; ++s) {
                const int32_t ns = q->el_node[27 * e + s];
                const int32_t *c0 = q->ncol.data() + q->nrow_ptr[ns], *c1 = q->ncol.data() + q->nrow_ptr[ns + 1];
                for (int t = 0; t < 27; ++t)
                    blk[729 * e + 27 * s + t] =
                        q->nrow_ptr[ns] + (std::lower_bound(c0, c1, q->el_node[27 * e + t]) - c0);
            }
    });
    for (int64_t k = 0; k < E * 729; ++k) cb_off[blk[k] + 1]++;
    for (int64_t b = 0; b < q->n_blocks; ++b) cb_off[b + 1] += cb_off[b];
    std::vector<int32_t> contrib(cb_off[q->n_blocks]);
    {
        std::vector<int64_t> pos(cb_off.begin(), cb_off.end() - 1);
        for (int64_t k = 0; k < E * 729; ++k) contrib[pos[blk[k]]++] = (int32_t)k;
    }
    blk.clear();
    std::vector<int64_t> vbase(q->n_blocks);
    std::vector<int32_t> vstride(q->n_blocks);
    for (int64_t n = 0; n < N; ++n) {
        const int64_t b0 = q->nrow_ptr[n], deg = q->nrow_ptr[n + 1] - b0;
        for (int64_t b = b0; b < q->nrow_ptr[n + 1]; ++b) {
            vbase[b] = 16 * b0 + 4 * (b - b0);
            vstride[b] = (int32_t)(4 * deg);
        }
    }
    if (!q->upload(&q->d_el_node, q->el_node) || !q->upload(&q->d_cb_off, cb_off) ||
        !q->upload(&q->d_contrib, contrib) || !q->upload(&q->d_vbase, vbase) ||
        !q->upload(&q->d_vstride, vstride) || !q->upload(&q->d_roff, ne_off) || !q->upload(&q->d_rlist, ne) ||
        !q->alloc(&q->d_em, (size_t)E * 729 * 16) || !q->alloc(&q->d_rrec, (size_t)E * 108)) {
        delete q;
        return qfail(nullptr, VMS_ENOMEM, "device allocation failed (Q2 set-up)");
    }
    for (hipEvent_t &ev : q->ev)
        if (hipEventCreate(&ev) != hipSuccess) {
            delete q;
            return qfail(nullptr, VMS_EHIP, "event creation failed");
        }
    *out = q;
    return VMS_OK;
}

int vms_q2_last_timing(vms_q2 *q, float *ms) {
    if (!q || !ms) return qfail(q, VMS_EINVAL, "null argument");
    if (!q->timed) return qfail(q, VMS_EINVAL, "no assembly to time");
    if (hipEventSynchronize(q->ev[2]) != hipSuccess || hipEventElapsedTime(&ms[0], q->ev[0], q->ev[1]) ||
        hipEventElapsedTime(&ms[1], q->ev[1], q->ev[2]))
        return qfail(q, VMS_EHIP, "event timing failed");
    return VMS_OK;
}

int vms_q2_sizes(vms_q2 *q, int64_t *n_nodes, int64_t *n_rows, int64_t *nnz) {
    if (!q) return qfail(nullptr, VMS_EINVAL, "null context");
    if (n_nodes) *n_nodes = q->n_nodes;
    if (n_rows) *n_rows = 4 * q->n_nodes;
    if (nnz) *nnz = q->nnz;
    return VMS_OK;
}

int vms_q2_export(vms_q2 *q, uint32_t what, void *dst) {
    if (!q || !dst) return qfail(q, VMS_EINVAL, "null context or destination");
    switch (what) {
        case VMS_EXPORT_NODE_XYZ: {
            int32_t *d = (int32_t *)dst;
            for (int64_t n = 0; n < q->n_nodes; ++n) {
                int64_t x, y, z;
                vms::unmorton3(q->node_key[n], x, y, z);
                d[n] = (int32_t)x;
                d[q->n_nodes + n] = (int32_t)y;
                d[2 * q->n_nodes + n] = (int32_t)z;
            }
            return VMS_OK;
        }
        case VMS_EXPORT_ROW_PTR:
            std::copy(q->row_ptr.begin(), q->row_ptr.end(), (int64_t *)dst);
            return VMS_OK;
        case VMS_EXPORT_COL_IDX: {
            int32_t *d = (int32_t *)dst;
            vms::parallel_for(q->n_nodes, [&](int64_t b, int64_t f, int) {
                for (int64_t n = b; n < f; ++n)
                    for (int c = 0; c < 4; ++c) {
                        int64_t k = q->row_ptr[4 * n + c];
                        for (int64_t bb = q->nrow_ptr[n]; bb < q->nrow_ptr[n + 1]; ++bb)
                            for (int j = 0; j < 4; ++j) d[k++] = 4 * q->ncol[bb] + j;
                    }
            });
            return VMS_OK;
        }
        default:
            return qfail(q, VMS_EINVAL, "unknown export selector");
    }
}

int vms_q2_assemble(vms_q2 *q, const vms_fields *f, double *csr_vals, double *resid) {
    if (!q || !f || !csr_vals) return qfail(q, VMS_EINVAL, "null argument");
    const double *fp[7] = {f->ux, f->uy, f->uz, f->p, f->ux0, f->uy0, f->uz0};
    for (const double *p : fp)
        if (!p) return qfail(q, VMS_EINVAL, "null field pointer");
    vmsk::Q2Args a{};
    a.n_el = q->E;
    a.el_node = q->d_el_node;
    for (int k = 0; k < 7; ++k) a.f[k] = fp[k];
    a.h = q->h;
    const vms_params &P = q->prm;
    const double nu = P.mu / P.rho;
    a.rho = P.rho;
    a.mu = P.mu;
    a.theta = P.theta;
    a.idt = 1.0 / P.dt;
    a.irho = 1.0 / P.rho;
    a.tau_a = P.c_t / (P.dt * P.dt);
    a.tau_b = 3.0 * P.c_i * nu * nu;
    a.em = q->d_em;
    a.rrec = q->d_rrec;
    (void)hipEventRecord(q->ev[0], q->stream);
    vmsk::launch_q2(q->stream, a);
    (void)hipEventRecord(q->ev[1], q->stream);
    vmsk::launch_gather_f64(q->stream, q->d_em, q->d_cb_off, q->d_contrib, q->d_vbase, q->d_vstride,
                            q->n_blocks, csr_vals);
    if (resid) vmsk::launch_q2_res_gather(q->stream, q->d_rrec, q->d_roff, q->d_rlist, q->n_nodes, resid);
    (void)hipEventRecord(q->ev[2], q->stream);
    q->timed = true;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return qfail(q, VMS_EHIP, std::string("launch failed: ") + hipGetErrorString(e));
    return VMS_OK;
}

const char *vms_q2_last_error(vms_q2 *q) { return q ? q->err.c_str() : g_q2_err.c_str(); }

void vms_q2_destroy(vms_q2 *q) {
    if (!q) return;
    (void)hipStreamSynchronize(q->stream);
    delete q;
}

}  // extern "C"

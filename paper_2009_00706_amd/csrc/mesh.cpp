// Host-side mesh derivation of libvms: vertices, hanging-node constraints
// (Alg. 3: hanging faces take I1d (x) I1d, hanging edges I1d, with
// I1d = [1/2 1/2]), independent node numbering, per-element master slots and
// the CSR pattern with its element-to-entry map.
//
// A vertex is hanging when it is a leaf corner lying in the interior of an
// edge or a face of another leaf. With 2:1 balance across faces, edges and
// vertices (checked here) only a leaf's edge midpoints and face centres can
// be such vertices, and their masters (the edge ends, the face corners) are
// never hanging themselves.
//
// The loops over elements and nodes run on host worker threads (par.h); every
// result is the one of the serial loop, independent of the thread count.
#include "mesh.h"

#include <algorithm>
#include <atomic>
#include <cstring>
#include <numeric>

#include "par.h"

namespace vms {

namespace {

// spread the low 21 bits of v to every third bit
inline uint64_t spread3(uint64_t v) {
    v &= 0x1fffffull;
    v = (v | v << 32) & 0x1f00000000ffffull;
    v = (v | v << 16) & 0x1f0000ff0000ffull;
    v = (v | v << 8) & 0x100f00f00f00f00full;
    v = (v | v << 4) & 0x10c30c30c30c30c3ull;
    v = (v | v << 2) & 0x1249249249249249ull;
    return v;
}

inline uint64_t compact3(uint64_t v) {
    v &= 0x1249249249249249ull;
    v = (v | v >> 2) & 0x10c30c30c30c30c3ull;
    v = (v | v >> 4) & 0x100f00f00f00f00full;
    v = (v | v >> 8) & 0x1f0000ff0000ffull;
    v = (v | v >> 16) & 0x1f00000000ffffull;
    v = (v | v >> 32) & 0x1fffffull;
    return v;
}

}  // namespace

// Morton code with x in bit 0, y in bit 1, z in bit 2 (21 bits per axis).
uint64_t morton3(uint64_t x, uint64_t y, uint64_t z) {
    return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}

void unmorton3(uint64_t k, int64_t &x, int64_t &y, int64_t &z) {
    x = (int64_t)compact3(k);
    y = (int64_t)compact3(k >> 1);
    z = (int64_t)compact3(k >> 2);
}

namespace {

// Open-addressing hash map uint64 key -> int32 value (keys never equal ~0).
// Filled by one thread, then read concurrently.
struct KeyMap {
    std::vector<uint64_t> keys;
    std::vector<int32_t> vals;
    uint64_t mask = 0;
    static constexpr uint64_t EMPTY = ~0ull;
    explicit KeyMap(size_t n) {
        size_t cap = 16;
        while (cap < 2 * n + 16) cap <<= 1;
        keys.assign(cap, EMPTY);
        vals.assign(cap, -1);
        mask = cap - 1;
    }
    static uint64_t mix(uint64_t k) {
        k ^= k >> 33; k *= 0xff51afd7ed558ccdull; k ^= k >> 33; k *= 0xc4ceb9fe1a85ec53ull;
        return k ^ (k >> 33);
    }
    void put(uint64_t k, int32_t v) {
        uint64_t i = mix(k) & mask;
        while (keys[i] != EMPTY && keys[i] != k) i = (i + 1) & mask;
        keys[i] = k; vals[i] = v;
    }
    int32_t get(uint64_t k) const {
        uint64_t i = mix(k) & mask;
        while (keys[i] != EMPTY) {
            if (keys[i] == k) return vals[i];
            i = (i + 1) & mask;
        }
        return -1;
    }
};

inline int64_t corner_coord(int64_t a, int c, int axis, int64_t side) {
    return a + (((c >> axis) & 1) ? side : 0);
}

// a hanging vertex found from one element: type 2 (edge) or 4 (face), masters
struct HangEvent {
    int32_t v;
    int8_t type;
    int32_t mast[4];
};

}  // namespace

int derive_mesh(const TreeIn &t, MeshHost &m, std::string &err) {
    const int64_t E = t.n;
    const int M = t.max_level;
    m = MeshHost();
    m.n_el = E;
    if (E <= 0) { err = "empty octree"; return -1; }
    // --- validate leaves ---
    const int64_t root = (int64_t)1 << M;
    for (int64_t e = 0; e < E; ++e) {
        int L = t.level[e];
        if (L > M) { err = "leaf level above max_level"; return -1; }
        int64_t s = (int64_t)1 << (M - L);
        int64_t a[3] = {t.ax[e], t.ay[e], t.az[e]};
        for (int k = 0; k < 3; ++k)
            if (a[k] < 0 || a[k] + s > root || (a[k] & (s - 1))) {
                err = "leaf anchor outside the root or not aligned to its size";
                return -1;
            }
    }
    // --- 2:1 balance (faces, edges, vertices): locate each leaf's 26 same-size
    //     neighbours among the leaves sorted by Morton key ---
    {
        std::vector<std::pair<uint64_t, int32_t>> ord(E);
        parallel_for(E, [&](int64_t b, int64_t f, int) {
            for (int64_t e = b; e < f; ++e) ord[e] = {morton3(t.ax[e], t.ay[e], t.az[e]), (int32_t)e};
        });
        parallel_sort(ord);
        for (int64_t i = 1; i < E; ++i)
            if (ord[i].first == ord[i - 1].first) { err = "two leaves share an anchor"; return -2; }
        std::vector<uint64_t> sk(E);
        for (int64_t i = 0; i < E; ++i) sk[i] = ord[i].first;
        std::atomic<bool> unbalanced{false};
        parallel_for(E, [&](int64_t b, int64_t f, int) {
            for (int64_t e = b; e < f && !unbalanced.load(std::memory_order_relaxed); ++e) {
                int L = t.level[e];
                int64_t s = (int64_t)1 << (M - L);
                for (int dz = -1; dz <= 1; ++dz)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dx = -1; dx <= 1; ++dx) {
                            if (!dx && !dy && !dz) continue;
                            int64_t q[3] = {t.ax[e] + dx * s, t.ay[e] + dy * s, t.az[e] + dz * s};
                            if (q[0] < 0 || q[1] < 0 || q[2] < 0 || q[0] >= root || q[1] >= root ||
                                q[2] >= root)
                                continue;
                            uint64_t k = morton3(q[0], q[1], q[2]);
                            auto it = std::upper_bound(sk.begin(), sk.end(), k);
                            if (it == sk.begin()) continue;  // not covered (domain with holes)
                            int32_t nb = ord[(it - sk.begin()) - 1].second;
                            int64_t ns = (int64_t)1 << (M - t.level[nb]);
                            bool covers = q[0] >= t.ax[nb] && q[0] < t.ax[nb] + ns && q[1] >= t.ay[nb] &&
                                          q[1] < t.ay[nb] + ns && q[2] >= t.az[nb] && q[2] < t.az[nb] + ns;
                            if (covers && (int)t.level[nb] < L - 1) unbalanced = true;
                        }
            }
        });
        if (unbalanced) { err = "octree is not 2:1 balanced"; return -2; }
    }
    // --- vertex table ---
    std::vector<uint64_t> ck((size_t)E * 8);
    parallel_for(E, [&](int64_t b, int64_t f, int) {
        for (int64_t e = b; e < f; ++e) {
            int64_t s = (int64_t)1 << (M - t.level[e]);
            for (int c = 0; c < 8; ++c)
                ck[8 * e + c] = morton3(corner_coord(t.ax[e], c, 0, s), corner_coord(t.ay[e], c, 1, s),
                                        corner_coord(t.az[e], c, 2, s));
        }
    });
    std::vector<uint64_t> vk(ck);
    parallel_sort(vk);
    vk.erase(std::unique(vk.begin(), vk.end()), vk.end());
    const int64_t NV = (int64_t)vk.size();
    KeyMap vmap(NV);
    for (int64_t v = 0; v < NV; ++v) vmap.put(vk[v], (int32_t)v);
    m.elem_vert.resize((size_t)E * 8);
    parallel_for((int64_t)ck.size(), [&](int64_t b, int64_t f, int) {
        for (int64_t i = b; i < f; ++i) m.elem_vert[i] = vmap.get(ck[i]);
    });
    std::vector<uint64_t>().swap(ck);
    m.vert_key = vk;

    // --- hanging vertices: edge midpoints and face centres that are corners ---
    // per vertex: number of masters (1 regular, 2 edge, 4 face) and master vertex
    // ids. Each thread lists what its elements find; the lists are applied in
    // element order, as the serial loop would write them.
    std::vector<int8_t> vtype(NV, 1);
    std::vector<int32_t> vmast((size_t)NV * 4, -1);
    for (int64_t v = 0; v < NV; ++v) vmast[4 * v] = (int32_t)v;
    {
        std::vector<std::vector<HangEvent>> ev(host_threads());
        const int T = parallel_for(E, [&](int64_t b, int64_t f, int th) {
            std::vector<HangEvent> &out = ev[th];
            for (int64_t e = b; e < f; ++e) {
                int64_t s = (int64_t)1 << (M - t.level[e]);
                if (s < 2) continue;
                int64_t h = s / 2;
                const int64_t a[3] = {t.ax[e], t.ay[e], t.az[e]};
                // edges: along axis k, the other two coordinates at 0 or s
                for (int k = 0; k < 3; ++k) {
                    int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
                    for (int o = 0; o < 4; ++o) {
                        int64_t p[3], q0[3], q1[3];
                        p[k] = a[k] + h; q0[k] = a[k]; q1[k] = a[k] + s;
                        p[k1] = q0[k1] = q1[k1] = a[k1] + ((o & 1) ? s : 0);
                        p[k2] = q0[k2] = q1[k2] = a[k2] + ((o & 2) ? s : 0);
                        int32_t v = vmap.get(morton3(p[0], p[1], p[2]));
                        if (v < 0) continue;
                        out.push_back({v, 2, {vmap.get(morton3(q0[0], q0[1], q0[2])),
                                              vmap.get(morton3(q1[0], q1[1], q1[2])), -1, -1}});
                    }
                }
                // faces: normal axis k at 0 or s, centre offset h in the other two
                for (int k = 0; k < 3; ++k) {
                    int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
                    for (int side = 0; side < 2; ++side) {
                        int64_t p[3];
                        p[k] = a[k] + (side ? s : 0);
                        p[k1] = a[k1] + h;
                        p[k2] = a[k2] + h;
                        int32_t v = vmap.get(morton3(p[0], p[1], p[2]));
                        if (v < 0) continue;
                        HangEvent hv{v, 4, {-1, -1, -1, -1}};
                        int n = 0;
                        for (int j2 = 0; j2 < 2; ++j2)
                            for (int j1 = 0; j1 < 2; ++j1) {
                                int64_t q[3];
                                q[k] = p[k];
                                q[k1] = a[k1] + (j1 ? s : 0);
                                q[k2] = a[k2] + (j2 ? s : 0);
                                hv.mast[n++] = vmap.get(morton3(q[0], q[1], q[2]));
                            }
                        out.push_back(hv);
                    }
                }
            }
        });
        for (int th = 0; th < T; ++th)
            for (const HangEvent &h : ev[th]) {
                vtype[h.v] = h.type;
                vmast[4 * (int64_t)h.v] = h.mast[0];
                vmast[4 * (int64_t)h.v + 1] = h.mast[1];
                if (h.type == 4) {
                    vmast[4 * (int64_t)h.v + 2] = h.mast[2];
                    vmast[4 * (int64_t)h.v + 3] = h.mast[3];
                }
            }
    }
    for (int64_t v = 0; v < NV; ++v) {
        if (vtype[v] == 1) continue;
        for (int j = 0; j < vtype[v]; ++j) {
            int32_t mv = vmast[4 * v + j];
            if (mv < 0 || vtype[mv] != 1) {
                err = "chained hanging constraint (octree not vertex-balanced)";
                return -2;
            }
        }
    }
    // --- independent nodes in Morton order (vk is sorted) ---
    std::vector<int32_t> node_of(NV, -1);
    int64_t nn = 0;
    for (int64_t v = 0; v < NV; ++v)
        if (vtype[v] == 1) { node_of[v] = (int32_t)nn++; m.node_key.push_back(vk[v]); }
    m.n_nodes = nn;
    m.n_hanging = NV - nn;
    m.vert_type = vtype;

    // --- element master slots (first appearance over corners 0..7) and C ---
    m.masters.assign((size_t)E * 8, -1);
    m.ccode.assign((size_t)E * 4, 0u);
    m.has_hang.assign(E, 0);
    m.nslot.assign(E, 0);
    std::atomic<bool> too_many{false};
    parallel_for(E, [&](int64_t b, int64_t f, int) {
        for (int64_t e = b; e < f; ++e) {
            int32_t *ms = &m.masters[8 * e];
            int ns = 0;
            uint32_t *cc = &m.ccode[4 * e];
            for (int a = 0; a < 8; ++a) {
                int32_t v = m.elem_vert[8 * e + a];
                int nmast = vtype[v];
                if (nmast != 1) m.has_hang[e] = 1;
                uint32_t code = nmast == 1 ? 3u : (nmast == 2 ? 2u : 1u);  // weight 1, 1/2, 1/4
                for (int j = 0; j < nmast; ++j) {
                    int32_t node = node_of[vmast[4 * (int64_t)v + j]];
                    int s = 0;
                    while (s < ns && ms[s] != node) ++s;
                    if (s == ns) {
                        if (ns == 8) { too_many = true; break; }
                        ms[ns++] = node;
                    }
                    int bit = 2 * (a * 8 + s);  // 64 entries x 2 bits in 4 words
                    cc[bit / 32] |= code << (bit % 32);
                }
            }
            m.nslot[e] = (uint8_t)ns;
        }
    });
    if (too_many) { err = "element with more than 8 master nodes"; return -2; }
    return 0;
}

int build_pattern(MeshHost &m, const std::vector<uint8_t> &active, std::string &err) {
    const int64_t E = m.n_el, N = m.n_nodes;
    // --- node-to-element incidence over active elements (list order is free:
    //     each node's adjacency is sorted below) ---
    std::vector<int64_t> inc_ptr(N + 1, 0);
    parallel_for(E, [&](int64_t b, int64_t f, int) {
        for (int64_t e = b; e < f; ++e) {
            if (!active[e]) continue;
            for (int s = 0; s < m.nslot[e]; ++s)
                __atomic_fetch_add(&inc_ptr[m.masters[8 * e + s] + 1], 1, __ATOMIC_RELAXED);
        }
    });
    for (int64_t n = 0; n < N; ++n) inc_ptr[n + 1] += inc_ptr[n];
    std::vector<int32_t> inc(inc_ptr[N]);
    {
        std::vector<int64_t> fill(inc_ptr.begin(), inc_ptr.end() - 1);
        parallel_for(E, [&](int64_t b, int64_t f, int) {
            for (int64_t e = b; e < f; ++e) {
                if (!active[e]) continue;
                for (int s = 0; s < m.nslot[e]; ++s) {
                    int64_t at = __atomic_fetch_add(&fill[m.masters[8 * e + s]], 1, __ATOMIC_RELAXED);
                    inc[at] = (int32_t)e;
                }
            }
        });
    }
    // --- node-level adjacency: the node itself and every master of its
    //     elements, sorted and unique; counted first, then written ---
    auto adjacency = [&](int64_t n, std::vector<int32_t> &buf) {
        buf.clear();
        buf.push_back((int32_t)n);
        for (int64_t i = inc_ptr[n]; i < inc_ptr[n + 1]; ++i) {
            const int64_t e = inc[i];
            for (int s = 0; s < m.nslot[e]; ++s) buf.push_back(m.masters[8 * e + s]);
        }
        std::sort(buf.begin(), buf.end());
        buf.erase(std::unique(buf.begin(), buf.end()), buf.end());
    };
    m.nrow_ptr.assign(N + 1, 0);
    parallel_for(N, [&](int64_t b, int64_t f, int) {
        std::vector<int32_t> buf;
        for (int64_t n = b; n < f; ++n) {
            adjacency(n, buf);
            m.nrow_ptr[n + 1] = (int64_t)buf.size();
        }
    });
    for (int64_t n = 0; n < N; ++n) m.nrow_ptr[n + 1] += m.nrow_ptr[n];
    m.ncol.resize(m.nrow_ptr[N]);
    parallel_for(N, [&](int64_t b, int64_t f, int) {
        std::vector<int32_t> buf;
        for (int64_t n = b; n < f; ++n) {
            adjacency(n, buf);
            std::memcpy(&m.ncol[m.nrow_ptr[n]], buf.data(), buf.size() * 4);
        }
    });
    std::vector<int64_t>().swap(inc_ptr);
    std::vector<int32_t>().swap(inc);
    // --- dof-level CSR: row 4n+c repeats node row n expanded to 4 columns per
    //     node, so row 4n+c starts at 16 nrow_ptr[n] + 4 c deg(n) ---
    m.row_ptr.assign(4 * N + 1, 0);
    parallel_for(N, [&](int64_t b, int64_t f, int) {
        for (int64_t n = b; n < f; ++n) {
            const int64_t deg = m.nrow_ptr[n + 1] - m.nrow_ptr[n];
            for (int c = 0; c < 4; ++c) m.row_ptr[4 * n + c] = 16 * m.nrow_ptr[n] + 4 * c * deg;
        }
    });
    m.row_ptr[4 * N] = 16 * m.nrow_ptr[N];
    m.nnz = m.row_ptr[4 * N];
    // --- element map: per slot s the row base (entry of (4 m_s, 4 m_0)) and the
    //     dof-row stride 4 deg; per slot pair (s, t) the block position of m_t in
    //     row m_s ---
    m.el_rowbase.assign((size_t)E * 8, 0);
    m.el_rowlen.assign((size_t)E * 8, 0);
    m.el_kk.assign((size_t)E * 64, 0);
    m.node_active.assign(N, 0);
    std::atomic<int> bad{0};  // bit 0: degree too large, bit 1: missing block
    parallel_for(E, [&](int64_t b, int64_t f, int) {
        for (int64_t e = b; e < f; ++e) {
            if (!active[e]) continue;
            const int32_t *ms = &m.masters[8 * e];
            for (int s = 0; s < m.nslot[e]; ++s) {
                int32_t r = ms[s];
                __atomic_store_n(&m.node_active[r], (uint8_t)1, __ATOMIC_RELAXED);
                int64_t b0 = m.nrow_ptr[r], deg = m.nrow_ptr[r + 1] - b0;
                if (deg > 65535) { bad.fetch_or(1); continue; }
                m.el_rowbase[8 * e + s] = m.row_ptr[4 * (int64_t)r];
                m.el_rowlen[8 * e + s] = (int32_t)(4 * deg);
                for (int t = 0; t < m.nslot[e]; ++t) {
                    const int32_t *lo = &m.ncol[b0], *hi = &m.ncol[b0 + deg];
                    const int32_t *it = std::lower_bound(lo, hi, ms[t]);
                    if (it == hi || *it != ms[t]) { bad.fetch_or(2); continue; }
                    m.el_kk[64 * e + 8 * s + t] = (uint16_t)(it - lo);
                }
            }
        }
    });
    if (bad & 1) { err = "node degree above 65535"; return -6; }
    if (bad & 2) { err = "pattern misses a block"; return -1; }
    // diagonal entry of every node's 4 rows, for identity blocks of inactive nodes
    m.diag_pos.assign(N, 0);
    parallel_for(N, [&](int64_t b, int64_t f, int) {
        for (int64_t n = b; n < f; ++n) {
            int64_t b0 = m.nrow_ptr[n], deg = m.nrow_ptr[n + 1] - b0;
            const int32_t *it = std::lower_bound(&m.ncol[b0], &m.ncol[b0] + deg, (int32_t)n);
            m.diag_pos[n] = (int32_t)(it - &m.ncol[b0]);
        }
    });
    return 0;
}

void fill_col_idx(const MeshHost &m, int32_t *dst) {
    parallel_for(m.n_nodes, [&](int64_t b, int64_t f, int) {
        for (int64_t n = b; n < f; ++n) {
            const int64_t b0 = m.nrow_ptr[n], deg = m.nrow_ptr[n + 1] - b0;
            for (int c = 0; c < 4; ++c) {
                int32_t *d = dst + m.row_ptr[4 * n + c];
                for (int64_t k = 0; k < deg; ++k)
                    for (int j = 0; j < 4; ++j) d[4 * k + j] = 4 * m.ncol[b0 + k] + j;
            }
        }
    });
}

}  // namespace vms

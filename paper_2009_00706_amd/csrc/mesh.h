// Host-side mesh structures of libvms (internal header).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace vms {

struct TreeIn {
    int64_t n;
    const int32_t *ax, *ay, *az;
    const uint8_t *level;
    int max_level;
};

struct MeshHost {
    int64_t n_el = 0, n_nodes = 0, n_hanging = 0, nnz = 0;
    std::vector<uint64_t> vert_key;   // unique corner positions, Morton sorted
    std::vector<int8_t> vert_type;    // 1 regular, 2 edge-hanging, 4 face-hanging
    std::vector<int32_t> elem_vert;   // [E][8] vertex of each corner
    std::vector<uint64_t> node_key;   // independent nodes, Morton sorted
    std::vector<int32_t> masters;     // [E][8] master node per slot, -1 unused
    std::vector<uint8_t> nslot;       // [E] number of used slots
    std::vector<uint32_t> ccode;      // [E][4] 2-bit weight code of C[a][s] (0, 1/4, 1/2, 1)
    std::vector<uint8_t> has_hang;    // [E] some corner is hanging
    // pattern
    std::vector<int64_t> nrow_ptr;    // node-level rows
    std::vector<int32_t> ncol;
    std::vector<int64_t> row_ptr;     // dof-level CSR (its column indices: fill_col_idx)
    std::vector<int64_t> el_rowbase;  // [E][8] first entry of dof row 4 m_s
    std::vector<int32_t> el_rowlen;   // [E][8] entries per dof row of m_s (4 deg)
    std::vector<uint16_t> el_kk;      // [E][8][8] block index of m_t within row m_s
    std::vector<uint8_t> node_active; // [N]
    std::vector<int32_t> diag_pos;    // [N] block index of the diagonal within the node row
};

uint64_t morton3(uint64_t x, uint64_t y, uint64_t z);
void unmorton3(uint64_t k, int64_t &x, int64_t &y, int64_t &z);

// 0 ok; -1 invalid input; -2 mesh error (balance, chained constraints)
int derive_mesh(const TreeIn &t, MeshHost &m, std::string &err);
// active[e] != 0 for non-IN elements; 0 ok, -1 internal, -6 unsupported
int build_pattern(MeshHost &m, const std::vector<uint8_t> &active, std::string &err);
// dof-level column indices (nnz int32) of the pattern, written to dst
void fill_col_idx(const MeshHost &m, int32_t *dst);

}  // namespace vms

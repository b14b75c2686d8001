// Host packing of a triangle surface for the exact in-out kernels of libvms
// (internal header): triangle coordinates and boxes, and a (y, z) bin grid of
// the triangles for rays along +x or -x. The device pointers of S are left unset; the
// caller places the four arrays in device memory and fills them in.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/vms.h"
#include "kernels.h"

namespace vms {

struct SurfacePack {
    vmsk::SurfDev S{};
    std::vector<double> tv;     // [n_tri][9]
    std::vector<double> tbox;   // [n_tri][6]
    std::vector<int32_t> off;   // [nby * nbz + 1]
    std::vector<int32_t> ids;   // triangle ids per bin
};

// Validates the surface (indices, finite vertices, closed and consistently
// oriented) and packs it. Returns VMS_OK, VMS_EINVAL or VMS_EMESH (err set).
int pack_surface(const vms_surface *s, SurfacePack &P, std::string &err);

}  // namespace vms

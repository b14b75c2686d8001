// Allocation-free exact in-out labels of libvms (gfx950).
//
// inout_classify_static answers what inout_classify answers in exact mode,
// for callers that cannot allocate device memory: the surface's staging (the
// packed triangles, their boxes and the (y, z) bin grid that the exact ray
// test reads) goes into the file-scope device array `scratch` below instead
// of library allocations. Each GPU holds its own copy of the array, from the
// first call on it until the process ends; its device address is looked up
// once per device (hipGetSymbolAddress with that device current) and only
// that address is ever handed to copies and kernels. Every call on a GPU
// reuses the same array, so calls that overlap on one GPU race; each call
// completes (synchronises its stream) before it returns.
#include "../../include/vms.h"

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "kernels.h"
#include "surface_pack.h"

static constexpr size_t SCRATCH_BYTES = (size_t)VMS_STATIC_SCRATCH_MIB << 20;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
unsigned char *g_ptr[MAX_DEVICES] = {};  // device address of `scratch`, per device
std::string g_err = "no error";

int sfail(int code, const std::string &m) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_err = m;
    return code;
}

// Device address of the current device's array (looked up on first use).
int scratch_ptr(unsigned char **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES)
        return sfail(VMS_EHIP, "no current device");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            g_err = std::string("scratch address lookup failed: ") + hipGetErrorString(e);
            return VMS_EHIP;
        }
        g_ptr[dev] = (unsigned char *)p;
    }
    *out = g_ptr[dev];
    return VMS_OK;
}

size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

int inout_classify_static(const vms_surface *surf, const double *px, const double *py,
                          const double *pz, int64_t n, uint8_t *labels, void *stream) {
    if (n < 0 || (n > 0 && (!px || !py || !pz || !labels)))
        return sfail(VMS_EINVAL, "null argument or negative size");
    vms::SurfacePack P;
    std::string err;
    int rc = vms::pack_surface(surf, P, err);
    if (rc) return sfail(rc, err);
    const size_t b_tv = up256(P.tv.size() * sizeof(double));
    const size_t b_tb = up256(P.tbox.size() * sizeof(double));
    const size_t b_off = up256(P.off.size() * sizeof(int32_t));
    const size_t b_ids = up256(P.ids.size() * sizeof(int32_t));
    const size_t need = b_tv + b_tb + b_off + b_ids;
    if (need > SCRATCH_BYTES)
        return sfail(VMS_EOVERFLOW, "surface staging needs " + std::to_string(need) +
                                        " bytes, above the static scratch of " +
                                        std::to_string(SCRATCH_BYTES) + " bytes");
    unsigned char *base = nullptr;
    if ((rc = scratch_ptr(&base))) return rc;
    hipStream_t st = (hipStream_t)stream;
    vmsk::SurfDev S = P.S;
    double *d_tv = (double *)base;
    double *d_tb = (double *)(base + b_tv);
    int32_t *d_off = (int32_t *)(base + b_tv + b_tb);
    int32_t *d_ids = (int32_t *)(base + b_tv + b_tb + b_off);
    if (hipMemcpyAsync(d_tv, P.tv.data(), P.tv.size() * sizeof(double), hipMemcpyHostToDevice, st) ||
        hipMemcpyAsync(d_tb, P.tbox.data(), P.tbox.size() * sizeof(double), hipMemcpyHostToDevice, st) ||
        hipMemcpyAsync(d_off, P.off.data(), P.off.size() * sizeof(int32_t), hipMemcpyHostToDevice, st) ||
        (P.ids.size() &&
         hipMemcpyAsync(d_ids, P.ids.data(), P.ids.size() * sizeof(int32_t), hipMemcpyHostToDevice, st)))
        return sfail(VMS_EHIP, "copy into the static scratch failed");
    S.tv = d_tv;
    S.tbox = d_tb;
    S.bin_off = d_off;
    S.bin_tri = d_ids;
    vmsk::launch_point_labels(st, S, n, px, py, pz, labels, nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return sfail(VMS_EHIP, std::string("launch failed: ") + hipGetErrorString(e));
    // the host staging dies with this call and the next call reuses the array
    if (hipStreamSynchronize(st) != hipSuccess) return sfail(VMS_EHIP, "stream synchronisation failed");
    return VMS_OK;
}

const char *inout_static_last_error(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_err.c_str();
}

}  // extern "C"

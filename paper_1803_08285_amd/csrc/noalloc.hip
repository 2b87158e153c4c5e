// sgwb_make_maps_band without allocation or caller workspace.
//
// The workspace of sgwb_make_maps_band (data- and pixel-side matrix operands,
// the form record, Bessel amplitudes, broadband partial sums) comes from a
// fixed array in device memory instead of the caller.  The array is a
// file-scope __device__ variable: every GPU the library runs on holds its own
// copy from the module's load there until the process ends.  Host code never
// uses the array's name as an address (on the host it is only a stand-in for
// the symbol): the device address is looked up once per device with
// hipGetSymbolAddress and kept.  Nothing is allocated or freed here, and the
// kernels need no cleared memory (every word they read is written first in
// the same call).
#include <mutex>

#include "sgwb_internal.h"

namespace {

constexpr size_t kScratchBytes = SGWB_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "scratch size is a multiple of the workspace alignment");

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};  // device address of `scratch` on each device, once looked up

// Device address of this device's scratch array (looked up on the first call
// on the device, with that device current).
int scratch_address(void **out)
{
    int dev = -1;
    int rc = sgwb::check_hip(hipGetDevice(&dev), "make_maps_band_noalloc: hipGetDevice");
    if (rc) return rc;
    if (dev < 0 || dev >= kMaxDevices)
        return sgwb::set_error(SGWB_EUNSUPPORTED, "make_maps_band_noalloc: device index %d beyond %d", dev,
                               kMaxDevices);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        rc = sgwb::check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)),
                             "make_maps_band_noalloc: hipGetSymbolAddress");
        if (rc) return rc;
        if (!p || (uintptr_t)p % 256)
            return sgwb::set_error(SGWB_EDEVICE, "make_maps_band_noalloc: scratch address %p not 256-byte aligned", p);
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return SGWB_OK;
}

}  // namespace

extern "C" int sgwb_make_maps_band_noalloc(const float *C, const float *w, int64_t ldc, int32_t nt, int32_t nf,
                                           const sgwb_fgrid *fg, int64_t k0, const float *gamma, const double *tau,
                                           int32_t npix, uint32_t flags, const float *H, int32_t k_lo, int32_t k_hi,
                                           float *X, float *Gam, float *Xbb, float *Gbb, hipStream_t stream)
{
    const size_t need = sgwb_make_maps_band_workspace_size(nt, nf, npix, flags);
    if (need == 0) return sgwb::set_error(SGWB_EINVAL, "make_maps_band_noalloc: nt, nf, npix must be >= 1");
    if (need > kScratchBytes)
        return sgwb::set_error(SGWB_ENOMEM,
                               "make_maps_band_noalloc: this call needs %zu bytes of workspace, the fixed scratch "
                               "array holds %zu (use sgwb_make_maps_band with a workspace)",
                               need, kScratchBytes);
    void *ws = nullptr;
    int rc = scratch_address(&ws);
    if (rc) return rc;
    return sgwb_make_maps_band(C, w, ldc, nt, nf, fg, k0, gamma, tau, npix, flags, H, k_lo, k_hi, X, Gam, Xbb, Gbb,
                               ws, kScratchBytes, stream);
}

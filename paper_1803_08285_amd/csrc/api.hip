// C ABI of libsgwb: argument checks, host-side detector set-up, launches.
#include <math.h>
#include <stdlib.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "broadband.h"
#include "fisher_general.h"
#include "sgwb_internal.h"

namespace sgwb {

static thread_local char g_err[512] = "";

int set_error(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

int check_hip(hipError_t e, const char *what)
{
    if (e == hipSuccess) return SGWB_OK;
    return set_error(SGWB_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Earth-fixed position (m) and response tensor D = (u u^T - v v^T) / 2 of an
// L-shaped detector: u = x-arm, v = y-arm, both horizontal, x-arm azimuth
// counter-clockwise from local East.
static void detector_frame(const sgwb_detector &d, double r[3], double D[9])
{
    const double k = kPi / 180.0;
    const double sl = sin(d.lat_deg * k), cl = cos(d.lat_deg * k);
    const double so = sin(d.lon_deg * k), co = cos(d.lon_deg * k);
    const double sa = sin(d.xarm_az_deg * k), ca = cos(d.xarm_az_deg * k);
    r[0] = kEarthRadius * cl * co;
    r[1] = kEarthRadius * cl * so;
    r[2] = kEarthRadius * sl;
    const double east[3] = {-so, co, 0.0};
    const double north[3] = {-sl * co, -sl * so, cl};
    double u[3], v[3];
    for (int i = 0; i < 3; ++i) {
        u[i] = ca * east[i] + sa * north[i];
        v[i] = ca * north[i] - sa * east[i];
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) D[3 * i + j] = 0.5 * (u[i] * u[j] - v[i] * v[j]);
}

static bool finite_det(const sgwb_detector &d)
{
    return isfinite(d.lat_deg) && isfinite(d.lon_deg) && isfinite(d.xarm_az_deg) && fabs(d.lat_deg) <= 90.0;
}

template <typename G>
static int build_geometry_impl(const sgwb_baseline *bl, int32_t nside, const sgwb_tgrid *tg, G *gamma,
                               double *tau, hipStream_t stream)
{
    if (!bl || !tg || !gamma || !tau) return set_error(SGWB_EINVAL, "build_geometry: null pointer");
    if (!is_pow2_nside(nside)) return set_error(SGWB_EINVAL, "build_geometry: nside %d is not a power of two in [1, 8192]", nside);
    if (tg->nt < 1 || tg->nt > 65535) return set_error(SGWB_EINVAL, "build_geometry: nt %d out of [1, 65535]", tg->nt);
    if (!isfinite(tg->t0_s) || !isfinite(tg->stride_s) || !isfinite(tg->seg_dur_s))
        return set_error(SGWB_EINVAL, "build_geometry: non-finite time grid");
    if (!finite_det(bl->a) || !finite_det(bl->b)) return set_error(SGWB_EINVAL, "build_geometry: bad detector");
    if (((uintptr_t)gamma % sizeof(G)) || ((uintptr_t)tau % 8)) return set_error(SGWB_EINVAL, "build_geometry: misaligned output");
    GeomArgs a;
    double ra[3], rb[3];
    detector_frame(bl->a, ra, a.DA);
    detector_frame(bl->b, rb, a.DB);
    for (int i = 0; i < 3; ++i) a.dx[i] = ra[i] - rb[i];
    a.t0 = tg->t0_s;
    a.stride = tg->stride_s;
    a.half_dur = 0.5 * tg->seg_dur_s;
    a.nt = tg->nt;
    a.nside = nside;
    a.npix = 12LL * nside * nside;
    return check_hip(launch_geometry<G>(a, gamma, tau, stream), "geometry kernel launch");
}

static int check_grid(const sgwb_fgrid *fg)
{
    if (!fg) return set_error(SGWB_EINVAL, "null frequency grid");
    if (!isfinite(fg->f0_hz) || !isfinite(fg->df_hz) || fg->df_hz <= 0.0)
        return set_error(SGWB_EINVAL, "frequency grid must be finite with df > 0");
    return SGWB_OK;
}

// C may be null only for callers that read no CSD (c_optional).
template <typename T>
static int check_maps_args(const T *C, const T *w, int64_t ldc, int32_t nt, int32_t nf, const sgwb_fgrid *fg,
                           int64_t k0, const T *gamma, const double *tau, int32_t npix, uint32_t flags,
                           MapArgs *a, bool c_optional = false)
{
    if ((!C && !c_optional) || !w || !gamma || !tau) return set_error(SGWB_EINVAL, "make_maps: null input pointer");
    if (nt < 1 || nf < 1 || npix < 1) return set_error(SGWB_EINVAL, "make_maps: nt, nf, npix must be >= 1");
    if (ldc < nf) return set_error(SGWB_EINVAL, "make_maps: ldc %lld < nf %d", (long long)ldc, nf);
    if (k0 < 0) return set_error(SGWB_EINVAL, "make_maps: k0 < 0");
    if (flags & ~(SGWB_MAPS_ANTIPODAL | SGWB_MAPS_VALU_X)) return set_error(SGWB_EINVAL, "make_maps: unknown flag bits");
    int rc = check_grid(fg);
    if (rc) return rc;
    if (((uintptr_t)C % (2 * sizeof(T))) || ((uintptr_t)w % sizeof(T)) || ((uintptr_t)gamma % sizeof(T)) ||
        ((uintptr_t)tau % 8))
        return set_error(SGWB_EINVAL, "make_maps: misaligned input");
    a->ldc = ldc;
    a->k0 = k0;
    a->nt = nt;
    a->nf = nf;
    a->npix = npix;
    a->f0 = fg->f0_hz;
    a->df = fg->df_hz;
    a->nside = 0;
    if (flags & SGWB_MAPS_ANTIPODAL) {
        a->nside = nside_of_npix(npix);
        if (a->nside == 0)
            return set_error(SGWB_EINVAL, "make_maps: SGWB_MAPS_ANTIPODAL needs npix = 12 nside^2, nside a power of two");
    }
    return SGWB_OK;
}

template <typename T>
static int reduce_band_impl(const T *X, const T *Gam, const T *H, int32_t nf, int32_t npix, int32_t k_lo,
                            int32_t k_hi, T *Xbb, T *Gbb, void *work, size_t work_bytes, hipStream_t stream)
{
    if (nf < 1 || npix < 1) return set_error(SGWB_EINVAL, "reduce_band: nf, npix must be >= 1");
    if (!(0 <= k_lo && k_lo <= k_hi && k_hi <= nf))
        return set_error(SGWB_EINVAL, "reduce_band: need 0 <= k_lo <= k_hi <= nf");
    const bool doX = X && Xbb, doG = Gam && Gbb;
    if ((X != nullptr) != (Xbb != nullptr) || (Gam != nullptr) != (Gbb != nullptr))
        return set_error(SGWB_EINVAL, "reduce_band: X/Xbb and Gam/Gbb must be given in pairs");
    if (!doX && !doG) return set_error(SGWB_EINVAL, "reduce_band: nothing to do");
    if (doG && !H) return set_error(SGWB_EINVAL, "reduce_band: H needed for Gbb");
    if (work && ((uintptr_t)work % 256)) return set_error(SGWB_EINVAL, "reduce_band: workspace not 256-byte aligned");
    return check_hip(launch_band<T>(doX ? X : nullptr, doG ? Gam : nullptr, H, nf, npix, k_lo, k_hi,
                                    doX ? Xbb : nullptr, doG ? Gbb : nullptr, work, work_bytes, stream),
                     "band kernel launch");
}

int check_maps_args_f32(const float *C, const float *w, int64_t ldc, int32_t nt, int32_t nf, const sgwb_fgrid *fg,
                        int64_t k0, const float *gamma, const double *tau, int32_t npix, uint32_t flags,
                        MapArgs *a)
{
    return check_maps_args<float>(C, w, ldc, nt, nf, fg, k0, gamma, tau, npix, flags, a);
}

// Wave-tile shape of the single-call beam GEMM; SGWB_BEAM_SHAPE=2x4 or 4x4
// overrides the default.
static int default_beam_shape()
{
    static int shape = [] {
        const char *e = getenv("SGWB_BEAM_SHAPE");
        if (e && strcmp(e, "4x4") == 0) return kBeamShape4x4;
        if (e && strcmp(e, "2x4") == 0) return kBeamShape2x4;
        return kBeamShape2x4;
    }();
    return shape;
}

// Dirty-map kernel choice: SGWB_X_KERNEL=valu forces the vector-unit recurrence,
// otherwise the matrix-core form runs where it applies.
constexpr int kXKernelAuto = 0, kXKernelValu = 1;
static int x_kernel_choice()
{
    static int k = [] {
        const char *e = getenv("SGWB_X_KERNEL");
        return (e && strcmp(e, "valu") == 0) ? kXKernelValu : kXKernelAuto;
    }();
    return k;
}

// What the last map call on this thread did for X: the host's choice, and for
// the matrix-core forms the device address of the call's form record and the
// stream it was queued on.
struct XFormRecord {
    int host = SGWB_XFORM_NONE;
    const double *rec = nullptr;
    hipStream_t stream = nullptr;
};
static thread_local XFormRecord g_xform;
constexpr int kXFormDevice = -2;  // host marker: the matrix-core prep chose on the device

static void note_xform(int host, const double *rec = nullptr, hipStream_t stream = nullptr)
{
    g_xform.host = host;
    g_xform.rec = rec;
    g_xform.stream = stream;
}

// Matrix-core dirty map for this call?  Applies with the antipodal flag where
// a form can meet the Earth's delay bound at this df, unless the vector form is
// forced.  *rc = SGWB_ENOMEM when it applies and a workspace was given that
// cannot hold it (no silent fallback); without a workspace the vector form runs.
static bool want_xm(const MapArgs &a, uint32_t flags, const void *workspace, size_t workspace_bytes,
                    size_t need, const char *who, int *rc)
{
    *rc = SGWB_OK;
    if ((flags & SGWB_MAPS_VALU_X) || x_kernel_choice() == kXKernelValu || !xm_eligible(a) || !workspace) return false;
    if (workspace_bytes < need) {
        *rc = set_error(SGWB_ENOMEM, "%s: the matrix-core dirty map needs a workspace of %zu bytes, %zu given", who,
                        need, workspace_bytes);
        return false;
    }
    return true;
}

}  // namespace sgwb

using namespace sgwb;

extern "C" {

int sgwb_last_x_form(int32_t *form)
{
    if (!form) return set_error(SGWB_EINVAL, "last_x_form: null pointer");
    *form = g_xform.host;
    if (g_xform.host != kXFormDevice) return SGWB_OK;  // host-side choices are final
    double rec[2];
    int rc = check_hip(hipStreamSynchronize(g_xform.stream), "last_x_form: stream synchronisation");
    if (!rc) rc = check_hip(hipMemcpy(rec, g_xform.rec, sizeof rec, hipMemcpyDeviceToHost), "last_x_form: read back");
    if (rc) {
        *form = SGWB_XFORM_NONE;
        return rc;
    }
    const int code = (int)rec[1];
    if (code == kXFormRejected) {
        *form = SGWB_XFORM_NONE;
        return set_error(SGWB_EINVAL, "last_x_form: the seeds failed the antipodal check or the delay bound "
                                      "(max |tau| = %.6g s); X was written as NaN", rec[0]);
    }
    *form = code;
    return SGWB_OK;
}

const char *sgwb_status_string(int status)
{
    switch (status) {
    case SGWB_OK: return "ok";
    case SGWB_EINVAL: return "invalid argument";
    case SGWB_ENOMEM: return "out of memory / workspace too small";
    case SGWB_EDEVICE: return "HIP device error";
    case SGWB_EBUSY: return "server queue full";
    case SGWB_EAGAIN: return "not finished yet";
    case SGWB_EUNSUPPORTED: return "unsupported device or option";
    default: return "unknown status";
    }
}

const char *sgwb_last_error(void) { return g_err; }

int sgwb_device_supported(void)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return check_hip(hipGetLastError(), "hipGetDevice");
    hipDeviceProp_t p;
    hipError_t e = hipGetDeviceProperties(&p, dev);
    if (e != hipSuccess) return check_hip(e, "hipGetDeviceProperties");
    return strncmp(p.gcnArchName, "gfx950", 6) == 0 ? 1 : 0;
}

int sgwb_build_geometry(const sgwb_baseline *bl, int32_t nside, const sgwb_tgrid *tg, float *gamma, double *tau,
                        hipStream_t stream)
{
    return build_geometry_impl<float>(bl, nside, tg, gamma, tau, stream);
}

int sgwb_build_geometry_f64(const sgwb_baseline *bl, int32_t nside, const sgwb_tgrid *tg, double *gamma,
                            double *tau, hipStream_t stream)
{
    return build_geometry_impl<double>(bl, nside, tg, gamma, tau, stream);
}

static size_t up256(size_t n) { return (n + 255) / 256 * 256; }

size_t sgwb_make_maps_workspace_size(int32_t nt, int32_t nf, int32_t npix, uint32_t flags)
{
    if (nt < 1 || nf < 1 || npix < 1) return 0;
    const int32_t ncol = (flags & SGWB_MAPS_ANTIPODAL) ? npix / 2 : npix;
    size_t n = up256(beam_workspace_bytes(nt, nf, ncol));
    // room for the matrix-core dirty map (largest strip count over all k0)
    if (flags & SGWB_MAPS_ANTIPODAL) n += up256(xm_workspace_bytes(63, nt, nf, npix));
    return n;
}

int sgwb_make_maps(const float *C, const float *w, int64_t ldc, int32_t nt, int32_t nf, const sgwb_fgrid *fg,
                   int64_t k0, const float *gamma, const double *tau, int32_t npix, uint32_t flags, float *X,
                   float *Gam, void *workspace, size_t workspace_bytes, hipStream_t stream)
{
    note_xform(SGWB_XFORM_NONE);
    MapArgs a;
    int rc = check_maps_args<float>(C, w, ldc, nt, nf, fg, k0, gamma, tau, npix, flags, &a);
    if (rc) return rc;
    if (workspace && (uintptr_t)workspace % 256) return set_error(SGWB_EINVAL, "make_maps: workspace not 256-byte aligned");
    const int32_t ncol = a.nside > 0 ? npix / 2 : npix;
    const size_t beam_bytes = up256(beam_workspace_bytes(nt, nf, ncol));
    if (Gam && (!workspace || workspace_bytes < beam_bytes))
        return set_error(SGWB_ENOMEM, "make_maps: workspace of %zu bytes needed, %zu given",
                         sgwb_make_maps_workspace_size(nt, nf, npix, flags), workspace ? workspace_bytes : (size_t)0);
    if (X) {
        const size_t xm_bytes = xm_workspace_bytes(k0, nt, nf, npix);
        const bool use_xm = want_xm(a, flags, workspace, workspace_bytes, beam_bytes + xm_bytes, "make_maps", &rc);
        if (rc) return rc;
        if (use_xm) {
            const double *rec = nullptr;
            rc = check_hip(launch_dirty_map_mfma(a, C, w, gamma, tau, X, reinterpret_cast<char *>(workspace) + beam_bytes,
                                                 stream, &rec),
                           "dirty-map (matrix cores) launch");
            if (!rc) note_xform(kXFormDevice, rec, stream);
        } else {
            rc = check_hip(launch_dirty_map<float>(a, C, w, gamma, tau, X, stream), "dirty-map kernel launch");
            if (!rc) note_xform(SGWB_XFORM_VALU);
        }
        if (rc) return rc;
    }
    if (Gam) {
        rc = check_hip(launch_beam_bf16x3(a, w, gamma, Gam, workspace, default_beam_shape(), stream), "beam kernel launch");
        if (rc) return rc;
    }
    return SGWB_OK;
}

size_t sgwb_fisher_overlap_workspace_size(int32_t nt, int32_t nf, int32_t npix, uint32_t flags)
{
    if (nt < 1 || nf < 1 || npix < 1) return 0;
    const int32_t ncol = (flags & SGWB_MAPS_ANTIPODAL) ? npix / 2 : npix;
    size_t n = up256(beam_workspace_bytes(nt, nf, ncol)) + up256(pair_workspace_bytes(nt, nf, npix));
    if (flags & SGWB_MAPS_ANTIPODAL) n += up256(xm_workspace_bytes(63, nt, nf, npix));
    return n;
}

int sgwb_fisher_overlap(const float *v, const float *u, const float *wn, int64_t ldc, int32_t nt, int32_t nf,
                        const sgwb_fgrid *fg, int64_t k0, const float *gamma, const double *tau, int32_t npix,
                        uint32_t flags, float *Gam, void *workspace, size_t workspace_bytes, hipStream_t stream)
{
    note_xform(SGWB_XFORM_NONE);
    if (!Gam) return set_error(SGWB_EINVAL, "fisher_overlap: null Gam");
    if (!u || !wn) return set_error(SGWB_EINVAL, "fisher_overlap: null neighbour series");
    if (((uintptr_t)u % 4) || ((uintptr_t)wn % 4)) return set_error(SGWB_EINVAL, "fisher_overlap: misaligned input");
    // v plays the role of w; no CSD is read
    MapArgs a;
    int rc = check_maps_args<float>(nullptr, v, ldc, nt, nf, fg, k0, gamma, tau, npix, flags, &a, true);
    if (rc) return rc;
    if (!workspace || (uintptr_t)workspace % 256) return set_error(SGWB_EINVAL, "fisher_overlap: workspace null or not 256-byte aligned");
    const int32_t ncol = a.nside > 0 ? npix / 2 : npix;
    const size_t beam_bytes = up256(beam_workspace_bytes(nt, nf, ncol));
    const size_t pair_bytes = up256(pair_workspace_bytes(nt, nf, npix));
    if (workspace_bytes < beam_bytes + pair_bytes)
        return set_error(SGWB_ENOMEM, "fisher_overlap: workspace of %zu bytes needed, %zu given",
                         sgwb_fisher_overlap_workspace_size(nt, nf, npix, flags), workspace_bytes);
    char *ws = reinterpret_cast<char *>(workspace);
    const bool use_xm = want_xm(a, flags, workspace, workspace_bytes,
                                beam_bytes + pair_bytes + xm_workspace_bytes(k0, nt, nf, npix), "fisher_overlap", &rc);
    if (rc) return rc;
    rc = check_hip(launch_beam_bf16x3(a, v, gamma, Gam, ws, default_beam_shape(), stream), "beam kernel launch");
    if (rc) return rc;
    const double *rec = nullptr;
    rc = check_hip(launch_fisher_neighbours(a, u, wn, gamma, tau, Gam, ws + beam_bytes, ws + beam_bytes + pair_bytes,
                                            use_xm, stream, &rec),
                   "fisher neighbour-term launch");
    if (!rc) note_xform(use_xm ? kXFormDevice : SGWB_XFORM_VALU, rec, stream);
    return rc;
}

int sgwb_fold(const float *C, const float *sinv, const uint8_t *present, int64_t ldc, int32_t ndays, int32_t nt,
              int32_t nf, double W, float *v, float *u, float *w, float *x, hipStream_t stream)
{
    if (!C || !sinv || !present || !v || !u || !w || !x) return set_error(SGWB_EINVAL, "fold: null pointer");
    if (ndays < 1 || nt < 1 || nf < 1) return set_error(SGWB_EINVAL, "fold: ndays, nt, nf must be >= 1");
    if (ldc < nf) return set_error(SGWB_EINVAL, "fold: ldc %lld < nf %d", (long long)ldc, nf);
    if (!std::isfinite(W) || W < 0.0) return set_error(SGWB_EINVAL, "fold: W must be finite and >= 0");
    if (((uintptr_t)C % 8) || ((uintptr_t)sinv % 4) || ((uintptr_t)x % 8) || ((uintptr_t)v % 4) ||
        ((uintptr_t)u % 4) || ((uintptr_t)w % 4))
        return set_error(SGWB_EINVAL, "fold: misaligned pointer");
    if (nt > 65535) return set_error(SGWB_EINVAL, "fold: nt > 65535 segments per day");
    return check_hip(launch_fold(C, sinv, present, ldc, ndays, nt, nf, W, v, u, w, x, stream), "fold kernel launch");
}

int sgwb_network_sum(const float *const *maps, int32_t nmaps, int64_t n, float *out, hipStream_t stream)
{
    if (!maps || !out) return set_error(SGWB_EINVAL, "network_sum: null pointer");
    if (nmaps < 1 || nmaps > kMaxNetworkMaps)
        return set_error(SGWB_EINVAL, "network_sum: nmaps must be 1..%d", kMaxNetworkMaps);
    if (n < 1) return set_error(SGWB_EINVAL, "network_sum: n must be >= 1");
    MapList l{};
    l.n = nmaps;
    for (int32_t m = 0; m < nmaps; ++m) {
        if (!maps[m]) return set_error(SGWB_EINVAL, "network_sum: map %d is null", m);
        l.p[m] = maps[m];
    }
    return check_hip(launch_network_sum(l, n, out, stream), "network-sum kernel launch");
}

int sgwb_contract_pixels(const float *M, int32_t nf, int32_t npix, const int32_t *pix, int32_t nsel, float *out,
                         hipStream_t stream)
{
    if (!M || !out) return set_error(SGWB_EINVAL, "contract_pixels: null pointer");
    if (nf < 1 || npix < 1) return set_error(SGWB_EINVAL, "contract_pixels: nf, npix must be >= 1");
    if (pix && nsel < 0) return set_error(SGWB_EINVAL, "contract_pixels: nsel < 0");
    if ((uintptr_t)pix % 4) return set_error(SGWB_EINVAL, "contract_pixels: misaligned pixel list");
    return check_hip(launch_contract(M, nf, npix, pix, pix ? nsel : 0, out, stream), "contraction kernel launch");
}

size_t sgwb_fisher_full_workspace_size(const sgwb_fgrid *fg, int64_t k0, int32_t chi, int32_t nt, int32_t npix)
{
    if (!fg || !std::isfinite(fg->f0_hz) || !std::isfinite(fg->df_hz) || fg->df_hz <= 0.0 || k0 < 0 || chi < 1 ||
        nt < 1 || npix < 1)
        return 0;
    const double f_max = fg->f0_hz + (double)(k0 + chi - 1) * fg->df_hz;
    if (!fisher_full_band_ok(f_max)) return 0;
    return fisher_full_workspace_bytes(f_max, chi, nt, npix);
}

int sgwb_fisher_full(const float *a, const float *b, int32_t rank, const float *H, int32_t nf, const sgwb_fgrid *fg,
                     int64_t k0, int32_t clo, int32_t chi, const float *gamma, const double *tau, int32_t nt,
                     int32_t npix, uint32_t flags, float *G, void *workspace, size_t workspace_bytes,
                     hipStream_t stream)
{
    if (!a || !b || !H || !fg || !gamma || !tau || !G) return set_error(SGWB_EINVAL, "fisher_full: null pointer");
    if (nt < 1 || nf < 1 || npix < 1) return set_error(SGWB_EINVAL, "fisher_full: nt, nf, npix must be >= 1");
    if (rank < 1 || rank > 64) return set_error(SGWB_EINVAL, "fisher_full: rank must be 1..64");
    if (!(0 <= clo && clo < chi && chi <= nf))
        return set_error(SGWB_EINVAL, "fisher_full: band [%d, %d) not inside [0, %d)", clo, chi, nf);
    if (!std::isfinite(fg->f0_hz) || !std::isfinite(fg->df_hz) || fg->df_hz <= 0.0 || fg->f0_hz < 0.0 || k0 < 0)
        return set_error(SGWB_EINVAL, "fisher_full: bad frequency grid");
    if (!fisher_full_band_ok(fg->f0_hz + (double)(k0 + chi - 1) * fg->df_hz))
        return set_error(SGWB_EINVAL, "fisher_full: band reaches above 24 kHz");
    if (((uintptr_t)a % 4) || ((uintptr_t)b % 4) || ((uintptr_t)H % 4) || ((uintptr_t)gamma % 4) ||
        ((uintptr_t)tau % 8) || ((uintptr_t)G % 4))
        return set_error(SGWB_EINVAL, "fisher_full: misaligned pointer");
    if (flags & ~SGWB_MAPS_ANTIPODAL) return set_error(SGWB_EINVAL, "fisher_full: unknown flag bits");
    int64_t nside = 0;
    if (flags & SGWB_MAPS_ANTIPODAL) {
        nside = nside_of_npix(npix);
        if (nside == 0)
            return set_error(SGWB_EINVAL, "fisher_full: SGWB_MAPS_ANTIPODAL needs npix = 12 nside^2, nside a power of two");
    }
    const int64_t ntile = ((int64_t)npix + 63) / 64;
    if (ntile * (ntile + 1) / 2 > 0x7fffffff) return set_error(SGWB_EINVAL, "fisher_full: npix too large");
    if (!workspace || (uintptr_t)workspace % 256)
        return set_error(SGWB_EINVAL, "fisher_full: workspace null or not 256-byte aligned");
    const size_t need = sgwb_fisher_full_workspace_size(fg, k0, chi, nt, npix);
    if (workspace_bytes < need)
        return set_error(SGWB_ENOMEM, "fisher_full: workspace of %zu bytes needed, %zu given", need, workspace_bytes);
    return check_hip(launch_fisher_full(a, b, rank, H, nf, clo, chi, fg->f0_hz, fg->df_hz, k0, gamma, tau, nt, npix,
                                        nside, G, workspace, stream),
                     "full Fisher launch");
}

// Checks shared by the general-weights size query and entry point; 0 or an
// error code (with the message set).
static int check_fisher_general(const sgwb_fgrid *fg, int64_t k0, int32_t clo, int32_t chi, int32_t nf, int32_t nt,
                                int32_t npix, uint32_t flags, int64_t *nside)
{
    if (!fg) return set_error(SGWB_EINVAL, "fisher_full_general: null pointer");
    if (nt < 1 || nf < 1 || npix < 1) return set_error(SGWB_EINVAL, "fisher_full_general: nt, nf, npix must be >= 1");
    if (nt > 65535) return set_error(SGWB_EINVAL, "fisher_full_general: nt above 65535");
    if (!(0 <= clo && clo < chi && chi <= nf))
        return set_error(SGWB_EINVAL, "fisher_full_general: band [%d, %d) not inside [0, %d)", clo, chi, nf);
    if (!std::isfinite(fg->f0_hz) || !std::isfinite(fg->df_hz) || fg->df_hz <= 0.0 || fg->f0_hz < 0.0 || k0 < 0)
        return set_error(SGWB_EINVAL, "fisher_full_general: bad frequency grid");
    if (!fisher_full_band_ok(fg->f0_hz + (double)(k0 + chi - 1) * fg->df_hz))
        return set_error(SGWB_EINVAL, "fisher_full_general: band reaches above 24 kHz");
    if (flags & ~SGWB_MAPS_ANTIPODAL) return set_error(SGWB_EINVAL, "fisher_full_general: unknown flag bits");
    *nside = 0;
    if (flags & SGWB_MAPS_ANTIPODAL) {
        *nside = nside_of_npix(npix);
        if (*nside == 0)
            return set_error(SGWB_EINVAL,
                             "fisher_full_general: SGWB_MAPS_ANTIPODAL needs npix = 12 nside^2, nside a power of two");
    }
    const int64_t ntile = ((int64_t)npix + 63) / 64;
    if (ntile * (ntile + 1) / 2 > 0x7fffffff) return set_error(SGWB_EINVAL, "fisher_full_general: npix too large");
    return SGWB_OK;
}

size_t sgwb_fisher_full_general_workspace_size(const sgwb_fgrid *fg, int64_t k0, int32_t clo, int32_t chi,
                                               int32_t nt, int32_t npix, uint32_t flags)
{
    int64_t nside = 0;
    if (!fg || check_fisher_general(fg, k0, clo, chi, chi, nt, npix, flags, &nside)) return 0;
    return fisher_full_general_workspace_bytes(fg->f0_hz, fg->df_hz, k0, clo, chi, nt, npix, nside);
}

int sgwb_fisher_full_general(const float *w, int64_t ldw, const float *H, int32_t nf, const sgwb_fgrid *fg,
                             int64_t k0, int32_t clo, int32_t chi, const float *gamma, const double *tau, int32_t nt,
                             int32_t npix, uint32_t flags, float *G, void *workspace, size_t workspace_bytes,
                             hipStream_t stream)
{
    if (!w || !H || !fg || !gamma || !tau || !G) return set_error(SGWB_EINVAL, "fisher_full_general: null pointer");
    int64_t nside = 0;
    int rc = check_fisher_general(fg, k0, clo, chi, nf, nt, npix, flags, &nside);
    if (rc) return rc;
    if (ldw < nf) return set_error(SGWB_EINVAL, "fisher_full_general: ldw < nf");
    if (((uintptr_t)w % 4) || ((uintptr_t)H % 4) || ((uintptr_t)gamma % 4) || ((uintptr_t)tau % 8) ||
        ((uintptr_t)G % 4))
        return set_error(SGWB_EINVAL, "fisher_full_general: misaligned pointer");
    if (!workspace || (uintptr_t)workspace % 256)
        return set_error(SGWB_EINVAL, "fisher_full_general: workspace null or not 256-byte aligned");
    const size_t need = sgwb_fisher_full_general_workspace_size(fg, k0, clo, chi, nt, npix, flags);
    if (workspace_bytes < need)
        return set_error(SGWB_ENOMEM, "fisher_full_general: workspace of %zu bytes needed, %zu given", need,
                         workspace_bytes);
    return check_hip(launch_fisher_full_general(w, ldw, H, clo, chi, fg->f0_hz, fg->df_hz, k0, gamma, tau, nt, npix,
                                                nside, G, workspace, stream),
                     "full Fisher (general weights) launch");
}

size_t sgwb_clean_map_workspace_size(int32_t n)
{
    return n < 1 ? 0 : cg_workspace_bytes(n);
}

int sgwb_clean_map_cg(const float *G, const float *X, int32_t n, int32_t niter, float *P, void *workspace,
                      size_t workspace_bytes, hipStream_t stream)
{
    if (!G || !X || !P) return set_error(SGWB_EINVAL, "clean_map_cg: null pointer");
    if (n < 1 || niter < 0) return set_error(SGWB_EINVAL, "clean_map_cg: n must be >= 1 and niter >= 0");
    if (((uintptr_t)G % 4) || ((uintptr_t)X % 4) || ((uintptr_t)P % 4))
        return set_error(SGWB_EINVAL, "clean_map_cg: misaligned pointer");
    if (!workspace || (uintptr_t)workspace % 256)
        return set_error(SGWB_EINVAL, "clean_map_cg: workspace null or not 256-byte aligned");
    if (workspace_bytes < cg_workspace_bytes(n))
        return set_error(SGWB_ENOMEM, "clean_map_cg: workspace of %zu bytes needed, %zu given",
                         cg_workspace_bytes(n), workspace_bytes);
    return check_hip(launch_clean_map_cg(G, X, n, niter, P, workspace, stream), "clean-map launch");
}

int sgwb_make_maps_f64(const double *C, const double *w, int64_t ldc, int32_t nt, int32_t nf,
                       const sgwb_fgrid *fg, int64_t k0, const double *gamma, const double *tau, int32_t npix,
                       uint32_t flags, double *X, double *Gam, hipStream_t stream)
{
    MapArgs a;
    int rc = check_maps_args<double>(C, w, ldc, nt, nf, fg, k0, gamma, tau, npix, flags, &a);
    if (rc) return rc;
    if (X) {
        rc = check_hip(launch_dirty_map<double>(a, C, w, gamma, tau, X, stream), "dirty-map kernel launch");
        if (rc) return rc;
    }
    if (Gam) {
        rc = check_hip(launch_beam_f64(a, w, gamma, Gam, stream), "beam kernel launch");
        if (rc) return rc;
    }
    return SGWB_OK;
}

size_t sgwb_make_maps_band_workspace_size(int32_t nt, int32_t nf, int32_t npix, uint32_t flags)
{
    const size_t base = sgwb_make_maps_workspace_size(nt, nf, npix, flags);
    if (!base) return 0;
    // X partial sums: at most nf / 64 + 2 strips (any k0); Gbb: one weight per segment
    const size_t rows_x = (size_t)nf / 64 + 2;
    return up256(base) + up256(rows_x * npix * sizeof(double)) + up256(band_gamma_scratch_bytes(nt, npix));
}

int sgwb_make_maps_band(const float *C, const float *w, int64_t ldc, int32_t nt, int32_t nf, const sgwb_fgrid *fg,
                        int64_t k0, const float *gamma, const double *tau, int32_t npix, uint32_t flags,
                        const float *H, int32_t k_lo, int32_t k_hi, float *X, float *Gam, float *Xbb, float *Gbb,
                        void *workspace, size_t workspace_bytes, hipStream_t stream)
{
    return sgwb::make_maps_band_seeded(C, w, ldc, nt, nf, fg, k0, gamma, tau, npix, flags, H, k_lo, k_hi, X, Gam, Xbb,
                                       Gbb, workspace, workspace_bytes, nullptr, stream);
}

}  // extern "C"

namespace sgwb {

int seed_products(const float *C, const float *w, int64_t ldc, int32_t nt, int32_t nf, const sgwb_fgrid *fg,
                  int64_t k0, const float *gamma, const double *tau, int32_t npix, void *seeds, hipStream_t stream,
                  bool *made)
{
    *made = false;
    MapArgs a;
    int rc = check_maps_args<float>(C, w, ldc, nt, nf, fg, k0, gamma, tau, npix, SGWB_MAPS_ANTIPODAL, &a);
    if (rc) return rc;
    if (!xm_eligible(a) || x_kernel_choice() == kXKernelValu) return SGWB_OK;  // no matrix-core form to prepare for
    if (!seeds || (uintptr_t)seeds % 256) return set_error(SGWB_EINVAL, "seed products: buffer null or misaligned");
    rc = check_hip(launch_xm_seed_products(a, gamma, tau, seeds, stream), "seed products launch");
    if (!rc) *made = true;
    return rc;
}

int make_maps_band_seeded(const float *C, const float *w, int64_t ldc, int32_t nt, int32_t nf, const sgwb_fgrid *fg,
                          int64_t k0, const float *gamma, const double *tau, int32_t npix, uint32_t flags,
                          const float *H, int32_t k_lo, int32_t k_hi, float *X, float *Gam, float *Xbb, float *Gbb,
                          void *workspace, size_t workspace_bytes, const void *seeds, hipStream_t stream)
{
    note_xform(SGWB_XFORM_NONE);
    if ((X && !Xbb) || (Gam && !Gbb))
        return set_error(SGWB_EINVAL, "make_maps_band: X needs Xbb and Gam needs Gbb");
    if (!Xbb && !Gbb) return set_error(SGWB_EINVAL, "make_maps_band: nothing to compute");
    if (Gbb && !H) return set_error(SGWB_EINVAL, "make_maps_band: null H");
    if (!(0 <= k_lo && k_lo <= k_hi && k_hi <= nf))
        return set_error(SGWB_EINVAL, "make_maps_band: band [%d, %d) not inside [0, %d]", k_lo, k_hi, nf);
    MapArgs a;
    int rc = check_maps_args<float>(C, w, ldc, nt, nf, fg, k0, gamma, tau, npix, flags, &a);
    if (rc) return rc;
    if (!workspace || (uintptr_t)workspace % 256)
        return set_error(SGWB_EINVAL, "make_maps_band: workspace null or not 256-byte aligned");
    const size_t need = sgwb_make_maps_band_workspace_size(nt, nf, npix, flags);
    if (workspace_bytes < need)
        return set_error(SGWB_ENOMEM, "make_maps_band: workspace of %zu bytes needed, %zu given", need,
                         workspace_bytes);
    const size_t base = up256(sgwb_make_maps_workspace_size(nt, nf, npix, flags));
    const size_t rows_x = (size_t)nf / 64 + 2;
    char *ws = reinterpret_cast<char *>(workspace);
    double *part_x = reinterpret_cast<double *>(ws + base);
    double *vband = reinterpret_cast<double *>(ws + base + up256(rows_x * npix * sizeof(double)));
    const int32_t ncol = a.nside > 0 ? npix / 2 : npix;
    const size_t beam_bytes = up256(beam_workspace_bytes(nt, nf, ncol));
    if (Xbb) {
        const bool use_xm =
            want_xm(a, flags, workspace, workspace_bytes, beam_bytes + xm_workspace_bytes(k0, nt, nf, npix),
                    "make_maps_band", &rc);
        if (rc) return rc;
        if (!X && !use_xm)
            return set_error(SGWB_EINVAL,
                             "make_maps_band: Xbb without X needs the matrix-core dirty map (antipodal seeds, "
                             "df <= 0.0344 Hz, no vector-unit request)");
        if (use_xm) {
            // the dirty map writes per-strip partial sums; one small kernel adds them
            MapArgs ab = a;
            ab.band_part = part_x;
            ab.band_lo = k_lo;
            ab.band_hi = k_hi;
            const double *rec = nullptr;
            rc = check_hip(launch_dirty_map_mfma(ab, C, w, gamma, tau, X, ws + beam_bytes, stream, &rec, seeds),
                           "dirty-map (matrix cores) launch");
            if (rc) return rc;
            note_xform(kXFormDevice, rec, stream);
            rc = check_hip(launch_band_partial_finish(part_x, xm_band_rows(a), npix, Xbb, stream), "band finish");
        } else {
            rc = check_hip(launch_dirty_map<float>(a, C, w, gamma, tau, X, stream), "dirty-map kernel launch");
            if (rc) return rc;
            note_xform(SGWB_XFORM_VALU);
            rc = check_hip(launch_band<float>(X, nullptr, nullptr, nf, npix, k_lo, k_hi, Xbb, nullptr, nullptr, 0,
                                              stream),
                           "band kernel launch");
        }
        if (rc) return rc;
    }
    if (Gbb) {
        if (Gam) {
            rc = check_hip(launch_beam_bf16x3(a, w, gamma, Gam, workspace, default_beam_shape(), stream),
                           "beam kernel launch");
            if (rc) return rc;
        }
        // Gbb from its definition, the band sum moved into the weights (no pass over Gam)
        rc = check_hip(launch_band_gamma(w, ldc, nt, H, k_lo, k_hi, gamma, npix, vband, Gbb, stream),
                       "band weights launch");
        if (rc) return rc;
    }
    return SGWB_OK;
}

// Broadband maps alone: the route (strips or delay tables) from the host
// arguments, and the table grid when that route is taken.
struct BbRoute {
    bool table = false;
    BbGrid grid;
    double seconds = 0.0;  // the cost estimate of the route taken
};

static int bb_route(int32_t nt, int32_t nf, int32_t npix, uint32_t flags, const sgwb_fgrid *fg, int32_t k_lo,
                    int32_t k_hi, double tau_bound, BbRoute *r)
{
    if ((flags & SGWB_BB_TABLE) && (flags & SGWB_BB_STRIPS))
        return set_error(SGWB_EINVAL, "broadband_maps: both routes forced");
    if (!(tau_bound >= 0.0) || !isfinite(tau_bound))
        return set_error(SGWB_EINVAL, "broadband_maps: tau_bound %g is not a finite bound >= 0", tau_bound);
    if (!(0 <= k_lo && k_lo < k_hi && k_hi <= nf))
        return set_error(SGWB_EINVAL, "broadband_maps: band [%d, %d) not a non-empty part of [0, %d)", k_lo, k_hi, nf);
    const double earth = 2.0 * kEarthRadius / kLightSpeed;
    const double bound = tau_bound > 0.0 ? tau_bound : earth;
    const int32_t nb = k_hi - k_lo;
    const bool have_grid = bb_grid(nb, fg->df_hz, bound, &r->grid);
    MapArgs a;  // what the matrix-core eligibility reads (k0 = 63: the most strips a call can span)
    a.k0 = 63;
    a.nt = nt;
    a.nf = nf;
    a.npix = npix;
    a.df = fg->df_hz;
    a.nside = (flags & SGWB_MAPS_ANTIPODAL) ? nside_of_npix(npix) : 0;
    // the strips route: the matrix-core dirty map over the call's columns
    const bool strips_ok = a.nside > 0 && !(flags & SGWB_MAPS_VALU_X) && x_kernel_choice() != kXKernelValu &&
                           xm_eligible(a) && bound <= earth;
    // Cost estimate (s), from timings of both routes on one MI355X (full day,
    // nside 8..128, bands of 16..4096 bins): the strips route takes ~0.19 ms
    // of preparation, ~1.2e11 (segment, pixel) seed items/s and ~4.2e13 map
    // terms/s over its whole 64-bin strips; the table route ~0.03 ms of
    // launches, ~1.5e13 float64 FMAs/s for the tables (4 per segment, bin and
    // node; the rate rises to ~2e13 with more nodes) and ~3.3e11 items/s in
    // the map pass (twice that for antipodal seeds, read once per pixel pair).
    const double strip_cols = (double)(((int64_t)nf + 63) / 64 * 64);
    const double strips = 1.9e-4 + (double)nt * npix / 1.2e11 + (double)nt * strip_cols * npix / 4.2e13;
    const double table = have_grid ? 3e-5 + (double)nt * nb * r->grid.G * 4.0 / 1.5e13 +
                                         (double)nt * npix / (a.nside > 0 ? 6.6e11 : 3.3e11)
                                   : HUGE_VAL;
    if (flags & SGWB_BB_STRIPS) {
        if (!strips_ok)
            return set_error(SGWB_EINVAL, "broadband_maps: the strips route needs the matrix-core dirty map "
                                          "(antipodal seeds, df <= 0.0344 Hz, seeds within 2R/c)");
        r->table = false;
        r->seconds = strips;
        return SGWB_OK;
    }
    if (!have_grid && ((flags & SGWB_BB_TABLE) || !strips_ok))
        return set_error(SGWB_EINVAL, "broadband_maps: a delay table for %d bins of %g Hz up to %g s would "
                                      "exceed 2^21 + 3 nodes", nb, fg->df_hz, bound);
    if ((flags & SGWB_BB_TABLE) || !strips_ok) {
        r->table = true;
        r->seconds = table;
        return SGWB_OK;
    }
    // SGWB_BB_ROUTE=table|strips in the environment sets the route of calls
    // that force none (read at every call; a route that does not apply is ignored)
    if (const char *e = getenv("SGWB_BB_ROUTE")) {
        if (strcmp(e, "strips") == 0) {
            r->table = false;
            r->seconds = strips;
            return SGWB_OK;
        }
        if (strcmp(e, "table") == 0 && have_grid) {
            r->table = true;
            r->seconds = table;
            return SGWB_OK;
        }
    }
    r->table = have_grid && table < strips;
    r->seconds = r->table ? table : strips;
    return SGWB_OK;
}

double broadband_cost_seconds(int32_t nt, int32_t nf, int32_t npix, uint32_t flags, const sgwb_fgrid *fg,
                              int32_t k_lo, int32_t k_hi, double tau_bound)
{
    BbRoute r;
    if (!fg || bb_route(nt, nf, npix, flags, fg, k_lo, k_hi, tau_bound, &r)) return -1.0;
    return r.seconds;
}

int broadband_maps_seeded(const float *C, const float *w, int64_t ldc, int32_t nt, int32_t nf, const sgwb_fgrid *fg,
                          int64_t k0, const float *gamma, const double *tau, int32_t npix, uint32_t flags,
                          double tau_bound, const float *H, int32_t k_lo, int32_t k_hi, float *Xbb, float *Gbb,
                          void *workspace, size_t workspace_bytes, const void *seeds, hipStream_t stream)
{
    note_xform(SGWB_XFORM_NONE);
    if (!Xbb && !Gbb) return set_error(SGWB_EINVAL, "broadband_maps: nothing to compute");
    if (Gbb && !H) return set_error(SGWB_EINVAL, "broadband_maps: null H");
    if (!fg) return set_error(SGWB_EINVAL, "broadband_maps: null grid");
    if (flags & ~(SGWB_MAPS_ANTIPODAL | SGWB_MAPS_VALU_X | SGWB_BB_TABLE | SGWB_BB_STRIPS))
        return set_error(SGWB_EINVAL, "broadband_maps: unknown flag bits");
    const uint32_t mflags = flags & (SGWB_MAPS_ANTIPODAL | SGWB_MAPS_VALU_X);
    MapArgs a;
    int rc = check_maps_args<float>(C, w, ldc, nt, nf, fg, k0, gamma, tau, npix, mflags, &a);
    if (rc) return rc;
    BbRoute r;
    rc = bb_route(nt, nf, npix, flags, fg, k_lo, k_hi, tau_bound, &r);
    if (rc) return rc;
    if (!r.table)
        return make_maps_band_seeded(C, w, ldc, nt, nf, fg, k0, gamma, tau, npix, mflags, H, k_lo, k_hi, nullptr,
                                     nullptr, Xbb, Gbb, workspace, workspace_bytes, seeds, stream);
    if (!workspace || (uintptr_t)workspace % 256)
        return set_error(SGWB_EINVAL, "broadband_maps: workspace null or not 256-byte aligned");
    const int32_t nb = k_hi - k_lo;
    const size_t need = bb_workspace_bytes(nt, npix, nb, r.grid);
    if (workspace_bytes < need)
        return set_error(SGWB_ENOMEM, "broadband_maps: workspace of %zu bytes needed, %zu given", need,
                         workspace_bytes);
    rc = check_hip(launch_broadband_table_maps(C, w, ldc, nt, k_lo, k_hi, fg->f0_hz, fg->df_hz, k0, H, gamma, tau,
                                               npix, a.nside, r.grid, Xbb, Gbb, workspace, stream),
                   "broadband table launch");
    if (!rc && Xbb) note_xform(SGWB_XFORM_TABLE);
    return rc;
}

}  // namespace sgwb

extern "C" {

double sgwb_baseline_delay_bound(const sgwb_baseline *bl)
{
    if (!bl || !finite_det(bl->a) || !finite_det(bl->b)) return 0.0;
    double ra[3], rb[3], D[9];
    detector_frame(bl->a, ra, D);
    detector_frame(bl->b, rb, D);
    const double d = sqrt((ra[0] - rb[0]) * (ra[0] - rb[0]) + (ra[1] - rb[1]) * (ra[1] - rb[1]) +
                          (ra[2] - rb[2]) * (ra[2] - rb[2]));
    // the seeds' delays are this chord's projections, computed in float64:
    // a relative margin of 1e-9 covers their rounding (and a co-located pair)
    return d / kLightSpeed * (1.0 + 1e-9) + 1e-15;
}

size_t sgwb_broadband_maps_workspace_size(int32_t nt, int32_t nf, int32_t npix, uint32_t flags, const sgwb_fgrid *fg,
                                          int32_t k_lo, int32_t k_hi, double tau_bound_s)
{
    if (!fg || nt < 1 || nf < 1 || npix < 1) return 0;
    BbRoute r;
    if (bb_route(nt, nf, npix, flags, fg, k_lo, k_hi, tau_bound_s, &r)) return 0;
    if (!r.table) return sgwb_make_maps_band_workspace_size(nt, nf, npix, flags & (SGWB_MAPS_ANTIPODAL | SGWB_MAPS_VALU_X));
    return bb_workspace_bytes(nt, npix, k_hi - k_lo, r.grid);
}

int sgwb_broadband_maps(const float *C, const float *w, int64_t ldc, int32_t nt, int32_t nf, const sgwb_fgrid *fg,
                        int64_t k0, const float *gamma, const double *tau, int32_t npix, uint32_t flags,
                        double tau_bound_s, const float *H, int32_t k_lo, int32_t k_hi, float *Xbb, float *Gbb,
                        void *workspace, size_t workspace_bytes, hipStream_t stream)
{
    return broadband_maps_seeded(C, w, ldc, nt, nf, fg, k0, gamma, tau, npix, flags, tau_bound_s, H, k_lo, k_hi, Xbb,
                                 Gbb, workspace, workspace_bytes, nullptr, stream);
}

size_t sgwb_reduce_band_workspace_size(int32_t npix, int32_t k_lo, int32_t k_hi)
{
    if (npix < 1 || k_lo < 0 || k_hi <= k_lo) return 0;
    return band_workspace_bytes(npix, k_lo, k_hi);
}

int sgwb_reduce_band(const float *X, const float *Gam, const float *H, int32_t nf, int32_t npix, int32_t k_lo,
                     int32_t k_hi, float *Xbb, float *Gbb, void *workspace, size_t workspace_bytes,
                     hipStream_t stream)
{
    return reduce_band_impl<float>(X, Gam, H, nf, npix, k_lo, k_hi, Xbb, Gbb, workspace, workspace_bytes, stream);
}

int sgwb_reduce_band_f64(const double *X, const double *Gam, const double *H, int32_t nf, int32_t npix,
                         int32_t k_lo, int32_t k_hi, double *Xbb, double *Gbb, hipStream_t stream)
{
    return reduce_band_impl<double>(X, Gam, H, nf, npix, k_lo, k_hi, Xbb, Gbb, nullptr, 0, stream);
}

int sgwb_healpix_centres(int32_t nside, double *xyz, int32_t *anti, hipStream_t stream)
{
    if (!is_pow2_nside(nside)) return set_error(SGWB_EINVAL, "healpix_centres: bad nside %d", nside);
    if (!xyz && !anti) return set_error(SGWB_EINVAL, "healpix_centres: nothing to do");
    return check_hip(launch_centres(nside, xyz, anti, stream), "centres kernel launch");
}

}  // extern "C"

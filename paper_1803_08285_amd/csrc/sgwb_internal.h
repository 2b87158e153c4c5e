// Internal declarations shared by the HIP translation units of libsgwb.
// gfx950 only (wave64, MFMA bf16 32x32x16).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "sgwb.h"
#include "tune_cache.h"

namespace sgwb {

constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr double kTwoPi = 6.283185307179586476925286766559005768;
constexpr double kEarthRadius = 6.371e6;        // m, spherical Earth
constexpr double kLightSpeed = 299792458.0;     // m/s
constexpr double kSiderealDay = 86164.0905;     // s (23 h 56 min 4.09 s)

// ---------------------------------------------------------------------------
// HEALPix RING indexing (Gorski et al. 2005).  For a pixel p in the northern
// half (p < npix / 2: polar-cap rings and belt rings down to the equator) this
// returns its ring i (1-based, counted from the north pole), its position j
// (0-based) in the ring, the ring length and the ring's first pixel index.
// ---------------------------------------------------------------------------
struct RingPos {
    int64_t ring, j, len, start;
};

__host__ __device__ inline RingPos ring_of_north(int64_t p, int64_t nside)
{
    RingPos r;
    const int64_t ncap = 2 * nside * (nside - 1);
    if (p < ncap) {
        // ring i holds pixels [2 i (i - 1), 2 i (i + 1))
        int64_t i = (int64_t)((1.0 + sqrt(1.0 + 2.0 * (double)p)) * 0.5);
        while (2 * i * (i + 1) <= p) ++i;
        while (i > 1 && 2 * i * (i - 1) > p) --i;
        r.ring = i;
        r.start = 2 * i * (i - 1);
        r.len = 4 * i;
    } else {
        const int64_t q = p - ncap;
        r.ring = q / (4 * nside) + nside;
        r.start = ncap + (r.ring - nside) * 4 * nside;
        r.len = 4 * nside;
    }
    r.j = p - r.start;
    return r;
}

// Antipode of a northern-half pixel: the mirror ring 4 nside - i starts at
// npix - start - len and the antipodal azimuth is half a ring further on.
__host__ __device__ inline int64_t antipode_north(const RingPos &r, int64_t npix)
{
    return npix - r.start - r.len + (r.j + r.len / 2) % r.len;
}

// Unit vector of a northern-half pixel centre, float64.
__host__ __device__ inline void centre_north(const RingPos &r, int64_t nside, double *x, double *y,
                                             double *z)
{
    const double ns = (double)nside;
    double zz, one_minus_z, phi;
    if (r.ring < nside) {
        const double i = (double)r.ring;
        one_minus_z = i * i / (3.0 * ns * ns);
        zz = 1.0 - one_minus_z;
        phi = ((double)r.j + 0.5) * (kPi * 0.5 / i);
    } else {
        zz = (double)(2 * nside - r.ring) * (2.0 / (3.0 * ns));
        one_minus_z = 1.0 - zz;
        // belt rings with (ring - nside) even are offset by half a pixel
        const double off = ((r.ring - nside) % 2 == 0) ? 0.5 : 0.0;
        phi = ((double)r.j + off) * (kPi * 0.5 / ns);
    }
    const double st = sqrt(one_minus_z * (1.0 + zz));
    double s, c;
    sincos(phi, &s, &c);
    *x = st * c;
    *y = st * s;
    *z = zz;
}

inline bool is_pow2_nside(int64_t nside) { return nside >= 1 && nside <= 8192 && (nside & (nside - 1)) == 0; }

// nside of a HEALPix npix, or 0 if npix is not 12 nside^2 with nside a power of two.
inline int64_t nside_of_npix(int64_t npix)
{
    if (npix % 12) return 0;
    int64_t n2 = npix / 12, ns = 1;
    while (ns * ns < n2) ns <<= 1;
    return (ns * ns == n2 && is_pow2_nside(ns)) ? ns : 0;
}

// ---------------------------------------------------------------------------
// Error reporting (thread-local text; no printing).
// ---------------------------------------------------------------------------
int set_error(int code, const char *fmt, ...);
int check_hip(hipError_t e, const char *what);

// ---------------------------------------------------------------------------
// Launchers implemented in the .hip files.  All validate nothing: the C-ABI
// entry points in api.hip do the checks first.
// ---------------------------------------------------------------------------
struct GeomArgs {
    double DA[9], DB[9];  // Earth-fixed detector response tensors
    double dx[3];         // x_a - x_b, metres, Earth-fixed
    double t0, stride, half_dur;
    int32_t nt;
    int64_t nside, npix;
};
template <typename G>
hipError_t launch_geometry(const GeomArgs &a, G *gamma, double *tau, hipStream_t s);
hipError_t launch_centres(int64_t nside, double *xyz, int32_t *anti, hipStream_t s);

struct MapArgs {
    int64_t ldc, k0;
    int32_t nt, nf, npix;
    int64_t nside;      // > 0 when the antipodal pairing is used
    double f0, df;
    int32_t unit_c = 0;      // C is not read: C = 1 + 0i, so y = w (real data)
    int32_t accumulate = 0;  // add the dirty map to X instead of writing it
    // Broadband partial sums written by the matrix-core dirty map (nullptr: none):
    // band_part[strip][pixel] = sum of the strip's X rows with columns in [band_lo, band_hi).
    double *band_part = nullptr;
    int32_t band_lo = 0, band_hi = 0;
    // Bound on |tau| that valid seeds of this call meet (s): 2 R / c for the
    // delays of a baseline on the Earth, 4 R / c for differences of two.
    double tau_limit = 2.0 * kEarthRadius / kLightSpeed;
};
// gate (optional): the dirty-map form record of a matrix-core launch on the
// same seeds ([0] largest |tau|, [1] form code); with it the kernel computes
// only where that record selected the vector-unit form (its workgroups exit
// at once otherwise).
template <typename T>
hipError_t launch_dirty_map(const MapArgs &a, const T *C, const T *w, const T *gamma,
                            const double *tau, T *X, hipStream_t s, const double *gate = nullptr);

// Network sums and pixel contractions.
constexpr int kMaxNetworkMaps = 32;
struct MapList {
    const float *p[kMaxNetworkMaps];
    int32_t n;
};
hipError_t launch_network_sum(const MapList &l, int64_t n, float *out, hipStream_t s);
hipError_t launch_contract(const float *M, int32_t nf, int32_t npix, const int32_t *pix, int32_t nsel, float *out,
                           hipStream_t s);

// fused broadband sums: out[p] = sum_{r < nrows} part[r][p] (float64, fixed order, rounded once)
hipError_t launch_band_partial_finish(const double *part, int64_t nrows, int32_t npix, float *out, hipStream_t s);
int64_t xm_band_rows(const MapArgs &a);    // rows of the dirty map's partial-sum array
// broadband Fisher diagonal from its definition with the band sum moved into
// the weights: Gbb[p] = sum_t v[t] gamma(t,p)^2, v[t] = sum_{c in [klo,khi)} H[c] w[t][c]
// (float64, fixed order, rounded once); scratch: band_gamma_scratch_bytes() of device memory
size_t band_gamma_scratch_bytes(int32_t nt, int32_t npix);
hipError_t launch_band_gamma(const float *w, int64_t ldw, int32_t nt, const float *H, int32_t klo, int32_t khi,
                             const float *gamma, int32_t npix, double *scratch, float *Gbb, hipStream_t s);

// full Fisher matrix of a band for separable weights, and its CG clean map
size_t fisher_full_workspace_bytes(double f_max, int32_t nbins, int32_t nt, int32_t npix);
bool fisher_full_band_ok(double f_max);
// nside > 0: antipodal seeds (only the northern rows and their antipodes are computed)
hipError_t launch_fisher_full(const float *a, const float *b, int32_t rank, const float *H, int32_t nf, int32_t clo,
                              int32_t chi, double f0, double df, int64_t k0, const float *gamma, const double *tau,
                              int32_t nt, int32_t npix, int64_t nside, float *G, void *work, hipStream_t s);
size_t cg_workspace_bytes(int32_t n);
hipError_t launch_clean_map_cg(const float *G, const float *X, int32_t n, int32_t niter, float *P, void *work,
                               hipStream_t s);

// Folding of several sidereal days into one (float32 in and out, float64 sums).
hipError_t launch_fold(const float *C, const float *sv, const uint8_t *present, int64_t ldc, int32_t ndays, int32_t nt,
                       int32_t nf, double W, float *v, float *u, float *w, float *x, hipStream_t s);

// Neighbour terms of the overlap-corrected Fisher diagonal, added into Gam.
size_t pair_workspace_bytes(int32_t nt, int32_t nf, int32_t npix);
hipError_t launch_fisher_neighbours(const MapArgs &a, const float *u, const float *wn, const float *gamma,
                                    const double *tau, float *Gam, void *pair_ws, void *xm_ws, bool use_xm,
                                    hipStream_t s, const double **form_rec = nullptr);

// Matrix-core dirty map (float32, antipodal seeds, df <= 0.0344 Hz).
// Jacobi-Anger forms by the largest |eta| = 2 pi 31.5 df max|tau| of the seeds:
// four terms up to kXmEtaFour, five with m = 2 unsplit up to kXmEtaM2, five
// with m = 2 split up to kXmEtaMax (truncation below 1e-6 there).
constexpr double kXmEtaFour = 0.07;
constexpr double kXmEtaM2 = 0.17;
constexpr double kXmEtaMax = 0.29;
// Form record written by the prep on the device and read by the main kernel
// (and by sgwb_last_x_form): SGWB_XFORM_* codes, or kXFormRejected when the
// seeds fail the antipodal spot check or exceed the call's delay bound (the
// map is then written as NaN).
constexpr int kXFormRejected = -1;
// Spot check of the exact antipodal symmetry of seeds (first, middle and last
// segment, every northern pixel): flags[kSymParts] of 0.0 (pass) or 1.0, one per
// workgroup, no atomics.
constexpr int kSymParts = 64;
hipError_t launch_antipodal_check(const float *gamma, const double *tau, int32_t nt, int64_t npix, int64_t nside,
                                  double *flags, hipStream_t s);
bool xm_eligible(const MapArgs &a);
size_t xm_workspace_bytes(int64_t k0, int32_t nt, int32_t nf, int32_t npix);
// form_rec (optional out): device address of the call's form record
hipError_t launch_dirty_map_mfma(const MapArgs &a, const float *C, const float *w, const float *gamma,
                                 const double *tau, float *X, void *work, hipStream_t s,
                                 const double **form_rec = nullptr, const void *seeds = nullptr);
// The seed-side products of the matrix-core dirty map (form record and Bessel
// amplitudes) depend on gamma, tau and df alone: a caller that keeps seeds
// resident computes them once into a buffer of xm_seed_bytes() and passes it
// as `seeds` above, which then skips their preparation.
size_t xm_seed_bytes(int32_t nt, int32_t npix);
hipError_t launch_xm_seed_products(const MapArgs &a, const float *gamma, const double *tau, void *seeds,
                                   hipStream_t s);
// sgwb_make_maps_band with the seed-side products of the matrix-core dirty map
// taken from `seeds` (nullptr: prepared in the workspace, as the C-ABI call
// does); seed_products fills such a buffer for resident seeds (*made false
// where no matrix-core form applies, and the buffer is then not used).
int make_maps_band_seeded(const float *C, const float *w, int64_t ldc, int32_t nt, int32_t nf, const sgwb_fgrid *fg,
                          int64_t k0, const float *gamma, const double *tau, int32_t npix, uint32_t flags,
                          const float *H, int32_t k_lo, int32_t k_hi, float *X, float *Gam, float *Xbb, float *Gbb,
                          void *workspace, size_t workspace_bytes, const void *seeds, hipStream_t stream);
int seed_products(const float *C, const float *w, int64_t ldc, int32_t nt, int32_t nf, const sgwb_fgrid *fg,
                  int64_t k0, const float *gamma, const double *tau, int32_t npix, void *seeds, hipStream_t stream,
                  bool *made);
struct XmArgs {
    MapArgs a;
    int64_t strip_first, nstrips, nchunks;
    double eta_scale;  // 2 pi 31.5 df
};
// One job of the multi-job matrix-core dirty map: operands prepared per job,
// one launch over the (strip, pixel block) tiles of all jobs.
struct XmJob {
    XmArgs x;
    const uint4 *A;  // data-side fragments (job workspace)
    const int *e;    // per-bin scale exponents (job workspace)
    double *tmax;    // form record: [0] largest |tau| of the job's seeds, [1] form code (job workspace, prep)
    float4 *amp;     // per (segment, pixel pair) Bessel amplitudes a_0..a_3 (job workspace, prep)
    float *amp4;     // and a_4
    const float *C, *w, *gamma;
    const double *tau;
    float *X;
    int64_t npblocks;
    int64_t tile_begin;
};
void fill_xmjob(XmJob *j, const MapArgs &a, const float *C, const float *w, const float *gamma, const double *tau,
                float *X, void *work);
int64_t xmjob_tiles(const XmJob &j);
hipError_t launch_xm_prep(const XmJob &j, hipStream_t s);
hipError_t launch_xm_batched(const XmJob *jobs_dev, int32_t njobs, int64_t grid, hipStream_t s);
hipError_t launch_xm_main(const XmJob &j, hipStream_t s);  // one job's tiles (after its prep)
int64_t xm_batched_grid(const XmJob *jobs, int32_t njobs);  // host job copies

// One job of the persistent multi-job dirty-map kernel (float32 path).
struct XJob {
    MapArgs a;
    const float *C, *w, *gamma;
    const double *tau;
    float *X;
    int64_t strip_first, nstrips, ncoltiles;
    int64_t tile_begin;  // first global tile index of this job
    int32_t strip_major; // 1: column tiles fastest within a strip
};
void fill_xjob(XJob *j, const MapArgs &a, const float *C, const float *w, const float *gamma, const double *tau,
               float *X, bool strip_major);
inline int64_t xjob_tiles(const XJob &j) { return j.nstrips * j.ncoltiles; }
hipError_t launch_dirty_map_batched(const XJob *jobs_dev, int32_t njobs, int64_t ntiles, int64_t grid, bool pair,
                                    hipStream_t s);

size_t beam_workspace_bytes(int32_t nt, int32_t nf, int32_t ncol);

// Split-bf16 beam GEMM.  Operand fragments: 32-wide blocks x 16-deep K-steps.
constexpr int kBlk = 32;  // rows/columns per MFMA block
constexpr int kKs = 16;   // segments per MFMA K-step
struct FragDims {
    int64_t nblk;  // 32-wide blocks
    int64_t nks;   // 16-deep K steps
};
__host__ __device__ inline FragDims frag_dims(int64_t n, int64_t nt)
{
    return FragDims{(n + kBlk - 1) / kBlk, (nt + kKs - 1) / kKs};
}
// wave-tile shapes of the beam GEMM (blocks of 32 x 32 outputs per wave):
// kBeamShape4x4, kBeamShape2x4 (tune_cache.h)
struct BJob {
    const uint4 *Wf, *Gf;  // fragment arrays in the job's workspace
    FragDims fm, fn;
    int32_t nf, npix;
    int64_t ncol, nside;   // nside > 0: antipodal pairs
    float *Gam;
    const float *w, *gamma;  // prep inputs
    int64_t ldw;
    int32_t nt;
    int64_t wg_begin;      // first workgroup of this job in a multi-job launch
};
void fill_bjob(BJob *jb, const MapArgs &a, const float *w, const float *gamma, float *Gam, void *work);
int64_t bjob_workgroups(const BJob &jb, int shape);
hipError_t launch_beam_prep(const BJob &jb, hipStream_t s);
hipError_t launch_beam_gemm(const BJob &jb, int shape, hipStream_t s);
hipError_t launch_beam_gemm_batched(const BJob *jobs_dev, int32_t njobs, int64_t nwg, int64_t grid, int shape,
                                    hipStream_t s);
hipError_t launch_beam_bf16x3(const MapArgs &a, const float *w, const float *gamma, float *Gam,
                              void *work, int shape, hipStream_t s);
hipError_t launch_beam_f64(const MapArgs &a, const double *w, const double *gamma, double *Gam,
                           hipStream_t s);

size_t band_workspace_bytes(int32_t npix, int32_t klo, int32_t khi);
template <typename T>
hipError_t launch_band(const T *X, const T *G, const T *H, int32_t nf, int32_t npix, int32_t klo,
                       int32_t khi, T *Xbb, T *Gbb, void *work, size_t work_bytes, hipStream_t s);

// ---------------------------------------------------------------------------
// Batched plans and their autotuner
// ---------------------------------------------------------------------------
// struct Tunables: tune_cache.h
bool tune_cache_load(const std::string &key, Tunables *t);
void tune_cache_store(const std::string &key, const Tunables &t);
std::string device_key();
int check_maps_args_f32(const float *C, const float *w, int64_t ldc, int32_t nt, int32_t nf, const sgwb_fgrid *fg,
                        int64_t k0, const float *gamma, const double *tau, int32_t npix, uint32_t flags,
                        MapArgs *a);

}  // namespace sgwb

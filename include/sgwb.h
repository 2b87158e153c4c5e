/*
 * sgwb.h - C ABI of the MI355X (gfx950) folded-data SGWB radiometer map-making
 * library (method of Ain, Suresh & Mitra, arXiv:1803.08285).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - All array pointers are DEVICE pointers unless marked (host).  The caller
 *    owns every buffer and keeps it alive until the work queued on `stream`
 *    has finished.  The library never frees caller memory.
 *  - Every call validates its arguments on the host before queuing anything
 *    and then returns at once; the GPU work runs asynchronously on `stream`
 *    (a hipStream_t; NULL = the default stream).  A device fault shows up at
 *    the next synchronisation of that stream.
 *  - Return value: SGWB_OK (0) or a negative SGWB_E* code; nothing is printed
 *    and no exception crosses the ABI.  sgwb_status_string() names a code and
 *    sgwb_last_error() gives the text of the last failure on this thread.
 *  - Layouts are row-major with the last index contiguous:
 *      seeds      gamma[nt][npix], tau[nt][npix]    (pixel-major rows)
 *      CSD        C[nt][ldc] complex (re, im interleaved), weights w[nt][ldc]
 *      maps       X[nf][npix], Gam[nf][npix]         (each row one HEALPix map)
 *  - Pixels are HEALPix RING pixels, npix = 12 nside^2, nside a power of two.
 *  - Results are bitwise reproducible: fixed summation order, no atomics.
 */
#ifndef SGWB_H
#define SGWB_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define SGWB_OK 0
#define SGWB_EINVAL (-1)       /* bad argument: null pointer, shape, nside, range  */
#define SGWB_ENOMEM (-2)       /* workspace too small / allocation failed          */
#define SGWB_EDEVICE (-3)      /* a HIP call failed (text in sgwb_last_error)       */
#define SGWB_EBUSY (-4)        /* server queue full: submit again later            */
#define SGWB_EUNSUPPORTED (-5) /* device is not gfx950, or option not available     */
#define SGWB_EAGAIN 1          /* server query not finished yet (not an error)     */

/* ---- geometry descriptions --------------------------------------------- */
/* An L-shaped detector with horizontal arms on a sphere of radius 6.371e6 m.
 * x-arm azimuth is measured counter-clockwise from local East; the y-arm is
 * at azimuth + 90 degrees.  Longitude is positive to the East.             */
typedef struct {
    double lat_deg, lon_deg, xarm_az_deg;
} sgwb_detector;

/* A baseline (Sec. II.A, Fig. 1): the delay uses x_a - x_b.                  */
typedef struct {
    sgwb_detector a, b;
} sgwb_baseline;

/* Folded sidereal day (Sec. II.B): segment k has mid time
 * t_k = t0_s + k stride_s + seg_dur_s / 2, in sidereal seconds after the
 * moment when the Earth-fixed and celestial frames coincide.                 */
typedef struct {
    int32_t nt;
    double t0_s, stride_s, seg_dur_s;
} sgwb_tgrid;

/* Absolute frequency grid f_k = f0_hz + k df_hz.  A call works on the nf
 * consecutive bins [k0, k0 + nf); the recurrence of the dirty map is
 * re-anchored at absolute bins k = 0 mod 64 (mod 32 in the float64 path), so
 * a sub-band gives bitwise the same rows as the full band.                    */
typedef struct {
    double f0_hz, df_hz;
} sgwb_fgrid;

/* ---- seeds: Sec. III.D (Fig. 3), "ORF seed matrices" ---------------------
 * gamma(t,p) = sum_{A=+,x} F^A_a(Omega_p, t) F^A_b(Omega_p, t)  (combined
 * antenna pattern at the pixel centre, no normalisation constant) and
 * tau(t,p) = Omega_p . (x_a(t) - x_b(t)) / c  in seconds, with the detector
 * tensors and separation rotated to sidereal time t_k in float64 on the GPU.
 * Output gamma[nt][npix] (float32 here, float64 in the _f64 variant) and
 * tau[nt][npix] float64.  The RING grid is antipodally symmetric and the
 * output is written exactly symmetric: gamma(t, a(p)) = gamma(t,p) and
 * tau(t, a(p)) = -tau(t,p) for the antipode a(p).
 * Errors: SGWB_EINVAL if a pointer is null, nt < 1, nside is not a power of
 * two in [1, 8192], or stride/duration are not finite.                      */
int sgwb_build_geometry(const sgwb_baseline *bl /*host*/, int32_t nside, const sgwb_tgrid *tg /*host*/,
                        float *gamma, double *tau, hipStream_t stream);
int sgwb_build_geometry_f64(const sgwb_baseline *bl /*host*/, int32_t nside,
                            const sgwb_tgrid *tg /*host*/, double *gamma, double *tau,
                            hipStream_t stream);

/* ---- narrowband maps: Eq. eq_dirtymap split per bin (Eq. eq:narrowband),
 *      and the per-bin Fisher diagonal (Eq. eq_fisher with p = p', Sec. III.A)
 *
 *   X(k,p)   = sum_t w(t,k) gamma(t,p) Re[ C(t,k) exp(2 pi i f_k tau(t,p)) ]
 *   Gam(k,p) = sum_t w(t,k) gamma(t,p)^2
 *
 * for the nf bins k0 .. k0 + nf - 1 of grid fg and every pixel p < npix.
 * w holds the folded inverse noise variance times the spectral shape
 * (the configs use w = H / P^2), so no constant prefactor is applied.
 * Inputs: C interleaved complex float32 [nt][ldc] (column c = bin k0 + c),
 * w float32 [nt][ldc], ldc >= nf; gamma float32 and tau float64 [nt][npix].
 * Outputs (may be NULL to skip): X, Gam float32 [nf][npix].
 * flags: SGWB_MAPS_ANTIPODAL promises that gamma/tau have the exact
 * antipodal symmetry that sgwb_build_geometry writes (npix = 12 nside^2) and
 * delays of a baseline on the Earth (|tau| <= 2 R / c); the kernels then
 * evaluate one phasor per antipodal pair and write both pixels.  Without the
 * flag any npix and any seeds are accepted.
 * X arithmetic, two forms with the same definition:
 *   matrix cores (used with SGWB_MAPS_ANTIPODAL, df <= 0.0344 Hz, i.e.
 *   2 pi 31.5 df 2R/c <= 0.29, and a workspace): per 64-bin strip, float64
 *   phase reduction at the strip centre and a Jacobi-Anger expansion of the
 *   phase across the strip (4 or 5 terms: the fewest the seeds' largest delay
 *   allows, measured on the device per call), contracted on float16 MFMA
 *   with hi + lo splits of the leading terms and float32 accumulation.  The
 *   same device pass spot-checks the promise of SGWB_MAPS_ANTIPODAL (exact
 *   symmetry on the first, middle and last segment, and the delay bound);
 *   seeds that fail it give X = NaN everywhere and sgwb_last_x_form()
 *   reports SGWB_EINVAL;
 *   vector units (without a workspace, without the flag, for larger df, with
 *   flag SGWB_MAPS_VALU_X, or with SGWB_X_KERNEL=valu in the environment):
 *   float64 phase reduction at anchor bins k = 0 mod 64 and a float32
 *   complex-rotation recurrence between anchors.
 * sgwb_last_x_form() names the form a call took.
 * Gam arithmetic: float32 inputs split into bfloat16 hi + lo, three MFMA
 * products (hi.hi + hi.lo + lo.hi), float32 accumulation.
 * Workspace: device memory of at least sgwb_make_maps_workspace_size() bytes,
 * 256-byte aligned, owned by the caller (NULL allowed when Gam is NULL; the
 * dirty map then uses the vector-unit form).
 * Errors: SGWB_EINVAL (null input, nt/nf/npix < 1, ldc < nf, k0 < 0, bad
 * grid, misaligned pointer), SGWB_ENOMEM (workspace given but smaller than
 * the form that applies needs; nothing falls back silently).               */
#define SGWB_MAPS_ANTIPODAL 1u
#define SGWB_MAPS_VALU_X 2u /* use the vector-unit dirty map even where the matrix-core form applies */
size_t sgwb_make_maps_workspace_size(int32_t nt, int32_t nf, int32_t npix, uint32_t flags);
int sgwb_make_maps(const float *C, const float *w, int64_t ldc, int32_t nt, int32_t nf,
                   const sgwb_fgrid *fg /*host*/, int64_t k0, const float *gamma, const double *tau,
                   int32_t npix, uint32_t flags, float *X, float *Gam, void *workspace,
                   size_t workspace_bytes, hipStream_t stream);

/* ---- which dirty-map form ran ------------------------------------------
 * The form of X that the last sgwb_make_maps, sgwb_make_maps_band or
 * sgwb_fisher_overlap call made on the calling thread took:
 *   SGWB_XFORM_NONE    the call computed no dirty map (or failed);
 *   SGWB_XFORM_VALU    vector-unit recurrence (chosen on the host, or by the
 *                      device when no matrix-core form meets the delays);
 *   SGWB_XFORM_MFMA4   matrix cores, four terms (|eta| <= 0.07);
 *   SGWB_XFORM_MFMA5   five terms, m = 2 unsplit (|eta| <= 0.17);
 *   SGWB_XFORM_MFMA5S  five terms, m = 2 split hi + lo (|eta| <= 0.29),
 *   SGWB_XFORM_TABLE   no narrowband map: sgwb_broadband_maps summed the band
 *                      first through per-segment delay tables,
 * with eta = 2 pi 31.5 df max|tau| of the call's seeds.  The matrix-core
 * choice is made on the device; for it this call synchronises the stream of
 * that call and reads the choice back from its workspace (16 bytes), so it
 * must come before that workspace is reused or freed.
 * Returns SGWB_OK, or SGWB_EINVAL if the seeds failed the antipodal spot check
 * of that call (its X is then NaN; *form = SGWB_XFORM_NONE), or SGWB_EDEVICE.  */
#define SGWB_XFORM_NONE 0
#define SGWB_XFORM_VALU 1
#define SGWB_XFORM_MFMA4 2
#define SGWB_XFORM_MFMA5 3
#define SGWB_XFORM_MFMA5S 4
#define SGWB_XFORM_TABLE 5
int sgwb_last_x_form(int32_t *form /*host*/);

/* ---- network sum: the sum over baselines I of Eq. eq:narrowband ------------
 * out[i] = sum_{m < nmaps} maps[m][i] for i < n: the narrowband (or broadband)
 * maps X or Gam of several baselines with one pixelisation and band, added
 * element-wise (float64 sums in map order, rounded once).
 * maps: host array of nmaps device pointers (1 <= nmaps <= 32); out may alias
 * none of them.  Errors: SGWB_EINVAL (null pointer, nmaps or n out of range).  */
int sgwb_network_sum(const float *const *maps /*host array of device pointers*/, int32_t nmaps, int64_t n,
                     float *out, hipStream_t stream);

/* ---- directed and isotropic contractions: Sec. V -------------------------
 * A directed search adds the values of the pixels that contain the source; the
 * isotropic search adds all pixels (HEALPix pixels have equal area: no
 * weights).  out[k] = sum_{j < nsel} M[k][pix[j]] for each of the nf rows of
 * M [nf][npix] (narrowband maps, or nf = 1 for a broadband map); pix = NULL
 * sums all npix pixels.  pix is a device array of int32 RING indices that the
 * caller keeps in range [0, npix).  float64 sums in a fixed order, rounded once.
 * Errors: SGWB_EINVAL (null M or out, nf/npix < 1, nsel < 0, misaligned pix). */
int sgwb_contract_pixels(const float *M, int32_t nf, int32_t npix, const int32_t *pix, int32_t nsel, float *out,
                         hipStream_t stream);

/* ---- folding: Sec. II.B (Eqs. eq_foldx, eq_foldgamma and the folded series
 * of overlapping windows) ------------------------------------------------------
 * The geometry repeats every sidereal day, so the data of ndays days, nt
 * segments each, sum into one folded day.  Segment tau of day d is absolute
 * segment a = d nt + tau; a segment contributes only if it has data
 * (present[a] != 0); eps = W for a neighbour a - 1 or a + 1 that has data and
 * 0 otherwise (the first segment of a day neighbours the previous day's last).
 * With s = sigma^-2:
 *   v(tau,k) = sum_d s_a
 *   u(tau,k) = sum_d eps_{a-1} (s_a + s_{a-1}) / 2
 *   w(tau,k) = sum_d eps_{a+1} (s_a + s_{a+1}) / 2
 *   x(tau,k) = sum_d [ s_a C_a - eps_{a-1} (s_a + s_{a-1}) / 2 C_{a-1}
 *                             - eps_{a+1} (s_a + s_{a+1}) / 2 C_{a+1} ]
 * W = 3/70 for 50%-overlapping Hann windows.
 * Inputs: C interleaved complex float32 [ndays][nt][ldc], sinv float32
 * [ndays][nt][ldc] (columns = bins), present uint8 [ndays][nt] (device).
 * Outputs: v, u, w float32 [nt][nf] and x interleaved complex float32 [nt][nf];
 * sums in float64, rounded once.  x and v feed sgwb_make_maps as C and w
 * (x with unit weights); v, u, w feed sgwb_fisher_overlap.
 * Errors: SGWB_EINVAL (null pointer, ndays/nt/nf < 1, ldc < nf, W not finite or
 * negative, misaligned pointer).                                              */
int sgwb_fold(const float *C, const float *sinv, const uint8_t *present, int64_t ldc, int32_t ndays, int32_t nt,
              int32_t nf, double W, float *v, float *u, float *w, float *x, hipStream_t stream);

/* ---- overlap-corrected Fisher diagonal: Sec. II.B, Eq. fwGamma with p = p' -
 * With 50%-overlapping windows the noise of neighbouring segments is
 * correlated and the folded data carry three real series v, u, w; the
 * per-bin Fisher diagonal is then
 *   Gam(k,p) = Re sum_t conj(K_t) [ K_t v(t,k) - K_{t-1} u(t,k) - K_{t+1} w(t,k) ],
 *   K_t = gamma(t,p) exp(+2 pi i f_k tau(t,p)),
 * i.e. sum_t v gamma_t^2 minus, for every pair of consecutive segments,
 * (u(t+1,k) + w(t,k)) gamma_t gamma_{t+1} cos 2 pi f_k (tau_{t+1} - tau_t).
 * The folded day is periodic (the geometry repeats every sidereal day):
 * segment nt - 1 is followed by segment 0, whose u row carries the pairs that
 * cross a day boundary (zero for data of a single day).
 * Inputs: v, u, w float32 [nt][ldc] (column c = bin k0 + c, ldc >= nf);
 * gamma float32, tau float64 [nt][npix] as for sgwb_make_maps, same flags.
 * Output: Gam float32 [nf][npix] (overwritten).
 * Arithmetic: the v term on the matrix cores as the split-bf16 beam GEMM; the
 * neighbour terms as a dirty map over the nt - 1 segment pairs (same forms and
 * tolerances as X in sgwb_make_maps, on the matrix cores where they apply).
 * Workspace: at least sgwb_fisher_overlap_workspace_size() bytes, 256-byte
 * aligned, owned by the caller.
 * Errors: SGWB_EINVAL (null pointer, nt/nf/npix < 1, ldc < nf, k0 < 0, bad grid
 * or flags, misaligned pointer), SGWB_ENOMEM (workspace too small).          */
size_t sgwb_fisher_overlap_workspace_size(int32_t nt, int32_t nf, int32_t npix, uint32_t flags);
int sgwb_fisher_overlap(const float *v, const float *u, const float *w, int64_t ldc, int32_t nt, int32_t nf,
                        const sgwb_fgrid *fg /*host*/, int64_t k0, const float *gamma, const double *tau,
                        int32_t npix, uint32_t flags, float *Gam, void *workspace, size_t workspace_bytes,
                        hipStream_t stream);

/* ---- full Fisher matrix of a band: Eq. eq_fisher, broadband H weighting of
 * Sec. V ----------------------------------------------------------------------
 * For weights given as a sum of rank separable terms,
 *   w(t,c) = sum_{r < rank} a_r(t) b_r(c)
 * (rank 1: a per-segment noise factor times a per-bin spectral factor, which is
 * how w = H / P^2 factors when the noise spectrum keeps its shape across
 * segments; weights of any other form, or of rank 2 and up, are better served
 * by sgwb_fisher_full_general below):
 *   G(p,q) = sum_{c in [clo,chi)} H(c) sum_t w(t,c) gamma(t,p) gamma(t,q)
 *              cos 2 pi f_{k0+c} (tau(t,p) - tau(t,q))
 *          = sum_r sum_t a_r(t) gamma(t,p) gamma(t,q) Wd_r(tau(t,p) - tau(t,q)),
 *   Wd_r(D) = sum_{c in [clo,chi)} H(c) b_r(c) cos 2 pi f_{k0+c} D.
 * Its diagonal is the band sum of the per-bin diagonal Gam (sgwb_reduce_band's
 * Gbb for the same w).
 * Inputs (device): a float32 [rank][nt]; b float32 [rank][nf], H float32 [nf]
 * (column c = bin k0 + c); gamma float32, tau float64 [nt][npix] as for
 * sgwb_make_maps.  0 <= clo < chi <= nf, 1 <= rank <= 64.
 * flags: 0 (every pixel a row and a column, any seeds), or
 * SGWB_MAPS_ANTIPODAL: the seeds have the exact antipodal symmetry that
 * sgwb_build_geometry writes (npix = 12 nside^2), so G(a(p),a(q)) = G(p,q) and
 * G(p,a(q)) = G(q,a(p)) for the antipode a; only the upper triangles of the
 * two northern blocks are computed (half the work) and each value is written
 * to its four entries.  Same tolerance; equal to the flag-free matrix up to
 * float32 rounding of the weight products.  The promise is spot-checked on the
 * device (first, middle and last segment); seeds that fail give G = NaN.
 * Output: G float32 [npix][npix] row-major, symmetric (overwritten).
 * Arithmetic, per rank: Wd_r and its derivative tabulated in float64 on 64
 * points per period of the highest band frequency over 0 <= D <= 4 R_earth / c,
 * turned into the float32 cubic Hermite interpolant of each interval (relative
 * error < 2.4e-7 of sum |H b_r|); delays enter as 32-bit fixed-point table
 * coordinates (resolution 2^-17 of a table step below 3 kHz, 2^-14 at the
 * 24 kHz limit), so tau_p - tau_q is exact and G exactly symmetric; float32
 * accumulation over t, then over the ranks.  Delays are clamped to
 * |tau| <= 2 R_earth / c.
 * Workspace: at least sgwb_fisher_full_workspace_size() bytes (0 for
 * arguments out of range), 256-byte aligned, owned by the caller.
 * Errors: SGWB_EINVAL (null pointer, nt/nf/npix < 1, rank out of range, band
 * out of range or reaching above 24 kHz, bad grid, unknown flag bits or the
 * antipodal flag with a non-HEALPix npix, misaligned pointer, more than
 * 2^31 - 1 matrix tiles), SGWB_ENOMEM (workspace too small).                 */
size_t sgwb_fisher_full_workspace_size(const sgwb_fgrid *fg /*host*/, int64_t k0, int32_t chi, int32_t nt,
                                       int32_t npix);
int sgwb_fisher_full(const float *a, const float *b, int32_t rank, const float *H, int32_t nf,
                     const sgwb_fgrid *fg /*host*/, int64_t k0, int32_t clo, int32_t chi, const float *gamma,
                     const double *tau, int32_t nt, int32_t npix, uint32_t flags, float *G, void *workspace,
                     size_t workspace_bytes, hipStream_t stream);

/* ---- full Fisher matrix for general weights: Eq. eq_fisher ------------------
 * The same matrix as sgwb_fisher_full, for weights w(t,c) given whole (the
 * folded w = H / P^2 of every segment and bin, of any rank):
 *   G(p,q) = sum_{c in [clo,chi)} H(c) sum_t w(t,c) gamma(t,p) gamma(t,q)
 *              cos 2 pi f_{k0+c} (tau(t,p) - tau(t,q))
 *          = sum_t gamma(t,p) gamma(t,q) Wd_t(tau(t,p) - tau(t,q)),
 *   Wd_t(D) = sum_{c in [clo,chi)} H(c) w(t,c) cos 2 pi f_{k0+c} D.
 * Inputs (device): w float32 [nt][ldw] (ldw >= nf; column c = bin k0 + c, as
 * the weights of sgwb_make_maps), H float32 [nf]; gamma float32, tau float64
 * [nt][npix]; 0 <= clo < chi <= nf, 1 <= nt <= 65535.  flags: 0 or
 * SGWB_MAPS_ANTIPODAL, as for sgwb_fisher_full (same spot check; seeds that
 * fail give G = NaN).
 * Output: G float32 [npix][npix] row-major, symmetric (overwritten).
 * Arithmetic: one table Wd_t per segment on the grid of sgwb_fisher_full, its
 * values and derivatives summed over the band in float64 on the matrix cores:
 * over the bins (weights times generated cosines and sines) on grids coarser
 * than 1/8 Hz, else over Jacobi-Anger moments of 16- to 64-bin strips (eight
 * terms, truncation below 1.6e-9 of sum |H w|); then the same float32 cubic
 * interpolants, fixed-point delays
 * and float32 accumulation over t; same tolerance.  The tables stop at the
 * largest delay difference the seeds can have, 2 max|tau| (found on the
 * device; |x_A - x_B| / c for seeds of sgwb_build_geometry), not at the
 * Earth's 4 R_earth / c.  For bands up to 1.88 kHz the tables stream through
 * LDS while each workgroup keeps its matrix tiles' sums in registers over all
 * segments; above, the tables are read from global memory.
 * Workspace: at least sgwb_fisher_full_general_workspace_size() bytes (0 for
 * arguments out of range), 256-byte aligned, owned by the caller: the tables
 * and the partial sums of their band sums, sized for the Earth bound, and the
 * strip moments (about 0.86 MB per segment for the full 20-1726 Hz band at
 * 1/32 Hz), and the fixed-point delays (4 bytes per seed).
 * Errors: SGWB_EINVAL (null pointer, nt/nf/npix out of range, ldw < nf, band
 * out of range or reaching above 24 kHz, bad grid, unknown flag bits or the
 * antipodal flag with a non-HEALPix npix, misaligned pointer, more than
 * 2^31 - 1 matrix tiles), SGWB_ENOMEM (workspace too small).                 */
size_t sgwb_fisher_full_general_workspace_size(const sgwb_fgrid *fg /*host*/, int64_t k0, int32_t clo, int32_t chi,
                                               int32_t nt, int32_t npix, uint32_t flags);
int sgwb_fisher_full_general(const float *w, int64_t ldw, const float *H, int32_t nf,
                             const sgwb_fgrid *fg /*host*/, int64_t k0, int32_t clo, int32_t chi,
                             const float *gamma, const double *tau, int32_t nt, int32_t npix, uint32_t flags,
                             float *G, void *workspace, size_t workspace_bytes, hipStream_t stream);

/* ---- clean map: Eq. eq_ML_linear and its footnote ---------------------------
 * The maximum-likelihood map P solves G P = X; G is poorly conditioned, so the
 * clean map is the conjugate-gradient iterate after niter steps from P = 0
 * (niter = 0 gives P = 0; a step whose residual or curvature is exactly zero
 * leaves P unchanged).  G float32 [n][n] symmetric positive semi-definite, X
 * float32 [n] (device); P float32 [n] (overwritten).  Vectors, dot products
 * and the matrix-vector products run in float64 with fixed-order sums; the
 * step scalars stay on the device (no host synchronisation).
 * Workspace: at least sgwb_clean_map_workspace_size() bytes, 256-byte aligned.
 * Errors: SGWB_EINVAL (null pointer, n < 1, niter < 0, misaligned pointer),
 * SGWB_ENOMEM (workspace too small).                                          */
size_t sgwb_clean_map_workspace_size(int32_t n);
int sgwb_clean_map_cg(const float *G, const float *X, int32_t n, int32_t niter, float *P, void *workspace,
                      size_t workspace_bytes, hipStream_t stream);

/* float64 variant of the same definition (all inputs and outputs double; Gam
 * accumulated in float64 on the vector units; no workspace).                  */
int sgwb_make_maps_f64(const double *C, const double *w, int64_t ldc, int32_t nt, int32_t nf,
                       const sgwb_fgrid *fg /*host*/, int64_t k0, const double *gamma,
                       const double *tau, int32_t npix, uint32_t flags, double *X, double *Gam,
                       hipStream_t stream);

/* ---- broadband maps: Sec. V, spectrum-weighted sum of narrowband maps -----
 *   Xbb(p) = sum_{k_lo <= k < k_hi} X(k,p)
 *   Gbb(p) = sum_{k_lo <= k < k_hi} H(k) Gam(k,p)
 * (w = H / P^2 already carries one factor of H into X and Gam).  X, Gam are
 * [nf][npix]; H[nf] is indexed like the rows.  Sums run in float64 in a fixed
 * order and are rounded once.  Either of X/Xbb or Gam/Gbb may be NULL.
 * Workspace (optional, caller-owned device memory, 256-byte aligned, at least
 * sgwb_reduce_band_workspace_size() bytes): with it the rows are reduced in
 * parallel slabs (needs npix % 4 == 0 and 16-byte aligned maps), without it
 * (NULL) a single-pass kernel runs.  Results are reproducible for a given
 * choice; the two choices may differ in the last bit.
 * Errors: SGWB_EINVAL if 0 <= k_lo <= k_hi <= nf fails, a needed pointer
 * is null or the workspace is misaligned.                                    */
size_t sgwb_reduce_band_workspace_size(int32_t npix, int32_t k_lo, int32_t k_hi);
int sgwb_reduce_band(const float *X, const float *Gam, const float *H, int32_t nf, int32_t npix,
                     int32_t k_lo, int32_t k_hi, float *Xbb, float *Gbb, void *workspace,
                     size_t workspace_bytes, hipStream_t stream);
int sgwb_reduce_band_f64(const double *X, const double *Gam, const double *H, int32_t nf,
                         int32_t npix, int32_t k_lo, int32_t k_hi, double *Xbb, double *Gbb,
                         hipStream_t stream);

/* ---- narrowband and broadband maps in one call: Secs. III.E and V ----------
 * X, Gam as sgwb_make_maps (same flags, same bits) and the broadband maps over
 * columns [k_lo, k_hi) of the same call, without reading the narrowband maps
 * back:
 *   Xbb(p) = sum_k X(k,p): where the matrix-core dirty map runs it also writes
 *     the float64 sum of each absolute 64-bin strip and one small kernel adds
 *     the strips in order, rounding once (equal to sgwb_reduce_band's Xbb up to
 *     the order of the float64 sums); otherwise the single-pass band kernel;
 *   Gbb(p) = sum_k H(k) Gam(k,p) = sum_t v(t) gamma(t,p)^2, v(t) = sum_k H(k) w(t,k):
 *     the band sum moved into the weights, float64 throughout, rounded once (the
 *     exact band-summed diagonal; sgwb_reduce_band of the split-bf16 Gam meets it
 *     within that map's 1e-4).
 * X needs Xbb and Gam needs Gbb; either pair may be NULL, not both.  The
 * broadband maps may also come alone, without their narrowband map (X or Gam
 * NULL):
 *   Gbb alone runs only the weight-side sum above (no beam GEMM);
 *   Xbb alone runs the matrix-core dirty map without writing any narrowband
 *     row (only the strip sums), so it needs that form: SGWB_MAPS_ANTIPODAL,
 *     df <= 0.0344 Hz and no vector-unit request, else SGWB_EINVAL.
 * Either way the broadband maps are bitwise those of the call with the
 * narrowband maps.  H[nf] is needed with Gbb.
 * Workspace: at least sgwb_make_maps_band_workspace_size() bytes, 256-byte
 * aligned, owned by the caller.
 * Errors: as sgwb_make_maps; SGWB_EINVAL also for a narrowband map without
 * its broadband map, no output at all, Xbb alone where the matrix-core form
 * does not apply, a band outside [0, nf] or a null H.                        */
size_t sgwb_make_maps_band_workspace_size(int32_t nt, int32_t nf, int32_t npix, uint32_t flags);
int sgwb_make_maps_band(const float *C, const float *w, int64_t ldc, int32_t nt, int32_t nf,
                        const sgwb_fgrid *fg /*host*/, int64_t k0, const float *gamma, const double *tau,
                        int32_t npix, uint32_t flags, const float *H, int32_t k_lo, int32_t k_hi, float *X,
                        float *Gam, float *Xbb, float *Gbb, void *workspace, size_t workspace_bytes,
                        hipStream_t stream);

/* ---- broadband maps alone, the band's bins summed first: Sec. V ------------
 * Xbb and Gbb over columns [k_lo, k_hi) as sgwb_make_maps_band defines them,
 * with no narrowband map.  The call takes one of two routes:
 *  - strips: sgwb_make_maps_band with X = Gam = NULL (the matrix-core dirty map
 *    of all nf columns writes only its strip sums; needs SGWB_MAPS_ANTIPODAL,
 *    df <= 0.0344 Hz, seeds within 2R/c; bitwise that call's result);
 *  - table: Eq. eq_dirtymap summed over the band with the sums over bins and
 *    segments exchanged,
 *      Xbb(p) = sum_t gamma(t,p) Re[e^{2 pi i f_c tau} Y_t(tau)], tau = tau(t,p),
 *      Y_t(tau) = sum_{k_lo <= k < k_hi} w(t,k) C(t,k) e^{2 pi i (f_k - f_c) tau},
 *    f_c the band's centre.  Y_t is tabulated per segment on the delay grid
 *    tau_j = (j - m - 1) h (float64 Horner sums, stored as float32), h =
 *    0.03 / (2 pi F), F = (k_hi - k_lo - 1) df / 2, m = ceil(tau_bound / h),
 *    and read by 4-point Lagrange interpolation (error below 1.9e-8 of
 *    sum_k |w C| per segment); the carrier phase is reduced in float64.  The
 *    error against the definition stays below 1e-6 of
 *    S_bb(p) = sum_t sum_k |gamma w C|.  Any df, any seeds within tau_bound.
 *    With SGWB_MAPS_ANTIPODAL each pixel pair's seeds are read once (the
 *    antipode's value is the table read at -tau), the promise spot-checked
 *    as on the strips route: seeds that fail give NaN maps.
 *  Gbb (either route): the band sum moved into the weights, as in
 *    sgwb_make_maps_band.
 * The route is chosen on the host from the arguments alone: SGWB_BB_TABLE or
 * SGWB_BB_STRIPS in flags forces one; otherwise SGWB_BB_ROUTE=table|strips in
 * the environment, where that route applies; otherwise the table route runs
 * where the strips route does not apply or a cost estimate (the tables' nt nb G
 * products and nt npix interpolations against the strips' preparation and
 * nt nf npix map terms, rates measured on an MI355X) favours it.
 * sgwb_last_x_form reports the route (SGWB_XFORM_TABLE, or the matrix-core
 * form).
 * tau_bound_s: a bound on |tau(t,p)| that the seeds meet, e.g.
 * sgwb_baseline_delay_bound() of their baseline; 0 takes 2R/c (any baseline
 * on the Earth).  In the table route a seed beyond it (or not a number) makes
 * Xbb NaN at its pixel.
 * Workspace: sgwb_broadband_maps_workspace_size() bytes for the same
 * arguments (the route's own need), 256-byte aligned, owned by the caller.
 * Errors: as sgwb_make_maps_band for the strips route; SGWB_EINVAL also for
 * no output, a forced route that does not apply, both routes forced, a bad
 * tau_bound_s, or a band whose table would exceed 2^21 + 3 nodes.            */
#define SGWB_BB_TABLE 4u
#define SGWB_BB_STRIPS 8u
/* |x_a - x_b| / c (s) of the baseline's two sites on the Earth sphere of
 * radius R (Sec. II.A, Eq. eq_overlap_red: the delay Omega . Delta x / c is
 * at most this for every direction and time), with a 1e-9 relative margin
 * for the seeds' rounding; 0.0 for a null or invalid baseline.  Host only.   */
double sgwb_baseline_delay_bound(const sgwb_baseline *bl /*host*/);
size_t sgwb_broadband_maps_workspace_size(int32_t nt, int32_t nf, int32_t npix, uint32_t flags,
                                          const sgwb_fgrid *fg /*host*/, int32_t k_lo, int32_t k_hi,
                                          double tau_bound_s);
int sgwb_broadband_maps(const float *C, const float *w, int64_t ldc, int32_t nt, int32_t nf,
                        const sgwb_fgrid *fg /*host*/, int64_t k0, const float *gamma, const double *tau,
                        int32_t npix, uint32_t flags, double tau_bound_s, const float *H, int32_t k_lo,
                        int32_t k_hi, float *Xbb, float *Gbb, void *workspace, size_t workspace_bytes,
                        hipStream_t stream);

/* ---- make_maps_band without allocation ---------------------------------
 * For callers that cannot allocate device memory or hand over a workspace
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  Same arguments (minus the workspace), same computation and the
 * same bits as sgwb_make_maps_band; the workspace is a fixed array of
 * SGWB_NOALLOC_SCRATCH_BYTES in device memory that the library holds on each
 * GPU it runs on, from its first use there until the process ends.  Nothing is
 * allocated or freed.  A call whose sgwb_make_maps_band_workspace_size()
 * exceeds SGWB_NOALLOC_SCRATCH_BYTES fails with SGWB_ENOMEM before any device
 * work (at nt = 898: nside 16 up to 4096 bins, nside 32 up to ~3500 bins).
 * All calls on one GPU share that array, which keeps the last call's contents:
 * calls that overlap in time on one GPU (several streams or threads) race and
 * give undefined maps; the caller serialises them.  The first call on a device
 * looks up the array's device address (hipGetSymbolAddress).
 * Errors: as sgwb_make_maps_band; SGWB_ENOMEM as above.                      */
#define SGWB_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int sgwb_make_maps_band_noalloc(const float *C, const float *w, int64_t ldc, int32_t nt, int32_t nf,
                                const sgwb_fgrid *fg /*host*/, int64_t k0, const float *gamma,
                                const double *tau, int32_t npix, uint32_t flags, const float *H,
                                int32_t k_lo, int32_t k_hi, float *X, float *Gam, float *Xbb, float *Gbb,
                                hipStream_t stream);

/* ---- batched plans ------------------------------------------------------
 * Several map jobs (baselines, resolutions, uneven bands; Sec. III.C notes
 * that maps of several baselines are made the same way and added) run as one
 * persistent dirty-map launch over the concatenated tiles of all jobs and one
 * persistent beam launch, together with each job's operand preparation and
 * optional broadband reduction, captured once in a HIP graph.
 * A job has the arguments of sgwb_make_maps (float32 only) plus an optional
 * broadband reduction of rows [band_lo, band_hi) into Xbb/Gbb (H needed for
 * Gbb).  The plan records the pointers: the caller keeps every buffer alive
 * and unchanged in size until sgwb_plan_destroy, and may change their
 * contents between launches.
 * flags: SGWB_PLAN_AUTOTUNE times candidate schedules on the current device
 * (a few seconds at full-band sizes, then cached on disk under the key of
 * the device and the job shapes; SGWB_TUNE_CACHE names the cache file);
 * without it the default schedule is used.  SGWB_PLAN_NO_GRAPH launches the
 * kernels directly instead of replaying a graph.  The schedule never changes
 * a result: maps are bitwise equal to the single-call path (sgwb_make_maps_band:
 * the broadband maps are taken the same way, from the dirty map's per-strip
 * sums and the weight-side Gbb).
 * plan_create allocates the workspaces and job tables (device memory owned by
 * the plan) and synchronises the device; plan_launch allocates nothing and
 * queues the graph asynchronously on `stream`.
 * Errors: SGWB_EINVAL (a job fails the sgwb_make_maps checks, computes
 * nothing, or has a bad band), SGWB_ENOMEM, SGWB_EDEVICE.                    */
typedef struct {
    const float *C, *w;
    int64_t ldc;
    int32_t nt, nf;
    sgwb_fgrid fg;
    int64_t k0;
    const float *gamma;
    const double *tau;
    int32_t npix;
    uint32_t flags;   /* SGWB_MAPS_ANTIPODAL */
    float *X, *Gam;   /* [nf][npix]; either may be NULL */
    const float *H;   /* [nf], for Gbb */
    int32_t band_lo, band_hi;
    float *Xbb, *Gbb; /* [npix] or NULL */
} sgwb_job;
typedef struct sgwb_plan sgwb_plan;
#define SGWB_PLAN_AUTOTUNE 1u
#define SGWB_PLAN_NO_GRAPH 2u
int sgwb_plan_create(const sgwb_job *jobs /*host*/, int32_t njobs, uint32_t flags, sgwb_plan **out);
int sgwb_plan_launch(sgwb_plan *plan, hipStream_t stream);
void sgwb_plan_destroy(sgwb_plan *plan);
/* JSON text describing the plan's schedule and tuning times (host buffer).  */
int sgwb_plan_describe(const sgwb_plan *plan, char *buf, size_t len);

/* ---- query server with continuous batching ------------------------------
 * Serves broadband maps (Sec. V) of a baseline, resolution and contiguous
 * band (Eq. eq_dirtymap split per bin and summed over the band, Eq. eq_fisher
 * diagonal summed the same way; sgwb_make_maps_band with the broadband maps
 * alone, so no narrowband map is kept): folding makes the day's data small enough to stay
 * resident (Sec. I), so every query reuses it and the cached seeds.
 * Datasets: the folded CSD C [nt][ldc] (interleaved complex float32), weights
 * w [nt][ldc] and shape H [nf] of one baseline, covering absolute bins
 * [k0, k0 + nf) of grid fg; device memory owned by the caller, kept alive and
 * unchanged until sgwb_server_destroy.  The seeds of each (dataset, nside)
 * are built on first use and kept, together with the dirty map's seed-side
 * products (its form record and Bessel amplitudes, which depend on the seeds
 * and df alone, so every band of the dataset shares them).
 * A worker thread admits queries while one of `slots` HIP streams is free and
 * the query's footprint (the make_maps_band workspace, the two result
 * maps, and new seeds) fits in an HBM arena of
 * hbm_budget_bytes (0: 60 % of the free memory) reserved at creation; queries
 * that arrive while others run are admitted as slots and memory free up, and
 * their kernels overlap on the device.  Admission is cost-aware: a query's
 * cost is the time sgwb_broadband_maps' cost rule estimates for it, counted in
 * map terms at the strips route's rate (4.2e13 terms/s; for a strips-route
 * query about its segments x bins x pixels); one of at least 3e10
 * (SGWB_SERVER_HEAVY_TERMS in the environment overrides the threshold) fills
 * the GPU alone, so at most
 * one such heavy query runs at a time (SGWB_SERVER_MAX_HEAVY, 1 to 64,
 * overrides) and heavy queries start in arrival order; lighter queries start
 * in arrival order among themselves, run in the other slots beside it and
 * may pass a heavy query that waits for its turn; a
 * query waiting for memory holds back every query behind it.  A query larger
 * than the whole arena fails with SGWB_ENOMEM; nothing is ever allocated
 * after creation.  Results are bitwise the same alone and in any mix.
 * submit is non-blocking (SGWB_EBUSY when queue_capacity queries are
 * pending; SGWB_EINVAL for a bad query, before any device work).  poll
 * returns SGWB_EAGAIN until the query is done, then SGWB_OK with the query's
 * status, device pointers to its result (valid until release) and
 * timestamps in seconds of the server clock.  fetch copies a finished result
 * into caller memory on `stream`.  stats writes a JSON summary.
 * destroy waits for running queries and frees everything the server owns.  */
typedef struct {
    const float *C, *w;
    int64_t ldc;
    int32_t nf;
    sgwb_fgrid fg;
    int64_t k0;
    const float *H;
    sgwb_baseline bl;
    sgwb_tgrid tg;
} sgwb_dataset;
typedef struct {
    const sgwb_dataset *datasets; /* host array */
    int32_t ndatasets;
    size_t hbm_budget_bytes;
    int32_t slots;          /* 1..16 concurrent queries */
    int32_t queue_capacity; /* <= 0: unbounded */
} sgwb_server_cfg;
typedef struct {
    int32_t dataset, nside;
    int32_t k_lo, k_hi; /* rows [k_lo, k_hi) of the dataset */
} sgwb_query;
typedef struct {
    int32_t status, npix;
    const float *Xbb, *Gbb; /* device */
    double t_submit_s, t_start_s, t_done_s;
} sgwb_result;
typedef struct sgwb_server sgwb_server;
int sgwb_server_create(const sgwb_server_cfg *cfg /*host*/, sgwb_server **out);
int sgwb_server_submit(sgwb_server *s, const sgwb_query *q /*host*/, uint64_t *ticket);
int sgwb_server_poll(sgwb_server *s, uint64_t ticket, sgwb_result *out /*host*/);
int sgwb_server_fetch(sgwb_server *s, uint64_t ticket, float *Xbb, float *Gbb, hipStream_t stream);
int sgwb_server_release(sgwb_server *s, uint64_t ticket);
int sgwb_server_stats(sgwb_server *s, char *buf /*host*/, size_t len);
void sgwb_server_destroy(sgwb_server *s);

/* ---- HEALPix helper: RING pixel centres (Sec. III.B) as float64 unit
 * vectors xyz[npix][3] (device), and the antipode table anti[npix] (device,
 * int32).  Either output may be NULL.                                        */
int sgwb_healpix_centres(int32_t nside, double *xyz, int32_t *anti, hipStream_t stream);

/* ---- status ------------------------------------------------------------ */
const char *sgwb_status_string(int status);
const char *sgwb_last_error(void);
/* 1 if the current device is a gfx950 part, 0 if not, negative on error.    */
int sgwb_device_supported(void);

#ifdef __cplusplus
}
#endif
#endif /* SGWB_H */

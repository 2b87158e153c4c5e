// Narrowband dirty map X(k,p) = sum_t w(t,k) gamma(t,p) Re[C(t,k) e^{2 pi i f_k tau(t,p)}]
// (Eq. eq_dirtymap split per frequency bin as in Eq. eq:narrowband) on gfx950.
//
// Work decomposition
//   * A workgroup owns 256 pixel columns (one per lane) and one strip of S
//     consecutive frequency bins that starts at an absolute bin k = 0 mod S
//     (S = 64 in float32, 32 in float64).  Lanes of a wave read coalesced
//     pixel-major rows of gamma and tau.
//   * The weighted CSD y(t,k) = w(t,k) C(t,k) of the strip is staged in LDS,
//     XTC segments at a time; every lane reads the same y (LDS broadcast).
//   * Per (t, pixel) the phase is reduced once per strip in float64,
//     frac(f_anchor tau), and turned into the anchor phasor z = gamma e^{i phi};
//     the remaining S-1 bins advance z by the rotor 1 + eps = e^{i 2 pi df tau},
//     z <- z + z eps (four FMAs), so no transcendental is evaluated per term.
//   * Antipodal pairing (HEALPix RING seeds from the geometry kernel): the
//     antipode p' of p has gamma(t,p') = gamma(t,p) and tau(t,p') = -tau(t,p),
//     so its phasor is conj(z).  With a = sum y_re z_re and b = sum y_im z_im,
//     X(k,p) = a - b and X(k,p') = a + b: one rotation serves two pixels.
//   * Fixed summation order over t, no atomics: bitwise reproducible, and the
//     absolute anchor grid makes a sub-band bitwise equal to the full band.
#include "sgwb_internal.h"

namespace sgwb {

template <typename T>
struct Cplx;
template <>
struct Cplx<float> {
    using type = float2;
};
template <>
struct Cplx<double> {
    using type = double2;
};

template <typename T>
struct StripTraits;
template <>
struct StripTraits<float> {
    static constexpr int S = 64;    // bins per anchor strip
    static constexpr int XTC = 32;  // segments per LDS stage
};
template <>
struct StripTraits<double> {
    static constexpr int S = 32;
    static constexpr int XTC = 16;
};

// Rotor 1 + eps = e^{i d} for the per-bin phase step d = 2 pi df tau:
// eps_re = cos d - 1, eps_im = sin d, each with full relative precision.
__device__ inline void rotor(float d, float *er, float *ei)
{
    const float d2 = d * d;
    if (fabsf(d) <= 0.25f) {
        // Taylor series; truncation error below 2e-9 relative for |d| <= 0.25.
        *er = -0.5f * d2 * (1.0f - d2 * (1.0f / 12.0f) * (1.0f - d2 * (1.0f / 30.0f)));
        *ei = d * (1.0f - d2 * (1.0f / 6.0f) * (1.0f - d2 * (1.0f / 20.0f)));
    } else {
        float sh, ch, s, c;
        sincosf(0.5f * d, &sh, &ch);
        sincosf(d, &s, &c);
        *er = -2.0f * sh * sh;
        *ei = s;
    }
}
__device__ inline void rotor(double d, double *er, double *ei)
{
    double sh, ch, s, c;
    sincos(0.5 * d, &sh, &ch);
    sincos(d, &s, &c);
    *er = -2.0 * sh * sh;
    *ei = s;
}

// Anchor phasor gamma e^{2 pi i x} for x = f tau cycles, given as x4 = 4 x.
// float64 reduction to the nearest quarter turn q (x4 - q in [-1/2, 1/2]),
// Taylor series for sin and cos on |theta| <= pi/4 (truncation below 3e-8),
// then a rotation by i^q.
__device__ inline void anchor4(float g, double x4, float *zr, float *zi)
{
    const double q = rint(x4);
    const float th = (float)(x4 - q) * 1.57079632679489662f;
    const int m = (int)q & 3;
    const float t2 = th * th;
    const float s =
        th * fmaf(t2, fmaf(t2, fmaf(t2, fmaf(t2, 2.75573192e-6f, -1.98412698e-4f), 8.33333333e-3f),
                           -1.66666667e-1f),
                  1.0f);
    const float c =
        fmaf(t2, fmaf(t2, fmaf(t2, fmaf(t2, 2.48015873e-5f, -1.38888889e-3f), 4.16666667e-2f), -0.5f), 1.0f);
    float cr = (m & 1) ? -s : c;
    float ci = (m & 1) ? c : s;
    if (m & 2) {
        cr = -cr;
        ci = -ci;
    }
    *zr = g * cr;
    *zi = g * ci;
}
__device__ inline void anchor4(double g, double x4, double *zr, double *zi)
{
    double x = 0.25 * x4;
    x -= rint(x);
    double s, c;
    sincospi(2.0 * x, &s, &c);
    *zr = g * c;
    *zi = g * s;
}

// Global-memory accesses.  The multi-job kernel reads its pointers out of a
// job table, so the compiler cannot tell them from LDS pointers and would use
// flat instructions, which count against the LDS counter as well; through
// these every access is a plain global one.
template <typename T>
__device__ inline __attribute__((address_space(1))) T *gmem(T *p)
{
    return (__attribute__((address_space(1))) T *)p;
}
template <typename C2>
__device__ inline C2 gload_c(const C2 *p, int64_t i)
{
    typedef decltype(p->x) R;
    typedef R v2 __attribute__((ext_vector_type(2)));
    const v2 v = ((const __attribute__((address_space(1))) v2 *)p)[i];
    C2 r;
    r.x = v.x;
    r.y = v.y;
    return r;
}

// One tile: 256 pixel columns (coltile) x one S-bin strip (absolute index strip).
// Called by every thread of a 256-thread workgroup; ys is the workgroup's LDS stage.
template <typename T, bool PAIR>
__device__ inline void dirty_map_tile(const MapArgs &a, int64_t strip, int64_t coltile,
                                      const typename Cplx<T>::type *__restrict__ C, const T *__restrict__ w,
                                      const T *__restrict__ gamma, const double *__restrict__ tau,
                                      T *__restrict__ X,
                                      typename Cplx<T>::type (*ys)[StripTraits<T>::S])
{
    using C2 = typename Cplx<T>::type;
    constexpr int S = StripTraits<T>::S;
    constexpr int XTC = StripTraits<T>::XTC;

    const int64_t ncol = PAIR ? (int64_t)a.npix / 2 : (int64_t)a.npix;
    const int64_t col = coltile * 256 + threadIdx.x;
    const bool active = col < ncol;
    const int64_t kabs0 = strip * S;                          // absolute first bin of the strip
    const int64_t c0 = kabs0 - a.k0;                           // its column in C (may be < 0)
    const double fa4 = 4.0 * (a.f0 + (double)kabs0 * a.df);   // anchor frequency, quarter turns
    const double two_pi_df = kTwoPi * a.df;

    T acc_a[S], acc_b[PAIR ? S : 1];
#pragma unroll
    for (int j = 0; j < S; ++j) acc_a[j] = T(0);
#pragma unroll
    for (int j = 0; j < (PAIR ? S : 1); ++j) acc_b[j] = T(0);

    const int64_t pcol = active ? col : 0;
    for (int tc = 0; tc < a.nt; tc += XTC) {
        const int tn = min(XTC, a.nt - tc);
        __syncthreads();
        for (int e = threadIdx.x; e < XTC * S; e += 256) {
            const int tt = e / S, kk = e % S;
            const int64_t c = c0 + kk;
            C2 y;
            y.x = T(0);
            y.y = T(0);
            if (tt < tn && c >= 0 && c < a.nf) {
                const int64_t off = (int64_t)(tc + tt) * a.ldc + c;
                const T wv = gmem(w)[off];
                if (a.unit_c) {
                    y.x = wv;
                } else {
                    const C2 cv = gload_c(C, off);
                    y.x = wv * cv.x;
                    y.y = wv * cv.y;
                }
            }
            ys[tt][kk] = y;
        }
        __syncthreads();
        if (!active) continue;
        for (int tt = 0; tt < tn; ++tt) {
            const int64_t g_off = (int64_t)(tc + tt) * a.npix + pcol;
            const T g = gmem(gamma)[g_off];
            const double ta = gmem(tau)[g_off];
            T zr, zi, er, ei;
            anchor4(g, fa4 * ta, &zr, &zi);
            rotor((T)(two_pi_df * ta), &er, &ei);
#pragma unroll
            for (int j = 0; j < S; ++j) {
                const C2 y = ys[tt][j];
                if (PAIR) {
                    acc_a[j] = fma(y.x, zr, acc_a[j]);
                    acc_b[j] = fma(y.y, zi, acc_b[j]);
                } else {
                    acc_a[j] = fma(y.x, zr, acc_a[j]);
                    acc_a[j] = fma(-y.y, zi, acc_a[j]);
                }
                // z <- z (1 + eps)
                T nr = fma(zr, er, zr);
                nr = fma(-zi, ei, nr);
                T ni = fma(zi, er, zi);
                ni = fma(zr, ei, ni);
                zr = nr;
                zi = ni;
            }
        }
    }
    if (!active) return;
    int64_t colB = 0;
    if (PAIR) colB = antipode_north(ring_of_north(col, a.nside), a.npix);
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const int64_t c = c0 + j;
        if (c < 0 || c >= a.nf) continue;
        auto row = gmem(X + c * (int64_t)a.npix);
        if (PAIR) {
            const T xa = acc_a[j] - acc_b[j], xb = acc_a[j] + acc_b[j];
            row[col] = a.accumulate ? row[col] + xa : xa;
            row[colB] = a.accumulate ? row[colB] + xb : xb;
        } else {
            row[col] = a.accumulate ? row[col] + acc_a[j] : acc_a[j];
        }
    }
}

template <typename T, bool PAIR>
__global__ __launch_bounds__(256) void dirty_map_kernel(MapArgs a, int64_t strip0,
                                                         const typename Cplx<T>::type *__restrict__ C,
                                                         const T *__restrict__ w,
                                                         const T *__restrict__ gamma,
                                                         const double *__restrict__ tau,
                                                         T *__restrict__ X, const double *__restrict__ gate)
{
    __shared__ typename Cplx<T>::type ys[StripTraits<T>::XTC][StripTraits<T>::S];
    // gated launch: only where the matrix-core prep found no accurate form
    if (gate && (int)gmem(gate)[1] != SGWB_XFORM_VALU) return;
    dirty_map_tile<T, PAIR>(a, strip0 + (int64_t)blockIdx.y, blockIdx.x, C, w, gamma, tau, X, ys);
}

// Persistent multi-job form: workgroup b takes tiles b, b + grid, b + 2 grid, ...
// of the concatenated tile list of all jobs (each job: its column tiles fastest
// within a strip, or its strips fastest, as the plan chose).  A tile's result
// does not depend on which workgroup computes it or when.  PAIR is uniform
// over the job table (the plan launches one table per pairing).
template <bool PAIR>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void dirty_map_batched_kernel(
    const XJob *__restrict__ jobs, int32_t njobs, int64_t ntiles)
{
    __shared__ float2 ys[StripTraits<float>::XTC][StripTraits<float>::S];
    for (int64_t g = blockIdx.x; g < ntiles; g += gridDim.x) {
        int j = 0;
        while (j + 1 < njobs && g >= jobs[j + 1].tile_begin) ++j;
        // read the job's fields as scalars (uniform over the workgroup)
        const MapArgs a = jobs[j].a;
        const int64_t local = g - jobs[j].tile_begin;
        const int64_t ncoltiles = jobs[j].ncoltiles, nstrips = jobs[j].nstrips;
        const int64_t strip0 = jobs[j].strip_first;
        int64_t strip, coltile;
        if (jobs[j].strip_major) {
            strip = strip0 + local / ncoltiles;
            coltile = local % ncoltiles;
        } else {
            coltile = local / nstrips;
            strip = strip0 + local % nstrips;
        }
        const float2 *C = reinterpret_cast<const float2 *>(jobs[j].C);
        dirty_map_tile<float, PAIR>(a, strip, coltile, C, jobs[j].w, jobs[j].gamma, jobs[j].tau, jobs[j].X, ys);
    }
}

void fill_xjob(XJob *j, const MapArgs &a, const float *C, const float *w, const float *gamma, const double *tau,
               float *X, bool strip_major)
{
    constexpr int S = StripTraits<float>::S;
    j->a = a;
    j->C = C;
    j->w = w;
    j->gamma = gamma;
    j->tau = tau;
    j->X = X;
    j->strip_first = a.k0 / S;
    j->nstrips = (a.k0 + a.nf - 1) / S - j->strip_first + 1;
    const int64_t ncol = a.nside > 0 ? a.npix / 2 : a.npix;
    j->ncoltiles = (ncol + 255) / 256;
    j->strip_major = strip_major ? 1 : 0;
    j->tile_begin = 0;
}

hipError_t launch_dirty_map_batched(const XJob *jobs_dev, int32_t njobs, int64_t ntiles, int64_t grid, bool pair,
                                    hipStream_t s)
{
    if (pair)
        hipLaunchKernelGGL(dirty_map_batched_kernel<true>, dim3((unsigned)grid), dim3(256), 0, s, jobs_dev, njobs,
                           ntiles);
    else
        hipLaunchKernelGGL(dirty_map_batched_kernel<false>, dim3((unsigned)grid), dim3(256), 0, s, jobs_dev, njobs,
                           ntiles);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_dirty_map(const MapArgs &a, const T *C, const T *w, const T *gamma,
                            const double *tau, T *X, hipStream_t s, const double *gate)
{
    using C2 = typename Cplx<T>::type;
    constexpr int S = StripTraits<T>::S;
    const bool pair = a.nside > 0;
    const int64_t ncol = pair ? a.npix / 2 : a.npix;
    const int64_t strip_first = a.k0 / S;
    const int64_t strip_last = (a.k0 + a.nf - 1) / S;
    const int64_t nstrips = strip_last - strip_first + 1;
    const C2 *Cc = reinterpret_cast<const C2 *>(C);
    // grid.y is limited to 65535 strips per launch; larger bands are split.
    for (int64_t s0 = 0; s0 < nstrips; s0 += 65535) {
        const int64_t ns = nstrips - s0 < 65535 ? nstrips - s0 : 65535;
        dim3 grid((unsigned)((ncol + 255) / 256), (unsigned)ns);
        if (pair)
            hipLaunchKernelGGL((dirty_map_kernel<T, true>), grid, dim3(256), 0, s, a, strip_first + s0, Cc,
                               w, gamma, tau, X, gate);
        else
            hipLaunchKernelGGL((dirty_map_kernel<T, false>), grid, dim3(256), 0, s, a, strip_first + s0,
                               Cc, w, gamma, tau, X, gate);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
template hipError_t launch_dirty_map<float>(const MapArgs &, const float *, const float *,
                                            const float *, const double *, float *, hipStream_t, const double *);
template hipError_t launch_dirty_map<double>(const MapArgs &, const double *, const double *,
                                             const double *, const double *, double *, hipStream_t,
                                             const double *);

}  // namespace sgwb

// Broadband dirty map with the sum over the band's bins taken first (Sec. V:
// the broadband map is the sum of the narrowband maps over a band; Eq.
// eq_dirtymap written per bin).  Exchanging the sums over bins and segments,
//   Xbb(p) = sum_t gamma(t,p) Re[ e^{2 pi i f_c tau} Y_t(tau) ],  tau = tau(t,p),
//   Y_t(tau) = sum_{k in band} y(t,k) e^{2 pi i (f_k - f_c) tau},  y = w C,
// with f_c the band's centre.  Y_t is a trigonometric polynomial in tau whose
// frequencies lie within F = (nb - 1) df / 2 of zero, so it is smooth on the
// scale 1 / F: one table per segment on a uniform delay grid, read with
// 4-point Lagrange interpolation, replaces the per-bin phase of every
// (segment, bin, pixel) term by one interpolation per (segment, pixel).
//
// Kernels: the tables (Horner's rule in e^{2 pi i df tau_j}, float64, one
// (segment, node) a thread), and the map pass (one pixel a thread, one chunk
// of segments a workgroup row, float64 partial sums added in a fixed order by
// the band finish kernel).
#include <math.h>
#include <stdint.h>

#include "broadband.h"

namespace sgwb {

// The delay grid: nodes tau_j = (j - m - 1) h, j = 0 .. 2m + 2, so that every
// |tau| <= m h has the four nodes j - 1 .. j + 2 around it.
//
// Spacing.  The interpolation error of 4 nodes is at most
// max|Y''''| max_x |(x+1) x (x-1) (x-2)| h^4 / 4! <= (2 pi F h)^4 (9/16) / 24 sum_k |y(t,k)|;
// 2 pi F h = kBbPhaseStep = 0.03 keeps it below 1.9e-8 of sum_k |y(t,k)|.
constexpr double kBbPhaseStep = 0.03;
constexpr int32_t kBbMaxHalf = 1 << 20;  // m: at most 2^21 + 3 nodes per table
constexpr int kBbNodes = 64;  // table nodes per workgroup (one wave)
constexpr int kBbBatch = 2;  // segments whose loads the map pass issues together

bool bb_grid(int32_t nb, double df, double bound, BbGrid *g)
{
    if (!(bound > 0.0) || !isfinite(bound) || nb < 1) return false;
    const double F = 0.5 * (nb - 1) * df;
    // a single bin (F = 0) makes Y_t constant: any spacing is exact
    const double h = F > 0.0 ? kBbPhaseStep / (2.0 * kPi * F) : bound;
    const double m = ceil(bound / h);
    if (!(m <= kBbMaxHalf)) return false;
    g->m = (int32_t)(m < 1.0 ? 1.0 : m);
    g->G = 2 * g->m + 3;
    g->h = h;
    g->bound = bound;
    return true;
}

static size_t up256_(size_t n) { return (n + 255) / 256 * 256; }

// Workspace: T [nt][G] float2 | the map pass's partial sums [segment
// chunks][npix] | the Fisher band weights' scratch (v, then its partial sums)
// | the antipodal spot check's flags.
struct BbLayout {
    size_t t, part, gam, flags, total;
};
static BbLayout bb_layout(int32_t nt, int32_t npix, const BbGrid &g)
{
    const size_t ntb = (size_t)band_gamma_chunks();  // the map pass's segment chunks
    BbLayout L;
    L.t = 0;
    L.part = L.t + up256_((size_t)nt * g.G * sizeof(float2));
    L.gam = L.part + up256_(ntb * (size_t)npix * sizeof(double));
    L.flags = L.gam + up256_(band_gamma_scratch_bytes(nt, npix));
    L.total = L.flags + up256_(kSymParts * sizeof(double));
    return L;
}

size_t bb_workspace_bytes(int32_t nt, int32_t npix, int32_t nb, const BbGrid &g)
{
    (void)nb;
    return bb_layout(nt, npix, g).total;
}

// T[t][j] = sum_k y(t,k) e^{2 pi i (k - kc) df tau_j}, kc = (nb - 1) / 2,
// y(t,k) = w[t][klo + k] C[t][klo + k]: with omega = e^{2 pi i df tau_j},
// T = omega^{-kc} sum_k y(t,k) omega^k, the sum by Horner's rule from the top
// bin down (|omega| = 1, so rounding errors do not grow with the power), all
// in float64; omega and omega^{-kc} from phases reduced in float64.  One wave
// a workgroup (blockIdx.x the segment, blockIdx.y a block of 64 nodes), its y
// staged through LDS 64 bins at a time (every lane then reads the same bin).
__global__ __launch_bounds__(kBbNodes) void bb_table_kernel(const float *__restrict__ C, const float *__restrict__ w,
                                                            int64_t ldc, int32_t klo, int32_t nb, int32_t G,
                                                            int32_t m, double dfh, float2 *__restrict__ T)
{
    __shared__ double2 ys[kBbNodes];
    const int32_t t = blockIdx.x, j = blockIdx.y * kBbNodes + threadIdx.x;
    const double node = (double)(j - m - 1);  // tau_j / h
    double turns = dfh * node;
    turns -= rint(turns);
    double os, oc;
    sincospi(2.0 * turns, &os, &oc);
    const int64_t row = (int64_t)t * ldc + klo;
    double ar = 0.0, ai = 0.0;
    for (int32_t kb = (nb - 1) / kBbNodes * kBbNodes; kb >= 0; kb -= kBbNodes) {
        const int32_t k = kb + (int32_t)threadIdx.x;
        double2 yv = make_double2(0.0, 0.0);
        if (k < nb) {
            const double wv = (double)w[row + k];
            yv = make_double2(wv * (double)C[2 * (row + k)], wv * (double)C[2 * (row + k) + 1]);
        }
        __syncthreads();  // the previous block's reads are done
        ys[threadIdx.x] = yv;
        __syncthreads();
        // bins past the band were staged as zeros: above the top bin they keep
        // the sum at exactly zero, so every block runs the full count
#pragma unroll 16
        for (int i = kBbNodes - 1; i >= 0; --i) {
            const double2 y = ys[i];
            const double nr = fma(ar, oc, fma(-ai, os, y.x));
            const double ni = fma(ar, os, fma(ai, oc, y.y));
            ar = nr;
            ai = ni;
        }
    }
    double back = 0.5 * (nb - 1) * dfh * node;  // omega^{-kc}
    back -= rint(back);
    double bs, bc;
    sincospi(-2.0 * back, &bs, &bc);
    if (j < G) T[(int64_t)t * G + j] = make_float2((float)(ar * bc - ai * bs), (float)(ar * bs + ai * bc));
}

// part[blockIdx.y][p] = sum over this chunk's segments t of
// gamma(t,p) Re[e^{2 pi i f_c tau} Y_t(tau)], Y_t from its table by 4-point
// Lagrange interpolation; a seed with |tau| beyond the grid's bound (or not a
// number) makes its pixel's sum NaN.  With v (GB), gpart[blockIdx.y][p] =
// sum_t v[t] gamma(t,p)^2 as band_gamma_kernel sums it (same chunks, same
// order, same arithmetic), from the gamma values this pass reads anyway.
template <bool GB>
__global__ __launch_bounds__(256) void bb_map_kernel(const float *__restrict__ gamma, const double *__restrict__ tau,
                                                     int32_t nt, int32_t npix, const float2 *__restrict__ T,
                                                     int32_t G, int32_t m, double h, double bound, double fc,
                                                     int32_t per, double *__restrict__ part,
                                                     const double *__restrict__ v, double *__restrict__ gpart)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= npix) return;
    const int32_t t0 = blockIdx.y * per, t1 = min(nt, t0 + per);
    double gacc = 0.0;
    const double inv_h = 1.0 / h, origin = (double)(m + 1);
    const double jmax = (double)(2 * m);
    double acc = 0.0;
    bool bad = false;
    // segments kBbBatch at a time: their seed loads, then their table reads, are
    // issued together (segments past t1 repeat t1 - 1 with weight zero; no
    // branch, so that the compiler keeps the loads ahead of the arithmetic)
    for (int32_t tq = t0; tq < t1; tq += kBbBatch) {
        double ta[kBbBatch];
        float g[kBbBatch];
#pragma unroll
        for (int e = 0; e < kBbBatch; ++e) {
            const int64_t o = (int64_t)min(tq + e, t1 - 1) * npix + p;
            ta[e] = tau[o];
            g[e] = gamma[o];
        }
        float2 a[kBbBatch][4];
        float x[kBbBatch];
#pragma unroll
        for (int e = 0; e < kBbBatch; ++e) {
            const double u = fma(ta[e], inv_h, origin);
            const double jd = fmin(fmax(floor(u), 1.0), jmax);  // NaN and out-of-range delays stay inside the table
            x[e] = (float)(u - jd);
            const float2 *row = T + (int64_t)min(tq + e, t1 - 1) * G + ((int32_t)jd - 1);
#pragma unroll
            for (int i = 0; i < 4; ++i) a[e][i] = row[i];
        }
#pragma unroll
        for (int e = 0; e < kBbBatch; ++e) {
            const bool valid = tq + e < t1;
            bad |= valid && !(fabs(ta[e]) <= bound);
            // Lagrange weights of the nodes at -1, 0, 1, 2
            const float xe = x[e], xp = xe + 1.0f, xm = xe - 1.0f, xm2 = xe - 2.0f;
            const float l0 = -(1.0f / 6.0f) * xe * xm * xm2;
            const float l1 = 0.5f * xp * xm * xm2;
            const float l2 = -0.5f * xp * xe * xm2;
            const float l3 = (1.0f / 6.0f) * xp * xe * xm;
            const float yr = fmaf(l0, a[e][0].x, fmaf(l1, a[e][1].x, fmaf(l2, a[e][2].x, l3 * a[e][3].x)));
            const float yi = fmaf(l0, a[e][0].y, fmaf(l1, a[e][1].y, fmaf(l2, a[e][2].y, l3 * a[e][3].y)));
            // carrier e^{2 pi i f_c tau}: the phase reduced in float64
            const double turns = fc * ta[e];
            const float r = (float)(turns - rint(turns));
            float sn, cs;
            sincospif(2.0f * r, &sn, &cs);
            acc = fma(valid ? (double)g[e] : 0.0, (double)fmaf(cs, yr, -sn * yi), acc);
            if (GB) {
                const double gd = (double)g[e];
                const double ga = fma(v[min(tq + e, t1 - 1)], gd * gd, gacc);
                gacc = valid ? ga : gacc;
            }
        }
    }
    part[(int64_t)blockIdx.y * npix + p] = bad ? (double)__builtin_nanf("") : acc;
    if (GB) gpart[(int64_t)blockIdx.y * npix + p] = gacc;
}

// The same sums for a pixel p of the northern half and its antipode pB at
// once, from p's seeds alone: antipodal seeds have gamma(t,pB) = gamma(t,p)
// and tau(t,pB) = -tau(t,p), and the delay grid is symmetric about zero, so
// pB's value is the table read at -tau with the conjugate carrier.  The
// seeds' promise is spot-checked (flags, one per part of the check): a failed
// check makes both maps NaN everywhere.
template <bool GB>
__global__ __launch_bounds__(256) void bb_map_pair_kernel(const float *__restrict__ gamma,
                                                          const double *__restrict__ tau, int32_t nt, int32_t npix,
                                                          int64_t nside, const float2 *__restrict__ T, int32_t G,
                                                          int32_t m, double h, double bound, double fc, int32_t per,
                                                          const double *__restrict__ flags, double *__restrict__ part,
                                                          const double *__restrict__ v, double *__restrict__ gpart)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= npix / 2) return;
    const int64_t pB = antipode_north(ring_of_north(p, nside), npix);
    const int32_t t0 = blockIdx.y * per, t1 = min(nt, t0 + per);
    const double inv_h = 1.0 / h, origin = (double)(m + 1);
    const double jmax = (double)(2 * m);
    double accA = 0.0, accB = 0.0, gacc = 0.0;
    bool bad = false;
    for (int32_t tq = t0; tq < t1; tq += kBbBatch) {
        double ta[kBbBatch];
        float g[kBbBatch];
#pragma unroll
        for (int e = 0; e < kBbBatch; ++e) {
            const int64_t o = (int64_t)min(tq + e, t1 - 1) * npix + p;
            ta[e] = tau[o];
            g[e] = gamma[o];
        }
        float2 a[kBbBatch][2][4];
        float x[kBbBatch][2];
#pragma unroll
        for (int e = 0; e < kBbBatch; ++e)
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const double u = fma(side ? -ta[e] : ta[e], inv_h, origin);
                const double jd = fmin(fmax(floor(u), 1.0), jmax);  // NaN and out-of-range delays stay inside the table
                x[e][side] = (float)(u - jd);
                const float2 *row = T + (int64_t)min(tq + e, t1 - 1) * G + ((int32_t)jd - 1);
#pragma unroll
                for (int i = 0; i < 4; ++i) a[e][side][i] = row[i];
            }
#pragma unroll
        for (int e = 0; e < kBbBatch; ++e) {
            const bool valid = tq + e < t1;
            bad |= valid && !(fabs(ta[e]) <= bound);
            float yr[2], yi[2];
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                // Lagrange weights of the nodes at -1, 0, 1, 2
                const float xe = x[e][side], xp = xe + 1.0f, xm = xe - 1.0f, xm2 = xe - 2.0f;
                const float l0 = -(1.0f / 6.0f) * xe * xm * xm2;
                const float l1 = 0.5f * xp * xm * xm2;
                const float l2 = -0.5f * xp * xe * xm2;
                const float l3 = (1.0f / 6.0f) * xp * xe * xm;
                const float2 *aa = a[e][side];
                yr[side] = fmaf(l0, aa[0].x, fmaf(l1, aa[1].x, fmaf(l2, aa[2].x, l3 * aa[3].x)));
                yi[side] = fmaf(l0, aa[0].y, fmaf(l1, aa[1].y, fmaf(l2, aa[2].y, l3 * aa[3].y)));
            }
            // carrier e^{2 pi i f_c tau} for p, its conjugate for pB
            const double turns = fc * ta[e];
            const float r = (float)(turns - rint(turns));
            float sn, cs;
            sincospif(2.0f * r, &sn, &cs);
            const double wg = valid ? (double)g[e] : 0.0;
            accA = fma(wg, (double)fmaf(cs, yr[0], -sn * yi[0]), accA);
            accB = fma(wg, (double)fmaf(cs, yr[1], sn * yi[1]), accB);
            if (GB) {
                const double gd = (double)g[e];
                const double ga = fma(v[min(tq + e, t1 - 1)], gd * gd, gacc);
                gacc = valid ? ga : gacc;
            }
        }
    }
    bool broken = false;
    for (int i = 0; i < kSymParts; ++i) broken |= flags[i] != 0.0;
    const double nan = (double)__builtin_nanf("");
    double *row = part + (int64_t)blockIdx.y * npix;
    row[p] = bad || broken ? nan : accA;
    row[pB] = bad || broken ? nan : accB;
    if (GB) {
        double *grow = gpart + (int64_t)blockIdx.y * npix;
        grow[p] = broken ? nan : gacc;
        grow[pB] = broken ? nan : gacc;
    }
}

hipError_t launch_broadband_table_maps(const float *C, const float *w, int64_t ldc, int32_t nt, int32_t klo,
                                       int32_t khi, double f0, double df, int64_t k0, const float *H,
                                       const float *gamma, const double *tau, int32_t npix, int64_t nside,
                                       const BbGrid &g, float *Xbb, float *Gbb, void *work, hipStream_t s)
{
    const int32_t nb = khi - klo;
    const BbLayout L = bb_layout(nt, npix, g);
    char *ws = reinterpret_cast<char *>(work);
    double *v = reinterpret_cast<double *>(ws + L.gam), *gpart = v + nt;
    const int32_t nchunks = band_gamma_chunks(), per = (nt + nchunks - 1) / nchunks;
    if (!Xbb) {  // Gbb alone: the weight-side kernels by themselves
        return launch_band_gamma(w, ldc, nt, H, klo, khi, gamma, npix, v, Gbb, s);
    }
    float2 *T = reinterpret_cast<float2 *>(ws + L.t);
    double *part = reinterpret_cast<double *>(ws + L.part);
    hipLaunchKernelGGL(bb_table_kernel, dim3((unsigned)nt, (unsigned)((g.G + kBbNodes - 1) / kBbNodes)),
                       dim3(kBbNodes), 0, s, C, w, ldc, klo, nb, g.G, g.m, df * g.h, T);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (Gbb) {
        e = launch_band_weights(w, ldc, nt, H, klo, khi, v, s);
        if (e != hipSuccess) return e;
    }
    // the band's centre: absolute bin k0 + klo + (nb - 1) / 2
    const double fc = f0 + ((double)(k0 + klo) + 0.5 * (nb - 1)) * df;
    if (nside > 0) {  // antipodal seeds: each thread a pixel pair
        double *flags = reinterpret_cast<double *>(ws + L.flags);
        e = launch_antipodal_check(gamma, tau, nt, npix, nside, flags, s);
        if (e != hipSuccess) return e;
        const dim3 pgrid((unsigned)((npix / 2 + 255) / 256), (unsigned)nchunks);
        if (Gbb)
            hipLaunchKernelGGL(bb_map_pair_kernel<true>, pgrid, dim3(256), 0, s, gamma, tau, nt, npix, nside,
                               (const float2 *)T, g.G, g.m, g.h, g.bound, fc, per, (const double *)flags, part,
                               (const double *)v, gpart);
        else
            hipLaunchKernelGGL(bb_map_pair_kernel<false>, pgrid, dim3(256), 0, s, gamma, tau, nt, npix, nside,
                               (const float2 *)T, g.G, g.m, g.h, g.bound, fc, per, (const double *)flags, part,
                               (const double *)nullptr, (double *)nullptr);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = launch_band_partial_finish(part, nchunks, npix, Xbb, s);
        if (e != hipSuccess || !Gbb) return e;
        return launch_band_partial_finish(gpart, nchunks, npix, Gbb, s);
    }
    const dim3 grid((unsigned)((npix + 255) / 256), (unsigned)nchunks);
    if (Gbb)
        hipLaunchKernelGGL(bb_map_kernel<true>, grid, dim3(256), 0, s, gamma, tau, nt, npix, (const float2 *)T, g.G,
                           g.m, g.h, g.bound, fc, per, part, (const double *)v, gpart);
    else
        hipLaunchKernelGGL(bb_map_kernel<false>, grid, dim3(256), 0, s, gamma, tau, nt, npix, (const float2 *)T, g.G,
                           g.m, g.h, g.bound, fc, per, part, (const double *)nullptr, (double *)nullptr);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_band_partial_finish(part, nchunks, npix, Xbb, s);
    if (e != hipSuccess || !Gbb) return e;
    return launch_band_partial_finish(gpart, nchunks, npix, Gbb, s);
}


}  // namespace sgwb

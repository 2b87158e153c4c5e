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
// Kernels: the table's phase factors E(k,j) (float64, rounded once), the
// tables T = y E (a complex product [nt x nb] x [nb x G], float64 sums over
// ranges of bins, the ranges added in order), and
// the map pass (one pixel a thread, one block of segments a workgroup row,
// float64 partial sums added in a fixed order by the band finish kernel).
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
constexpr int kBbTileT = 64, kBbTileJ = 64, kBbTileK = 16;
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

// Bin ranges of the table product: enough workgroups to fill the chip (about
// 1024), each range a whole number of 16-bin steps.
static int32_t bb_splits(int32_t nt, int32_t nb, const BbGrid &g, int32_t *kper)
{
    const int64_t tiles = (int64_t)((g.G + kBbTileJ - 1) / kBbTileJ) * ((nt + kBbTileT - 1) / kBbTileT);
    const int32_t steps = (nb + kBbTileK - 1) / kBbTileK;
    int64_t want = (1024 + tiles - 1) / tiles;
    if (want > steps) want = steps;
    if (want < 1) want = 1;
    const int32_t per_steps = (int32_t)((steps + want - 1) / want);
    *kper = per_steps * kBbTileK;
    return (nb + *kper - 1) / *kper;
}

// Workspace: E [nb][G] float2 | T [nt][G] float2 | the map pass's partial sums
// [segment chunks][npix] | the table product's partial sums [ranges][nt][G]
// double2 | the Fisher band weights' scratch (v, then its partial sums).
struct BbLayout {
    size_t e, t, part, tpart, gam, total;
};
static BbLayout bb_layout(int32_t nt, int32_t npix, int32_t nb, const BbGrid &g)
{
    int32_t kper;
    const int32_t ns = bb_splits(nt, nb, g, &kper);
    const size_t ntb = (size_t)band_gamma_chunks();  // the map pass's segment chunks
    BbLayout L;
    L.e = 0;
    L.t = L.e + up256_((size_t)nb * g.G * sizeof(float2));
    L.part = L.t + up256_((size_t)nt * g.G * sizeof(float2));
    L.tpart = L.part + up256_(ntb * (size_t)npix * sizeof(double));
    L.gam = L.tpart + up256_((size_t)ns * nt * g.G * sizeof(double2));
    L.total = L.gam + up256_(band_gamma_scratch_bytes(nt, npix));
    return L;
}

size_t bb_workspace_bytes(int32_t nt, int32_t npix, int32_t nb, const BbGrid &g)
{
    return bb_layout(nt, npix, nb, g).total;
}

// E[k][j] = e^{2 pi i (k - kc) df tau_j}, kc = (nb - 1) / 2: the phase in
// turns, (k - kc) (df h) (j - m - 1), in float64, reduced to [-1/2, 1/2] and
// turned into the phasor in float64, rounded once to float32.
__global__ __launch_bounds__(256) void bb_phase_kernel(int32_t nb, int32_t G, int32_t m, double dfh,
                                                       float2 *__restrict__ E)
{
    const int64_t n = (int64_t)nb * G;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int32_t k = (int32_t)(i / G), j = (int32_t)(i - (int64_t)k * G);
        const double turns = ((double)k - 0.5 * (nb - 1)) * dfh * (double)(j - m - 1);
        const double r = turns - rint(turns);
        double s, c;
        sincospi(2.0 * r, &s, &c);
        E[i] = make_float2((float)c, (float)s);
    }
}

// T[t][j] = sum_k y(t,k) E[k][j], y(t,k) = w[t][klo + k] C[t][klo + k]: a
// 64 x 64 tile of (segment, node) per 256-thread workgroup, 16 bins at a time
// through LDS (y and E as float64 pairs; y staged 16 consecutive bins of a row
// per 16 lanes, E 64 consecutive nodes per wave); thread (ty, tx) holds
// segments ty + 16 a and nodes tx + 16 b, a, b < 4, summed in float64 in bin
// order.
__global__ __launch_bounds__(256) void bb_table_kernel(const float *__restrict__ C, const float *__restrict__ w,
                                                       int64_t ldc, int32_t nt, int32_t klo, int32_t nb, int32_t G,
                                                       int32_t kper, const float2 *__restrict__ E,
                                                       double2 *__restrict__ Tpart)
{
    __shared__ double2 ys[kBbTileT][kBbTileK + 1];  // padded: the four rows a wave reads fall in different banks
    __shared__ double2 es[kBbTileK][kBbTileJ];
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const int32_t j0 = blockIdx.x * kBbTileJ, t0 = blockIdx.y * kBbTileT;
    double2 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = make_double2(0.0, 0.0);
    const int32_t kb = blockIdx.z * kper, ke = min(nb, kb + kper);
    for (int32_t k0 = kb; k0 < ke; k0 += kBbTileK) {
        // stage: 64 x 16 of y and 16 x 64 of E, four of each per thread (zero past the ends)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = tid + 256 * r;
            {
                const int kk = e & 15, c = e >> 4;
                const int32_t k = k0 + kk, t = t0 + c;
                double2 yv = make_double2(0.0, 0.0);
                if (k < ke && t < nt) {
                    const int64_t o = (int64_t)t * ldc + klo + k;
                    const double wv = (double)w[o];
                    yv = make_double2(wv * (double)C[2 * o], wv * (double)C[2 * o + 1]);
                }
                ys[c][kk] = yv;
            }
            {
                const int kk = e >> 6, c = e & 63;
                const int32_t k = k0 + kk, j = j0 + c;
                double2 ev = make_double2(0.0, 0.0);
                if (k < ke && j < G) {
                    const float2 v = E[(int64_t)k * G + j];
                    ev = make_double2((double)v.x, (double)v.y);
                }
                es[kk][c] = ev;
            }
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < kBbTileK; ++kk) {
            double2 yv[4], ev[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) yv[a] = ys[ty + 16 * a][kk];
#pragma unroll
            for (int b = 0; b < 4; ++b) ev[b] = es[kk][tx + 16 * b];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    acc[a][b].x = fma(yv[a].x, ev[b].x, fma(-yv[a].y, ev[b].y, acc[a][b].x));
                    acc[a][b].y = fma(yv[a].x, ev[b].y, fma(yv[a].y, ev[b].x, acc[a][b].y));
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int32_t t = t0 + ty + 16 * a;
        if (t >= nt) continue;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int32_t j = j0 + tx + 16 * b;
            if (j < G) Tpart[((int64_t)blockIdx.z * nt + t) * G + j] = acc[a][b];
        }
    }
}

// T[i] = sum over the bin ranges r, in order, of Tpart[r][i], rounded once.
__global__ __launch_bounds__(256) void bb_table_finish_kernel(const double2 *__restrict__ Tpart, int64_t n,
                                                              int32_t nsplit, float2 *__restrict__ T)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        double2 a = Tpart[i];
        for (int32_t r = 1; r < nsplit; ++r) {
            const double2 b = Tpart[(int64_t)r * n + i];
            a.x += b.x;
            a.y += b.y;
        }
        T[i] = make_float2((float)a.x, (float)a.y);
    }
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

hipError_t launch_broadband_table_maps(const float *C, const float *w, int64_t ldc, int32_t nt, int32_t klo,
                                       int32_t khi, double f0, double df, int64_t k0, const float *H,
                                       const float *gamma, const double *tau, int32_t npix, const BbGrid &g,
                                       float *Xbb, float *Gbb, void *work, hipStream_t s)
{
    const int32_t nb = khi - klo;
    const BbLayout L = bb_layout(nt, npix, nb, g);
    char *ws = reinterpret_cast<char *>(work);
    double *v = reinterpret_cast<double *>(ws + L.gam), *gpart = v + nt;
    const int32_t nchunks = band_gamma_chunks(), per = (nt + nchunks - 1) / nchunks;
    if (!Xbb) {  // Gbb alone: the weight-side kernels by themselves
        return launch_band_gamma(w, ldc, nt, H, klo, khi, gamma, npix, v, Gbb, s);
    }
    int32_t kper;
    const int32_t ns = bb_splits(nt, nb, g, &kper);
    float2 *E = reinterpret_cast<float2 *>(ws + L.e);
    float2 *T = reinterpret_cast<float2 *>(ws + L.t);
    double *part = reinterpret_cast<double *>(ws + L.part);
    double2 *Tpart = reinterpret_cast<double2 *>(ws + L.tpart);
    const int64_t ne = (int64_t)nb * g.G;
    hipLaunchKernelGGL(bb_phase_kernel, dim3((unsigned)std::min<int64_t>((ne + 255) / 256, 16384)), dim3(256), 0, s,
                       nb, g.G, g.m, df * g.h, E);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(bb_table_kernel, dim3((unsigned)((g.G + kBbTileJ - 1) / kBbTileJ),
                                             (unsigned)((nt + kBbTileT - 1) / kBbTileT), (unsigned)ns),
                       dim3(256), 0, s, C, w, ldc, nt, klo, nb, g.G, kper, (const float2 *)E, Tpart);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nT = (int64_t)nt * g.G;
    hipLaunchKernelGGL(bb_table_finish_kernel, dim3((unsigned)std::min<int64_t>((nT + 255) / 256, 16384)), dim3(256),
                       0, s, (const double2 *)Tpart, nT, ns, T);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (Gbb) {
        e = launch_band_weights(w, ldc, nt, H, klo, khi, v, s);
        if (e != hipSuccess) return e;
    }
    // the band's centre: absolute bin k0 + klo + (nb - 1) / 2
    const double fc = f0 + ((double)(k0 + klo) + 0.5 * (nb - 1)) * df;
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

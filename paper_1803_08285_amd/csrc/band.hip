// Broadband maps (Sec. V): Xbb(p) = sum_k X(k,p), Gbb(p) = sum_k H(k) Gam(k,p)
// over rows [klo, khi).  A streaming reduction bound by HBM bandwidth.
//
// Split path (workspace given, float32 maps, npix % 4 == 0, 16-byte aligned):
//   stage 1: the rows are cut into nsplit contiguous slabs; a workgroup owns 256
//            pixel columns of one slab (one float4 per lane, 1 KB per wave
//            load), its four waves take every fourth row with four rows of X
//            and four of Gam in flight, sum in float64 and combine the waves
//            through LDS in a fixed order into partial[slab][column];
//   stage 2: one thread per column adds the slab partials in slab order and
//            rounds once.
// Single-pass path (no workspace): each workgroup owns 64 columns and sixteen
// waves stride the rows; the same fixed-order combine.  Both paths are bitwise
// reproducible for a given (npix, klo, khi).
#include <type_traits>

#include "sgwb_internal.h"

namespace sgwb {

// ---------------------------------------------------------------- single pass
constexpr int kBandCols = 64;
constexpr int kBandWaves = 16;
constexpr int kBandUnroll = 8;

template <typename T>
__global__ __launch_bounds__(1024) void band_kernel(const T *__restrict__ X, const T *__restrict__ G,
                                                    const T *__restrict__ H, int32_t npix, int32_t klo,
                                                    int32_t khi, T *__restrict__ Xbb, T *__restrict__ Gbb)
{
    __shared__ double sx[kBandWaves][kBandCols], sg[kBandWaves][kBandCols];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int64_t col = (int64_t)blockIdx.x * kBandCols + lane;
    const bool active = col < npix;
    const int64_t pc = active ? col : 0;
    double ax = 0.0, ag = 0.0;
    const bool doX = X != nullptr, doG = G != nullptr;
    int64_t k = klo + wv;
    const int64_t step = kBandWaves;
    for (; k + (kBandUnroll - 1) * step < khi; k += kBandUnroll * step) {
        T vx[kBandUnroll], vg[kBandUnroll], vh[kBandUnroll];
#pragma unroll
        for (int u = 0; u < kBandUnroll; ++u) {
            const int64_t kk = k + u * step;
            vx[u] = doX ? X[kk * npix + pc] : T(0);
            vg[u] = doG ? G[kk * npix + pc] : T(0);
            vh[u] = doG ? H[kk] : T(0);
        }
#pragma unroll
        for (int u = 0; u < kBandUnroll; ++u) {
            ax += (double)vx[u];
            ag = fma((double)vh[u], (double)vg[u], ag);
        }
    }
    for (; k < khi; k += step) {
        if (doX) ax += (double)X[k * npix + pc];
        if (doG) ag = fma((double)H[k], (double)G[k * npix + pc], ag);
    }
    sx[wv][lane] = ax;
    sg[wv][lane] = ag;
    __syncthreads();
    if (wv == 0 && active) {
        double tx = 0.0, tg = 0.0;
#pragma unroll
        for (int i = 0; i < kBandWaves; ++i) {
            tx += sx[i][lane];
            tg += sg[i][lane];
        }
        if (doX) Xbb[col] = (T)tx;
        if (doG) Gbb[col] = (T)tg;
    }
}

// ---------------------------------------------------------------- split path
constexpr int kSplitCols = 256;  // 64 lanes x float4
constexpr int kSplitWaves = 4;
constexpr int kSplitUnroll = 4;
constexpr int kSplitMinRows = 64;
constexpr int64_t kSplitTargetBlocks = 2048;

struct SplitPlan {
    int64_t ntiles, nsplit, rows_per;
};

static SplitPlan split_plan(int32_t npix, int32_t klo, int32_t khi)
{
    SplitPlan p;
    const int64_t rows = khi - klo;
    p.ntiles = (npix + kSplitCols - 1) / kSplitCols;
    int64_t ns = (kSplitTargetBlocks + p.ntiles - 1) / p.ntiles;
    const int64_t maxs = rows / kSplitMinRows > 1 ? rows / kSplitMinRows : 1;
    if (ns > maxs) ns = maxs;
    if (ns > 1024) ns = 1024;
    if (ns < 1) ns = 1;
    p.rows_per = (rows + ns - 1) / ns;
    p.nsplit = rows > 0 ? (rows + p.rows_per - 1) / p.rows_per : 1;
    return p;
}

size_t band_workspace_bytes(int32_t npix, int32_t klo, int32_t khi)
{
    const SplitPlan p = split_plan(npix, klo, khi);
    return (size_t)p.nsplit * (size_t)npix * 2 * sizeof(double);
}

__device__ inline void acc4(double a[4], float4 v)
{
    a[0] += (double)v.x;
    a[1] += (double)v.y;
    a[2] += (double)v.z;
    a[3] += (double)v.w;
}
__device__ inline void facc4(double a[4], double h, float4 v)
{
    a[0] = fma(h, (double)v.x, a[0]);
    a[1] = fma(h, (double)v.y, a[1]);
    a[2] = fma(h, (double)v.z, a[2]);
    a[3] = fma(h, (double)v.w, a[3]);
}

__global__ __launch_bounds__(256) void band_split_kernel(const float *__restrict__ X, const float *__restrict__ G,
                                                         const float *__restrict__ H, int32_t npix, int32_t klo,
                                                         int32_t khi, int64_t rows_per,
                                                         double *__restrict__ part)
{
    __shared__ double sx[kSplitWaves][kSplitCols], sg[kSplitWaves][kSplitCols];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int64_t col = (int64_t)blockIdx.x * kSplitCols + 4 * lane;
    const bool active = col < npix;
    const int64_t pc = active ? col : 0;
    const int64_t r0 = klo + (int64_t)blockIdx.y * rows_per;
    const int64_t r1 = r0 + rows_per < khi ? r0 + rows_per : khi;
    const bool doX = X != nullptr, doG = G != nullptr;
    double ax[4] = {0, 0, 0, 0}, ag[4] = {0, 0, 0, 0};
    int64_t k = r0 + wv;
    const int64_t step = kSplitWaves;
    const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
    for (; k + (kSplitUnroll - 1) * step < r1; k += kSplitUnroll * step) {
        float4 vx[kSplitUnroll], vg[kSplitUnroll];
        float vh[kSplitUnroll];
#pragma unroll
        for (int u = 0; u < kSplitUnroll; ++u) {
            const int64_t kk = k + u * step;
            vx[u] = doX ? *reinterpret_cast<const float4 *>(X + kk * npix + pc) : z4;
            vg[u] = doG ? *reinterpret_cast<const float4 *>(G + kk * npix + pc) : z4;
            vh[u] = doG ? H[kk] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < kSplitUnroll; ++u) {
            acc4(ax, vx[u]);
            facc4(ag, (double)vh[u], vg[u]);
        }
    }
    for (; k < r1; k += step) {
        if (doX) acc4(ax, *reinterpret_cast<const float4 *>(X + k * npix + pc));
        if (doG) facc4(ag, (double)H[k], *reinterpret_cast<const float4 *>(G + k * npix + pc));
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        sx[wv][4 * lane + e] = ax[e];
        sg[wv][4 * lane + e] = ag[e];
    }
    __syncthreads();
    // 256 threads combine the four waves for the 256 columns of the tile
    const int c = threadIdx.x;
    const int64_t gc = (int64_t)blockIdx.x * kSplitCols + c;
    if (gc < npix) {
        double tx = 0.0, tg = 0.0;
#pragma unroll
        for (int i = 0; i < kSplitWaves; ++i) {
            tx += sx[i][c];
            tg += sg[i][c];
        }
        double *row = part + (int64_t)blockIdx.y * 2 * npix;
        row[gc] = tx;
        row[npix + gc] = tg;
    }
}

__global__ __launch_bounds__(256) void band_finish_kernel(const double *__restrict__ part, int32_t npix,
                                                          int64_t nsplit, float *__restrict__ Xbb,
                                                          float *__restrict__ Gbb)
{
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= npix) return;
    double tx = 0.0, tg = 0.0;
    for (int64_t s = 0; s < nsplit; ++s) {
        tx += part[s * 2 * npix + c];
        tg += part[s * 2 * npix + npix + c];
    }
    if (Xbb) Xbb[c] = (float)tx;
    if (Gbb) Gbb[c] = (float)tg;
}

template <typename T>
hipError_t launch_band(const T *X, const T *G, const T *H, int32_t nf, int32_t npix, int32_t klo,
                       int32_t khi, T *Xbb, T *Gbb, void *work, size_t work_bytes, hipStream_t s)
{
    (void)nf;
    const bool split = std::is_same<T, float>::value && work != nullptr && npix % 4 == 0 &&
                       work_bytes >= band_workspace_bytes(npix, klo, khi) &&
                       ((uintptr_t)X % 16) == 0 && ((uintptr_t)G % 16) == 0 && khi > klo;
    if (split) {
        const SplitPlan p = split_plan(npix, klo, khi);
        double *part = reinterpret_cast<double *>(work);
        hipLaunchKernelGGL(band_split_kernel, dim3((unsigned)p.ntiles, (unsigned)p.nsplit), dim3(256), 0, s,
                           reinterpret_cast<const float *>(X), reinterpret_cast<const float *>(G),
                           reinterpret_cast<const float *>(H), npix, klo, khi, p.rows_per, part);
        hipLaunchKernelGGL(band_finish_kernel, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, s, part, npix,
                           p.nsplit, reinterpret_cast<float *>(Xbb), reinterpret_cast<float *>(Gbb));
        return hipGetLastError();
    }
    const unsigned nblk = (unsigned)((npix + kBandCols - 1) / kBandCols);
    hipLaunchKernelGGL(band_kernel<T>, dim3(nblk), dim3(64 * kBandWaves), 0, s, X, G, H, npix, klo, khi, Xbb, Gbb);
    return hipGetLastError();
}
template hipError_t launch_band<float>(const float *, const float *, const float *, int32_t, int32_t, int32_t,
                                       int32_t, float *, float *, void *, size_t, hipStream_t);
template hipError_t launch_band<double>(const double *, const double *, const double *, int32_t, int32_t,
                                        int32_t, int32_t, double *, double *, void *, size_t, hipStream_t);

// Broadband sums from partial sums written per 64-bin strip (dirty map) or per
// segment chunk (Fisher diagonal): out[p] = sum_{r < nrows} part[r][p] in
// float64, rounded once.  A workgroup takes 64 pixels (one per lane); wave w
// sums rows w, w + 8, ... in order and the eight partial sums are added in
// wave order: one fixed order for every call.
constexpr int kFinishWaves = 8;

__global__ __launch_bounds__(64 * kFinishWaves) void band_partial_finish_kernel(const double *__restrict__ part,
                                                                                int64_t nrows, int32_t npix,
                                                                                float *__restrict__ out)
{
    __shared__ double red[kFinishWaves][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int32_t p = blockIdx.x * 64 + lane;
    double acc = 0.0;
    if (p < npix)
        for (int64_t r = wv; r < nrows; r += kFinishWaves) acc += part[r * npix + p];
    red[wv][lane] = acc;
    __syncthreads();
    if (wv != 0 || p >= npix) return;
    double sum = red[0][lane];
#pragma unroll
    for (int k = 1; k < kFinishWaves; ++k) sum += red[k][lane];
    out[p] = (float)sum;
}

hipError_t launch_band_partial_finish(const double *part, int64_t nrows, int32_t npix, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(band_partial_finish_kernel, dim3((unsigned)((npix + 63) / 64)), dim3(64 * kFinishWaves), 0, s,
                       part, nrows, npix, out);
    return hipGetLastError();
}

// v[t] = sum_{c in [klo,khi)} H[c] w[t][c]: one workgroup of 1024 threads per
// segment, per-thread strides over the bins in four interleaved partial sums,
// then a fixed tree (float64).
constexpr int kWeightThreads = 1024;

__global__ __launch_bounds__(kWeightThreads) void band_weight_kernel(const float *__restrict__ w, int64_t ldw,
                                                                     const float *__restrict__ H, int32_t klo,
                                                                     int32_t khi, double *__restrict__ v)
{
    __shared__ double red[kWeightThreads];
    const float *row = w + (int64_t)blockIdx.x * ldw;
    // four independent partial sums per thread (their loads go out together),
    // added in a fixed order
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int32_t c = klo + threadIdx.x;
    for (; c + 3 * kWeightThreads < khi; c += 4 * kWeightThreads) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
            acc[u] = fma((double)H[c + u * kWeightThreads], (double)row[c + u * kWeightThreads], acc[u]);
    }
    for (int u = 0; c < khi; c += kWeightThreads, ++u) acc[u] = fma((double)H[c], (double)row[c], acc[u]);
    red[threadIdx.x] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    __syncthreads();
    for (int st = kWeightThreads / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) v[blockIdx.x] = red[0];
}

// Gbb[p] = sum_t v[t] gamma(t,p)^2 (float64, rounded once): kBandTChunks
// segment chunks per pixel block write partial sums in segment order, then a
// second kernel adds the chunks in order.  One thread per pixel, coalesced rows.
constexpr int kBandTChunks = 32;

__global__ __launch_bounds__(256) void band_gamma_kernel(const float *__restrict__ gamma, int32_t npix, int32_t nt,
                                                         const double *__restrict__ v, double *__restrict__ part)
{
    const int32_t p = blockIdx.x * 256 + threadIdx.x;
    if (p >= npix) return;
    const int32_t per = (nt + kBandTChunks - 1) / kBandTChunks;
    const int32_t t0 = blockIdx.y * per, t1 = min(t0 + per, nt);
    double acc = 0.0;
    for (int32_t t = t0; t < t1; ++t) {
        const double g = (double)gamma[(int64_t)t * npix + p];
        acc = fma(v[t], g * g, acc);
    }
    part[(int64_t)blockIdx.y * npix + p] = acc;
}

int32_t band_gamma_chunks() { return kBandTChunks; }

hipError_t launch_band_weights(const float *w, int64_t ldw, int32_t nt, const float *H, int32_t klo, int32_t khi,
                               double *v, hipStream_t s)
{
    hipLaunchKernelGGL(band_weight_kernel, dim3((unsigned)nt), dim3(kWeightThreads), 0, s, w, ldw, H, klo, khi, v);
    return hipGetLastError();
}

size_t band_gamma_scratch_bytes(int32_t nt, int32_t npix)
{
    return ((size_t)nt + (size_t)kBandTChunks * npix) * sizeof(double);
}

hipError_t launch_band_gamma(const float *w, int64_t ldw, int32_t nt, const float *H, int32_t klo, int32_t khi,
                             const float *gamma, int32_t npix, double *scratch, float *Gbb, hipStream_t s)
{
    double *v = scratch, *part = scratch + nt;
    hipLaunchKernelGGL(band_weight_kernel, dim3((unsigned)nt), dim3(kWeightThreads), 0, s, w, ldw, H, klo, khi, v);
    hipLaunchKernelGGL(band_gamma_kernel, dim3((unsigned)((npix + 255) / 256), kBandTChunks), dim3(256), 0, s, gamma,
                       npix, nt, v, part);
    return launch_band_partial_finish(part, kBandTChunks, npix, Gbb, s);
}

}  // namespace sgwb

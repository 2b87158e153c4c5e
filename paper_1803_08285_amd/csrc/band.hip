// Broadband maps (Sec. V): Xbb(p) = sum_k X(k,p), Gbb(p) = sum_k H(k) Gam(k,p)
// over rows [klo, khi).  A streaming reduction bound by HBM bandwidth: each
// workgroup owns 64 pixel columns; its four waves take rows klo + w, klo + w + 4,
// ... with eight rows in flight per wave, sum in float64, and combine through
// LDS in a fixed order (bitwise reproducible).
#include "sgwb_internal.h"

namespace sgwb {

constexpr int kBandCols = 64;
constexpr int kBandWaves = 4;
constexpr int kBandUnroll = 8;

template <typename T>
__global__ __launch_bounds__(256) void band_kernel(const T *__restrict__ X, const T *__restrict__ G,
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

template <typename T>
hipError_t launch_band(const T *X, const T *G, const T *H, int32_t nf, int32_t npix, int32_t klo,
                       int32_t khi, T *Xbb, T *Gbb, hipStream_t s)
{
    (void)nf;
    const unsigned nblk = (unsigned)((npix + kBandCols - 1) / kBandCols);
    hipLaunchKernelGGL(band_kernel<T>, dim3(nblk), dim3(256), 0, s, X, G, H, npix, klo, khi, Xbb, Gbb);
    return hipGetLastError();
}
template hipError_t launch_band<float>(const float *, const float *, const float *, int32_t, int32_t,
                                       int32_t, int32_t, float *, float *, hipStream_t);
template hipError_t launch_band<double>(const double *, const double *, const double *, int32_t, int32_t,
                                        int32_t, int32_t, double *, double *, hipStream_t);

}  // namespace sgwb

// Network sums over baselines (the sum over I of Eq. eq:narrowband) and the
// directed and isotropic contractions of Sec. V: a directed search for a
// source adds the values of the pixels that contain it; the isotropic search
// adds all pixels (HEALPix pixels have equal area, so no weights).  Both sums
// accumulate in float64 in a fixed order and round once, so results are
// reproducible bit for bit.  HBM-bound.
#include <stdint.h>

#include "sgwb_internal.h"

namespace sgwb {

typedef float f32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void network_sum_kernel(MapList l, int64_t n, float *__restrict__ out)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        double acc = 0.0;
        for (int m = 0; m < l.n; ++m) acc += (double)l.p[m][i];
        out[i] = (float)acc;
    }
}

// The same sums four elements at a time (16-byte nontemporal loads: every
// value is read once), two vectors in flight per thread; the order of the
// sums per element is the same, so the bits are too.
__global__ __launch_bounds__(256) void network_sum4_kernel(MapList l, int64_t n4, f32x4 *__restrict__ out)
{
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += 2 * stride) {
        const int64_t i2 = i + stride < n4 ? i + stride : i;  // a lone last vector is summed twice, stored once
        double a[2][4] = {};
        for (int m = 0; m < l.n; ++m) {
            const f32x4 *src = reinterpret_cast<const f32x4 *>(l.p[m]);
            const f32x4 u = __builtin_nontemporal_load(src + i), v = __builtin_nontemporal_load(src + i2);
            a[0][0] += (double)u.x;
            a[0][1] += (double)u.y;
            a[0][2] += (double)u.z;
            a[0][3] += (double)u.w;
            a[1][0] += (double)v.x;
            a[1][1] += (double)v.y;
            a[1][2] += (double)v.z;
            a[1][3] += (double)v.w;
        }
        const f32x4 r0 = {(float)a[0][0], (float)a[0][1], (float)a[0][2], (float)a[0][3]};
        __builtin_nontemporal_store(r0, out + i);
        if (i2 != i) {
            const f32x4 r1 = {(float)a[1][0], (float)a[1][1], (float)a[1][2], (float)a[1][3]};
            __builtin_nontemporal_store(r1, out + i2);
        }
    }
}

// One workgroup per row; each thread sums a fixed stride of the selection, then
// a fixed tree over the 256 partial sums.  V4: the whole row in 16-byte loads
// (thread t takes elements 4t .. 4t + 3, then 4 (t + 256) .., in that order).
template <bool V4>
__global__ __launch_bounds__(256) void contract_kernel(const float *__restrict__ M, int32_t npix,
                                                       const int32_t *__restrict__ pix, int32_t nsel,
                                                       float *__restrict__ out)
{
    __shared__ double red[256];
    const float *row = M + (int64_t)blockIdx.x * npix;
    double acc = 0.0;
    if constexpr (V4) {
        const f32x4 *r4 = reinterpret_cast<const f32x4 *>(row);
        for (int32_t j = threadIdx.x; j < npix / 4; j += 256) {
            const f32x4 v = __builtin_nontemporal_load(r4 + j);
            acc += (double)v.x;
            acc += (double)v.y;
            acc += (double)v.z;
            acc += (double)v.w;
        }
    } else {
        const int32_t n = pix ? nsel : npix;
        for (int32_t j = threadIdx.x; j < n; j += 256) acc += (double)row[pix ? pix[j] : j];
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = (float)red[0];
}

static bool aligned16(const void *p) { return reinterpret_cast<uintptr_t>(p) % 16 == 0; }

hipError_t launch_network_sum(const MapList &l, int64_t n, float *out, hipStream_t s)
{
    bool v4 = n % 4 == 0 && aligned16(out);
    for (int m = 0; m < l.n; ++m) v4 = v4 && aligned16(l.p[m]);
    if (v4) {
        const int64_t n4 = n / 4;
        const unsigned g = (unsigned)std::min<int64_t>((n4 + 511) / 512, 8192);
        hipLaunchKernelGGL(network_sum4_kernel, dim3(g), dim3(256), 0, s, l, n4, reinterpret_cast<f32x4 *>(out));
        return hipGetLastError();
    }
    const unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(network_sum_kernel, dim3(g), dim3(256), 0, s, l, n, out);
    return hipGetLastError();
}

hipError_t launch_contract(const float *M, int32_t nf, int32_t npix, const int32_t *pix, int32_t nsel, float *out,
                           hipStream_t s)
{
    if (!pix && npix % 4 == 0 && aligned16(M))
        hipLaunchKernelGGL(contract_kernel<true>, dim3((unsigned)nf), dim3(256), 0, s, M, npix, pix, nsel, out);
    else
        hipLaunchKernelGGL(contract_kernel<false>, dim3((unsigned)nf), dim3(256), 0, s, M, npix, pix, nsel, out);
    return hipGetLastError();
}

}  // namespace sgwb

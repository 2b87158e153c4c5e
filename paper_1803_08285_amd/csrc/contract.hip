// Network sums over baselines (the sum over I of Eq. eq:narrowband) and the
// directed and isotropic contractions of Sec. V: a directed search for a
// source adds the values of the pixels that contain it; the isotropic search
// adds all pixels (HEALPix pixels have equal area, so no weights).  Both sums
// accumulate in float64 in a fixed order and round once, so results are
// reproducible bit for bit.  HBM-bound.
#include "sgwb_internal.h"

namespace sgwb {

__global__ __launch_bounds__(256) void network_sum_kernel(MapList l, int64_t n, float *__restrict__ out)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        double acc = 0.0;
        for (int m = 0; m < l.n; ++m) acc += (double)l.p[m][i];
        out[i] = (float)acc;
    }
}

// One workgroup per row; each thread sums a fixed stride of the selection, then
// a fixed tree over the 256 partial sums.
__global__ __launch_bounds__(256) void contract_kernel(const float *__restrict__ M, int32_t npix,
                                                       const int32_t *__restrict__ pix, int32_t nsel,
                                                       float *__restrict__ out)
{
    __shared__ double red[256];
    const float *row = M + (int64_t)blockIdx.x * npix;
    const int32_t n = pix ? nsel : npix;
    double acc = 0.0;
    for (int32_t j = threadIdx.x; j < n; j += 256) acc += (double)row[pix ? pix[j] : j];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = (float)red[0];
}

hipError_t launch_network_sum(const MapList &l, int64_t n, float *out, hipStream_t s)
{
    const unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(network_sum_kernel, dim3(g), dim3(256), 0, s, l, n, out);
    return hipGetLastError();
}

hipError_t launch_contract(const float *M, int32_t nf, int32_t npix, const int32_t *pix, int32_t nsel, float *out,
                           hipStream_t s)
{
    hipLaunchKernelGGL(contract_kernel, dim3((unsigned)nf), dim3(256), 0, s, M, npix, pix, nsel, out);
    return hipGetLastError();
}

}  // namespace sgwb

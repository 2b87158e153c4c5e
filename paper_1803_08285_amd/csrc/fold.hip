// Folding (Sec. II.B): the data of ndays sidereal days, nt segments each
// (segment tau of day d is absolute segment a = d nt + tau), summed into one
// folded day.  With s = sigma^-2, eps = W for a neighbour a +- 1 that exists
// and has data, and only segments with data contributing:
//   v_tau = sum_d s_a
//   u_tau = sum_d eps_{a-1} (s_a + s_{a-1}) / 2,  w_tau = sum_d eps_{a+1} (s_a + s_{a+1}) / 2
//   x_tau = sum_d [ s_a C_a - eps_{a-1} (s_a + s_{a-1}) / 2 C_{a-1}
//                           - eps_{a+1} (s_a + s_{a+1}) / 2 C_{a+1} ]
// The neighbour of a day's first segment is the previous day's last segment.
// One thread per (folded segment, bin): per day it reads its segment and the
// two neighbours (the neighbour rows are other threads' own rows, read at
// about the same time, so they come from L2; HBM sees each row once) and
// accumulates in float64 in the oracle's order; one rounding to float32 at the
// end.  Few registers and loads issued ahead of the uniform presence branches,
// so many waves per SIMD keep enough loads in flight for an HBM-bound sweep.
#include "sgwb_internal.h"

namespace sgwb {

__global__ __launch_bounds__(256) void fold_kernel(const float2 *__restrict__ C, const float *__restrict__ sv,
                                                   const uint8_t *__restrict__ present, int64_t ldc, int32_t ndays,
                                                   int32_t nt, int32_t nf, double W, float *__restrict__ v,
                                                   float *__restrict__ u, float *__restrict__ w,
                                                   float2 *__restrict__ x)
{
#pragma clang fp contract(off)  // the oracle's order and roundings: sums bitwise equal before the final rounding
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int tau = blockIdx.y;
    if (c >= nf) return;
    const int64_t nseg = (int64_t)ndays * nt;
    const double hw = 0.5 * W;
    double vs = 0.0, us = 0.0, ws = 0.0, xr = 0.0, xi = 0.0;
    // Branch-free per day (selects, not products, so data of segments without
    // data never reach the sums, whatever they hold), four days per iteration
    // so that their loads are in flight together.
#pragma unroll 4
    for (int d = 0; d < ndays; ++d) {
        const int64_t a = (int64_t)d * nt + tau;
        const int64_t ap = a > 0 ? a - 1 : a, an = a + 1 < nseg ? a + 1 : a;  // clamped: loads stay in bounds
        const bool pa = present[a] != 0;
        const bool pp = pa && a > 0 && present[ap] != 0;
        const bool pn = pa && a + 1 < nseg && present[an] != 0;
        const float s0 = sv[a * ldc + c], s1 = sv[ap * ldc + c], s2 = sv[an * ldc + c];
        const float2 c0 = C[a * ldc + c], c1 = C[ap * ldc + c], c2 = C[an * ldc + c];
        if (pa) {  // uniform over the workgroup
            const double sa = s0;
            vs += sa;
            xr += sa * (double)c0.x;
            xi += sa * (double)c0.y;
            if (pp) {
                const double e = hw * (sa + (double)s1);
                us += e;
                xr -= e * (double)c1.x;
                xi -= e * (double)c1.y;
            }
            if (pn) {
                const double e = hw * (sa + (double)s2);
                ws += e;
                xr -= e * (double)c2.x;
                xi -= e * (double)c2.y;
            }
        }
    }
    const int64_t o = (int64_t)tau * nf + c;
    v[o] = (float)vs;
    u[o] = (float)us;
    w[o] = (float)ws;
    x[o] = make_float2((float)xr, (float)xi);
}

hipError_t launch_fold(const float *C, const float *sv, const uint8_t *present, int64_t ldc, int32_t ndays, int32_t nt,
                       int32_t nf, double W, float *v, float *u, float *w, float *x, hipStream_t s)
{
    const dim3 grid((unsigned)((nf + 255) / 256), (unsigned)nt);
    hipLaunchKernelGGL(fold_kernel, grid, dim3(256), 0, s, reinterpret_cast<const float2 *>(C), sv, present, ldc,
                       ndays, nt, nf, W, v, u, w, reinterpret_cast<float2 *>(x));
    return hipGetLastError();
}

}  // namespace sgwb

// Folding (Sec. II.B): the data of ndays sidereal days, nt segments each
// (segment tau of day d is absolute segment a = d nt + tau), summed into one
// folded day.  With s = sigma^-2, eps = W for a neighbour a +- 1 that exists
// and has data, and only segments with data contributing:
//   v_tau = sum_d s_a
//   u_tau = sum_d eps_{a-1} (s_a + s_{a-1}) / 2,  w_tau = sum_d eps_{a+1} (s_a + s_{a+1}) / 2
//   x_tau = sum_d [ s_a C_a - eps_{a-1} (s_a + s_{a-1}) / 2 C_{a-1}
//                           - eps_{a+1} (s_a + s_{a+1}) / 2 C_{a+1} ]
// The neighbour of a day's first segment is the previous day's last segment.
// A workgroup owns 256 bins x kFoldRows folded segments; per day it reads the
// kFoldRows + 2 absolute segments it needs (coalesced rows) and accumulates in
// float64; one rounding to float32 at the end.  HBM-bound: each input row is
// read (kFoldRows + 2) / kFoldRows times.
#include "sgwb_internal.h"

namespace sgwb {

constexpr int kFoldRows = 8;

__global__ __launch_bounds__(256) void fold_kernel(const float2 *__restrict__ C, const float *__restrict__ sv,
                                                   const uint8_t *__restrict__ present, int64_t ldc, int32_t ndays,
                                                   int32_t nt, int32_t nf, double W, float *__restrict__ v,
                                                   float *__restrict__ u, float *__restrict__ w,
                                                   float2 *__restrict__ x)
{
#pragma clang fp contract(off)  // the oracle's order and roundings: sums bitwise equal before the final rounding
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int tau0 = blockIdx.y * kFoldRows;
    const bool col_ok = c < nf;
    const int64_t cc = col_ok ? c : 0;
    const int64_t nseg = (int64_t)ndays * nt;
    double vs[kFoldRows], us[kFoldRows], ws[kFoldRows], xr[kFoldRows], xi[kFoldRows];
#pragma unroll
    for (int r = 0; r < kFoldRows; ++r) vs[r] = us[r] = ws[r] = xr[r] = xi[r] = 0.0;
    const double hw = 0.5 * W;
    for (int d = 0; d < ndays; ++d) {
        // absolute segments a0 - 1 .. a0 + kFoldRows (index j = 0 .. kFoldRows + 1)
        const int64_t a0 = (int64_t)d * nt + tau0;
        double s[kFoldRows + 2], re[kFoldRows + 2], im[kFoldRows + 2];
        bool pr[kFoldRows + 2];
#pragma unroll
        for (int j = 0; j < kFoldRows + 2; ++j) {
            // neighbours are consecutive in absolute time: a row past the end of the
            // folded day is the next day's first segment (the successor of tau = nt - 1)
            const int64_t a = a0 - 1 + j;
            pr[j] = a >= 0 && a < nseg && present[a];
            s[j] = re[j] = im[j] = 0.0;
            if (pr[j]) {
                s[j] = sv[a * ldc + cc];
                const float2 cv = C[a * ldc + cc];
                re[j] = cv.x;
                im[j] = cv.y;
            }
        }
#pragma unroll
        for (int r = 0; r < kFoldRows; ++r) {
            const int j = r + 1;
            if (tau0 + r >= nt || !pr[j]) continue;
            vs[r] += s[j];
            xr[r] += s[j] * re[j];
            xi[r] += s[j] * im[j];
            if (pr[j - 1]) {
                const double e = hw * (s[j] + s[j - 1]);
                us[r] += e;
                xr[r] -= e * re[j - 1];
                xi[r] -= e * im[j - 1];
            }
            if (pr[j + 1]) {
                const double e = hw * (s[j] + s[j + 1]);
                ws[r] += e;
                xr[r] -= e * re[j + 1];
                xi[r] -= e * im[j + 1];
            }
        }
    }
    if (!col_ok) return;
#pragma unroll
    for (int r = 0; r < kFoldRows; ++r) {
        const int tau = tau0 + r;
        if (tau >= nt) break;
        const int64_t o = (int64_t)tau * nf + c;
        v[o] = (float)vs[r];
        u[o] = (float)us[r];
        w[o] = (float)ws[r];
        x[o] = make_float2((float)xr[r], (float)xi[r]);
    }
}

hipError_t launch_fold(const float *C, const float *sv, const uint8_t *present, int64_t ldc, int32_t ndays, int32_t nt,
                       int32_t nf, double W, float *v, float *u, float *w, float *x, hipStream_t s)
{
    const dim3 grid((unsigned)((nf + 255) / 256), (unsigned)((nt + kFoldRows - 1) / kFoldRows));
    hipLaunchKernelGGL(fold_kernel, grid, dim3(256), 0, s, reinterpret_cast<const float2 *>(C), sv, present, ldc,
                       ndays, nt, nf, W, v, u, w, reinterpret_cast<float2 *>(x));
    return hipGetLastError();
}

}  // namespace sgwb

// Folding (Sec. II.B): the data of ndays sidereal days, nt segments each
// (segment tau of day d is absolute segment a = d nt + tau), summed into one
// folded day.  With s = sigma^-2, eps = W for a neighbour a +- 1 that exists
// and has data, and only segments with data contributing:
//   v_tau = sum_d s_a
//   u_tau = sum_d eps_{a-1} (s_a + s_{a-1}) / 2,  w_tau = sum_d eps_{a+1} (s_a + s_{a+1}) / 2
//   x_tau = sum_d [ s_a C_a - eps_{a-1} (s_a + s_{a-1}) / 2 C_{a-1}
//                           - eps_{a+1} (s_a + s_{a+1}) / 2 C_{a+1} ]
// The neighbour of a day's first segment is the previous day's last segment.
// One thread per (group of kFoldT consecutive folded segments, bin): per day it
// reads the group's rows and the two neighbouring rows (kFoldT + 2 rows for
// kFoldT outputs, where one thread per segment read three rows per output)
// and accumulates each output in float64 in the oracle's order; one rounding
// to float32 at the end.  Loads are issued ahead of the uniform presence
// branches, so the waves keep enough loads in flight for an HBM-bound sweep.
#include "sgwb_internal.h"

namespace sgwb {

constexpr int kFoldT = 4;  // consecutive folded segments per thread

__global__ __launch_bounds__(256) void fold_kernel(const float2 *__restrict__ C, const float *__restrict__ sv,
                                                   const uint8_t *__restrict__ present, int64_t ldc, int32_t ndays,
                                                   int32_t nt, int32_t nf, double W, float *__restrict__ v,
                                                   float *__restrict__ u, float *__restrict__ w,
                                                   float2 *__restrict__ x)
{
#pragma clang fp contract(off)  // the oracle's order and roundings: sums bitwise equal before the final rounding
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int tau0 = blockIdx.y * kFoldT;
    if (c >= nf) return;
    const int64_t nseg = (int64_t)ndays * nt;
    const double hw = 0.5 * W;
    double vs[kFoldT], us[kFoldT], ws[kFoldT], xr[kFoldT], xi[kFoldT];
#pragma unroll
    for (int k = 0; k < kFoldT; ++k) vs[k] = us[k] = ws[k] = xr[k] = xi[k] = 0.0;
    // Branch-free loads (selects, not products, so data of segments without
    // data never reach the sums, whatever they hold); rows are clamped into
    // the array, and a clamped row is never used.
#pragma unroll 2
    for (int d = 0; d < ndays; ++d) {
        const int64_t a0 = (int64_t)d * nt + tau0;  // the group's first segment
        float s[kFoldT + 2];
        float2 cc[kFoldT + 2];
        bool pr[kFoldT + 2];
#pragma unroll
        for (int r = 0; r < kFoldT + 2; ++r) {
            const int64_t a = min(max(a0 - 1 + r, (int64_t)0), nseg - 1);
            s[r] = sv[a * ldc + c];
            cc[r] = C[a * ldc + c];
            pr[r] = present[a] != 0;
        }
#pragma unroll
        for (int k = 0; k < kFoldT; ++k) {
            if (tau0 + k >= nt) break;  // the last group is ragged (uniform)
            const int64_t a = a0 + k;   // rows k, k + 1, k + 2 are a - 1, a, a + 1
            const bool pa = pr[k + 1];
            const bool pp = pa && a > 0 && pr[k];
            const bool pn = pa && a + 1 < nseg && pr[k + 2];
            if (pa) {  // uniform over the workgroup
                const double sa = s[k + 1];
                vs[k] += sa;
                xr[k] += sa * (double)cc[k + 1].x;
                xi[k] += sa * (double)cc[k + 1].y;
                if (pp) {
                    const double e = hw * (sa + (double)s[k]);
                    us[k] += e;
                    xr[k] -= e * (double)cc[k].x;
                    xi[k] -= e * (double)cc[k].y;
                }
                if (pn) {
                    const double e = hw * (sa + (double)s[k + 2]);
                    ws[k] += e;
                    xr[k] -= e * (double)cc[k + 2].x;
                    xi[k] -= e * (double)cc[k + 2].y;
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < kFoldT; ++k) {
        if (tau0 + k >= nt) break;
        const int64_t o = (int64_t)(tau0 + k) * nf + c;
        v[o] = (float)vs[k];
        u[o] = (float)us[k];
        w[o] = (float)ws[k];
        x[o] = make_float2((float)xr[k], (float)xi[k]);
    }
}

hipError_t launch_fold(const float *C, const float *sv, const uint8_t *present, int64_t ldc, int32_t ndays, int32_t nt,
                       int32_t nf, double W, float *v, float *u, float *w, float *x, hipStream_t s)
{
    const dim3 grid((unsigned)((nf + 255) / 256), (unsigned)((nt + kFoldT - 1) / kFoldT));
    hipLaunchKernelGGL(fold_kernel, grid, dim3(256), 0, s, reinterpret_cast<const float2 *>(C), sv, present, ldc,
                       ndays, nt, nf, W, v, u, w, reinterpret_cast<float2 *>(x));
    return hipGetLastError();
}

}  // namespace sgwb

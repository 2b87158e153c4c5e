// Full Fisher information matrix of a band and the conjugate-gradient clean map
// (Eqs. eq_fisher, eq_ML_linear and its footnote; broadband H weighting of
// Sec. V), for separable weights w(t,f) = a(t) b(f):
//   G(p,q) = sum_{k in band} H_k sum_t w(t,k) gamma_p gamma_q cos 2 pi f_k (tau_p - tau_q)
//          = sum_t a_t gamma_p(t) gamma_q(t) W(tau_p(t) - tau_q(t)),
//   W(D)   = sum_{k in band} H_k b_k cos 2 pi f_k D.
// Route (not the paper's): the band sum is done once, into a table of W and
// its derivative on a grid of delay differences D_j = j delta >= 0 (W is even)
// with 64 points per period of the band's highest frequency, up to 4 R / c; the
// matrix then costs one cubic Hermite interpolation per (t, p, q)
// (relative error below (2 pi / 64)^4 / 384 = 2.4e-7).  Delay differences are
// taken in float64 before the table index is formed.
#include "sgwb_internal.h"

namespace sgwb {

constexpr int kFt = 64;      // matrix tile edge
constexpr int kFtSeg = 16;   // segments staged per step
constexpr double kTableMaxDelay = 4.0 * kEarthRadius / kLightSpeed;  // |tau_p - tau_q| bound on the Earth

void fisher_table_geometry(double f_max, double *delta, int32_t *J)
{
    *delta = 1.0 / (64.0 * std::max(f_max, 1e-3));
    *J = (int32_t)std::ceil(kTableMaxDelay / *delta) + 2;  // entries 0..J
}

// Table entry j: (W(D_j), delta dW/dD (D_j)), phases reduced in float64 at every
// 64th bin and advanced by a float64 rotation in between.
__global__ __launch_bounds__(256) void delay_table_kernel(const float *__restrict__ H, const float *__restrict__ b,
                                                          int32_t clo, int32_t chi, double f0, double df, int64_t k0,
                                                          double delta, int32_t J, float2 *__restrict__ table)
{
    const int32_t j = blockIdx.x * 256 + threadIdx.x;
    if (j > J) return;
    const double D = (double)j * delta;
    double er, ei;
    sincospi(2.0 * df * D, &ei, &er);
    double sw = 0.0, sd = 0.0;
    for (int32_t c0 = clo; c0 < chi; c0 += 64) {
        const double fa = f0 + (double)(k0 + c0) * df;
        const double x = fa * D, r = x - rint(x);
        double zr, zi;
        sincospi(2.0 * r, &zi, &zr);
        const int32_t c1 = min(c0 + 64, chi);
        for (int32_t c = c0; c < c1; ++c) {
            const double hb = (double)H[c] * (double)b[c];
            const double f = f0 + (double)(k0 + c) * df;
            sw += hb * zr;
            sd -= hb * 2.0 * M_PI * f * zi;
            const double nr = zr * er - zi * ei, ni = zr * ei + zi * er;
            zr = nr;
            zi = ni;
        }
    }
    table[j] = make_float2((float)sw, (float)(sd * delta));
}

// Upper-triangle tile k of an n x n tile grid: row r, column c >= r.
__device__ __forceinline__ void tri_tile(int64_t k, int64_t n, int64_t &r, int64_t &c)
{
    const double m = (double)(2 * n + 1);
    r = (int64_t)((m - sqrt(m * m - 8.0 * (double)k)) * 0.5);
    auto start = [n](int64_t rr) { return rr * n - rr * (rr - 1) / 2; };
    while (r > 0 && start(r) > k) --r;
    while (start(r + 1) <= k) ++r;
    c = r + (k - start(r));
}

__global__ __launch_bounds__(256) void fisher_full_kernel(const float *__restrict__ a, const float *__restrict__ gamma,
                                                          const double *__restrict__ tau, int32_t nt, int32_t npix,
                                                          const float2 *__restrict__ table, int32_t J, double inv_delta,
                                                          float *__restrict__ G)
{
    __shared__ float gP[kFtSeg][kFt], gQ[kFtSeg][kFt];
    __shared__ double tP[kFtSeg][kFt], tQ[kFtSeg][kFt];
    const int64_t nT = (npix + kFt - 1) / kFt;
    int64_t tr, tc;
    tri_tile(blockIdx.x, nT, tr, tc);
    const int ty = threadIdx.x / 16, tx = threadIdx.x % 16;
    float acc[4][4] = {};
    const int jmax = J - 1;
    for (int t0 = 0; t0 < nt; t0 += kFtSeg) {
        __syncthreads();
        for (int e = threadIdx.x; e < kFtSeg * kFt; e += 256) {
            const int tt = e / kFt, i = e % kFt, t = t0 + tt;
            const int64_t p = tr * kFt + i, q = tc * kFt + i;
            const bool ok = t < nt;
            const float at = ok ? a[t] : 0.0f;
            gP[tt][i] = ok && p < npix ? at * gamma[(int64_t)t * npix + p] : 0.0f;
            tP[tt][i] = ok && p < npix ? tau[(int64_t)t * npix + p] : 0.0;
            gQ[tt][i] = ok && q < npix ? gamma[(int64_t)t * npix + q] : 0.0f;
            tQ[tt][i] = ok && q < npix ? tau[(int64_t)t * npix + q] : 0.0;
        }
        __syncthreads();
        const int tn = min(kFtSeg, nt - t0);
        for (int tt = 0; tt < tn; ++tt) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float gp = gP[tt][ty * 4 + i];
                const double tp = tP[tt][ty * 4 + i];
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    // |D| makes (p,q) and (q,p) the same arithmetic
                    const double u = fabs(tp - tQ[tt][tx * 4 + jj]) * inv_delta;
                    const int k = min((int)u, jmax);
                    const float s = fminf((float)(u - (double)k), 1.0f);
                    const float2 w0 = table[k], w1 = table[k + 1];
                    const float s2 = s * s, s3 = s2 * s;
                    const float W = (2.0f * s3 - 3.0f * s2 + 1.0f) * w0.x + (s3 - 2.0f * s2 + s) * w0.y +
                                    (3.0f * s2 - 2.0f * s3) * w1.x + (s3 - s2) * w1.y;
                    acc[i][jj] = fmaf(gp * gQ[tt][tx * 4 + jj], W, acc[i][jj]);
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int64_t p = tr * kFt + ty * 4 + i, q = tc * kFt + tx * 4 + jj;
            // a diagonal tile writes its upper triangle and the mirror of it
            if (p < npix && q < npix && (tr != tc || p <= q)) {
                G[p * npix + q] = acc[i][jj];
                G[q * npix + p] = acc[i][jj];
            }
        }
}

size_t fisher_full_workspace_bytes(double f_max)
{
    double delta;
    int32_t J;
    fisher_table_geometry(f_max, &delta, &J);
    return (size_t)(J + 1) * sizeof(float2);
}

hipError_t launch_fisher_full(const float *a, const float *b, const float *H, int32_t clo, int32_t chi, double f0,
                              double df, int64_t k0, const float *gamma, const double *tau, int32_t nt, int32_t npix,
                              float *G, void *work, hipStream_t s)
{
    const double f_max = f0 + (double)(k0 + chi - 1) * df;
    double delta;
    int32_t J;
    fisher_table_geometry(f_max, &delta, &J);
    float2 *table = reinterpret_cast<float2 *>(work);
    hipLaunchKernelGGL(delay_table_kernel, dim3((unsigned)((J + 1 + 255) / 256)), dim3(256), 0, s, H, b, clo, chi,
                       f0, df, k0, delta, J, table);
    const int64_t nT = (npix + kFt - 1) / kFt, ntiles = nT * (nT + 1) / 2;
    if (ntiles > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fisher_full_kernel, dim3((unsigned)ntiles), dim3(256), 0, s, a, gamma, tau, nt, npix, table, J,
                       1.0 / delta, G);
    return hipGetLastError();
}

// ---- conjugate gradient on G P = X (float64 vectors, fixed-order sums) ----
constexpr int kCgParts = 256;

__global__ __launch_bounds__(256) void cg_matvec_kernel(const float *__restrict__ G, const double *__restrict__ p,
                                                        int32_t n, double *__restrict__ q)
{
    __shared__ double red[256];
    const float *row = G + (int64_t)blockIdx.x * n;
    double acc = 0.0;
    for (int32_t j = threadIdx.x; j < n; j += 256) acc += (double)row[j] * p[j];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) q[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void cg_dot_kernel(const double *__restrict__ x, const double *__restrict__ y,
                                                     int32_t n, double *__restrict__ part)
{
    __shared__ double red[256];
    double acc = 0.0;
    for (int32_t j = blockIdx.x * 256 + threadIdx.x; j < n; j += kCgParts * 256) acc += x[j] * y[j];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void cg_dot_final_kernel(const double *__restrict__ part, double *__restrict__ out)
{
    __shared__ double red[256];
    red[threadIdx.x] = part[threadIdx.x];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

// x = 0, r = p = X
__global__ __launch_bounds__(256) void cg_init_kernel(const float *__restrict__ X, int32_t n, double *__restrict__ x,
                                                      double *__restrict__ r, double *__restrict__ p)
{
    const int32_t j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    x[j] = 0.0;
    r[j] = p[j] = (double)X[j];
}

// alpha = rr / pq (0 once the residual vanishes); x += alpha p; r -= alpha q
__global__ __launch_bounds__(256) void cg_step_kernel(double *__restrict__ x, double *__restrict__ r,
                                                      const double *__restrict__ p, const double *__restrict__ q,
                                                      const double *__restrict__ rr, const double *__restrict__ pq,
                                                      int32_t n)
{
    const int32_t j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const double alpha = (rr[0] != 0.0 && pq[0] != 0.0) ? rr[0] / pq[0] : 0.0;
    x[j] += alpha * p[j];
    r[j] -= alpha * q[j];
}

// p = r + (rr_new / rr) p
__global__ __launch_bounds__(256) void cg_dir_kernel(double *__restrict__ p, const double *__restrict__ r,
                                                     const double *__restrict__ rr, const double *__restrict__ rr_new,
                                                     int32_t n)
{
    const int32_t j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const double beta = rr[0] != 0.0 ? rr_new[0] / rr[0] : 0.0;
    p[j] = r[j] + beta * p[j];
}

__global__ __launch_bounds__(256) void cg_out_kernel(const double *__restrict__ x, int32_t n, float *__restrict__ P)
{
    const int32_t j = blockIdx.x * 256 + threadIdx.x;
    if (j < n) P[j] = (float)x[j];
}

size_t cg_workspace_bytes(int32_t n)
{
    return (size_t)4 * n * sizeof(double) + (kCgParts + 8) * sizeof(double);
}

hipError_t launch_clean_map_cg(const float *G, const float *X, int32_t n, int32_t niter, float *P, void *work,
                               hipStream_t s)
{
    double *x = reinterpret_cast<double *>(work), *r = x + n, *p = r + n, *q = p + n, *part = q + n;
    double *sc = part + kCgParts;  // sc[0], sc[1]: |r|^2 of even/odd iterations; sc[2]: p.q
    const unsigned g = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(cg_init_kernel, dim3(g), dim3(256), 0, s, X, n, x, r, p);
    hipLaunchKernelGGL(cg_dot_kernel, dim3(kCgParts), dim3(256), 0, s, r, r, n, part);
    hipLaunchKernelGGL(cg_dot_final_kernel, dim3(1), dim3(256), 0, s, part, sc);
    for (int32_t it = 0; it < niter; ++it) {
        double *rr = sc + (it & 1), *rr_new = sc + ((it + 1) & 1);
        hipLaunchKernelGGL(cg_matvec_kernel, dim3((unsigned)n), dim3(256), 0, s, G, p, n, q);
        hipLaunchKernelGGL(cg_dot_kernel, dim3(kCgParts), dim3(256), 0, s, p, q, n, part);
        hipLaunchKernelGGL(cg_dot_final_kernel, dim3(1), dim3(256), 0, s, part, sc + 2);
        hipLaunchKernelGGL(cg_step_kernel, dim3(g), dim3(256), 0, s, x, r, p, q, rr, sc + 2, n);
        hipLaunchKernelGGL(cg_dot_kernel, dim3(kCgParts), dim3(256), 0, s, r, r, n, part);
        hipLaunchKernelGGL(cg_dot_final_kernel, dim3(1), dim3(256), 0, s, part, rr_new);
        hipLaunchKernelGGL(cg_dir_kernel, dim3(g), dim3(256), 0, s, p, r, rr, rr_new, n);
    }
    hipLaunchKernelGGL(cg_out_kernel, dim3(g), dim3(256), 0, s, x, n, P);
    return hipGetLastError();
}

}  // namespace sgwb

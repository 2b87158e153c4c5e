// Fisher diagonal with the overlapping-window neighbour terms (Sec. II.B,
// Eq. fwGamma with p = p'):
//   Gam(k,p) = Re sum_t conj(K_t) [K_t v_t - K_{t-1} u_t - K_{t+1} w_t],
//   K_t = gamma(t,p) e^{2 pi i f_k tau(t,p)}.
// The folded day is periodic (the geometry repeats every sidereal day), so
// segment nt - 1 is followed by segment 0.  The v term is the plain diagonal
// sum_t v gamma^2 (the beam GEMM).  The two neighbour terms of a pair of
// consecutive segments (q, q+ = q + 1 mod nt) are
//   -(u_{q+} + w_q) gamma_q gamma_{q+} cos 2 pi f_k (tau_{q+} - tau_q)
// (real parts of conj(K_{q+}) K_q u_{q+} and conj(K_q) K_{q+} w_q, cos being
// even), i.e. a dirty map over the nt pairs with real data
// y'(q,k) = -(u(q+,k) + w(q,k)), seeds gamma'(q,p) = gamma_q gamma_{q+} and
// tau'(q,p) = tau_{q+} - tau_q.  The derived seeds keep the exact antipodal
// symmetry of the originals (gamma' even, tau' odd), so the same kernels run
// on them, adding into Gam.
#include "sgwb_internal.h"

namespace sgwb {

__global__ __launch_bounds__(256) void pair_seeds_kernel(const float *__restrict__ gamma,
                                                         const double *__restrict__ tau, int64_t n, int64_t npix,
                                                         float *__restrict__ g2, double *__restrict__ t2)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int64_t j = i + npix < n ? i + npix : i + npix - n;  // same pixel, next segment (periodic)
        g2[i] = gamma[i] * gamma[j];
        t2[i] = tau[j] - tau[i];
    }
}

__global__ __launch_bounds__(256) void pair_weights_kernel(const float *__restrict__ u, const float *__restrict__ wn,
                                                           int64_t ldc, int32_t nq, int32_t nf,
                                                           float *__restrict__ y)
{
    const int64_t n = (int64_t)nq * nf;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int64_t q = i / nf, c = i - q * nf, qn = q + 1 < nq ? q + 1 : 0;
        y[i] = -(u[qn * ldc + c] + wn[q * ldc + c]);
    }
}

size_t pair_workspace_bytes(int32_t nt, int32_t nf, int32_t npix)
{
    if (nt < 1) return 0;
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t nq = (size_t)nt;
    return up(nq * npix * sizeof(float)) + up(nq * npix * sizeof(double)) + up(nq * nf * sizeof(float));
}

hipError_t launch_fisher_neighbours(const MapArgs &a, const float *u, const float *wn, const float *gamma,
                                    const double *tau, float *Gam, void *pair_ws, void *xm_ws, bool use_xm,
                                    hipStream_t s, const double **form_rec)
{
    const int32_t nq = a.nt;  // pairs (q, q + 1 mod nt)
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    char *p = reinterpret_cast<char *>(pair_ws);
    float *g2 = reinterpret_cast<float *>(p);
    p += up((size_t)nq * a.npix * sizeof(float));
    double *t2 = reinterpret_cast<double *>(p);
    p += up((size_t)nq * a.npix * sizeof(double));
    float *y = reinterpret_cast<float *>(p);

    const int64_t ns = (int64_t)nq * a.npix, nw = (int64_t)nq * a.nf;
    const unsigned gs = (unsigned)std::min<int64_t>((ns + 255) / 256, 65536);
    const unsigned gw = (unsigned)std::min<int64_t>((nw + 255) / 256, 65536);
    hipLaunchKernelGGL(pair_seeds_kernel, dim3(gs), dim3(256), 0, s, gamma, tau, ns, (int64_t)a.npix, g2, t2);
    hipLaunchKernelGGL(pair_weights_kernel, dim3(gw), dim3(256), 0, s, u, wn, a.ldc, nq, a.nf, y);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;

    MapArgs b = a;
    b.nt = nq;
    b.ldc = a.nf;
    b.unit_c = 1;
    b.accumulate = 1;
    // a pair delay is a difference of two delays: |tau'| <= 4 R / c.  Adjacent
    // segments of a full day keep it far smaller, but a partial day's wrap pair
    // (nt - 1, 0) or a short day can reach that bound, beyond what the
    // matrix-core forms cover at this df; the form record then selects the
    // vector-unit kernel, launched behind the matrix-core one and gated on it.
    b.tau_limit = 4.0 * kEarthRadius / kLightSpeed;
    if (!use_xm) return launch_dirty_map<float>(b, nullptr, y, g2, t2, Gam, s);
    const double *rec = nullptr;
    e = launch_dirty_map_mfma(b, nullptr, y, g2, t2, Gam, xm_ws, s, &rec);
    if (e != hipSuccess) return e;
    if (form_rec) *form_rec = rec;
    if (kTwoPi * 31.5 * b.df * b.tau_limit > kXmEtaMax) e = launch_dirty_map<float>(b, nullptr, y, g2, t2, Gam, s, rec);
    return e;
}

}  // namespace sgwb

// ORF seed matrices gamma(t,p), tau(t,p) (Sec. III.D, Fig. 3) on gfx950.
//
// One thread per (segment t, northern-half pixel q).  In float64 the thread
// finds the HEALPix centre of q, rotates it from the celestial frame into the
// Earth-fixed frame of sidereal time t_k (the inverse of the Earth's rotation,
// equivalent to rotating the detector tensors forward), and evaluates
//   gamma = sum_A F^A_a F^A_b = 2 tr(P Da P Db) - tr(P Da) tr(P Db),
//   P = I - n n^T (projector transverse to the direction n),
//   tau   = n . (x_a - x_b) / c.
// The antipode a(q) gets gamma and -tau, so the stored seeds are exactly
// antipodally symmetric.
#include "sgwb_internal.h"

namespace sgwb {

template <typename G>
__global__ __launch_bounds__(256) void geometry_kernel(GeomArgs a, G *__restrict__ gamma,
                                                        double *__restrict__ tau)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int t = blockIdx.y;
    const int64_t nhalf = a.npix / 2;
    if (q >= nhalf || t >= a.nt) return;

    const RingPos r = ring_of_north(q, a.nside);
    double nx, ny, nz;
    centre_north(r, a.nside, &nx, &ny, &nz);

    // Earth-fixed components of the celestial direction at sidereal angle th:
    // n_earth = R_z(-th) n.
    const double tk = a.t0 + (double)t * a.stride + a.half_dur;
    const double th = kTwoPi * tk / kSiderealDay;
    double s, c;
    sincos(th, &s, &c);
    const double ex = c * nx + s * ny;
    const double ey = -s * nx + c * ny;
    const double ez = nz;

    // u = Da n, v = Db n (symmetric tensors), alpha = n.Da.n, beta = n.Db.n
    const double *A = a.DA, *B = a.DB;
    const double ux = A[0] * ex + A[1] * ey + A[2] * ez;
    const double uy = A[3] * ex + A[4] * ey + A[5] * ez;
    const double uz = A[6] * ex + A[7] * ey + A[8] * ez;
    const double vx = B[0] * ex + B[1] * ey + B[2] * ez;
    const double vy = B[3] * ex + B[4] * ey + B[5] * ez;
    const double vz = B[6] * ex + B[7] * ey + B[8] * ez;
    const double alpha = ex * ux + ey * uy + ez * uz;
    const double beta = ex * vx + ey * vy + ez * vz;
    double trAB = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) trAB += A[i] * B[i];
    const double trA = A[0] + A[4] + A[8];
    const double trB = B[0] + B[4] + B[8];
    // tr(P Da P Db) = tr(Da Db) - 2 u.v + alpha beta ; tr(P D) = tr D - n.D.n
    const double tPAPB = trAB - 2.0 * (ux * vx + uy * vy + uz * vz) + alpha * beta;
    const double g = 2.0 * tPAPB - (trA - alpha) * (trB - beta);
    const double d = (ex * a.dx[0] + ey * a.dx[1] + ez * a.dx[2]) / kLightSpeed;

    const int64_t row = (int64_t)t * a.npix;
    const int64_t qa = antipode_north(r, a.npix);
    const G gv = (G)g;
    gamma[row + q] = gv;
    gamma[row + qa] = gv;
    tau[row + q] = d;
    tau[row + qa] = -d;
}

template <typename G>
hipError_t launch_geometry(const GeomArgs &a, G *gamma, double *tau, hipStream_t s)
{
    const int64_t nhalf = a.npix / 2;
    dim3 grid((unsigned)((nhalf + 255) / 256), (unsigned)a.nt);
    hipLaunchKernelGGL(geometry_kernel<G>, grid, dim3(256), 0, s, a, gamma, tau);
    return hipGetLastError();
}
template hipError_t launch_geometry<float>(const GeomArgs &, float *, double *, hipStream_t);
template hipError_t launch_geometry<double>(const GeomArgs &, double *, double *, hipStream_t);

__global__ __launch_bounds__(256) void centres_kernel(int64_t nside, double *__restrict__ xyz,
                                                      int32_t *__restrict__ anti)
{
    const int64_t npix = 12 * nside * nside;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= npix / 2) return;
    const RingPos r = ring_of_north(q, nside);
    const int64_t qa = antipode_north(r, npix);
    if (xyz) {
        double x, y, z;
        centre_north(r, nside, &x, &y, &z);
        xyz[3 * q] = x;
        xyz[3 * q + 1] = y;
        xyz[3 * q + 2] = z;
        xyz[3 * qa] = -x;
        xyz[3 * qa + 1] = -y;
        xyz[3 * qa + 2] = -z;
    }
    if (anti) {
        anti[q] = (int32_t)qa;
        anti[qa] = (int32_t)q;
    }
}

hipError_t launch_centres(int64_t nside, double *xyz, int32_t *anti, hipStream_t s)
{
    const int64_t nhalf = 6 * nside * nside;
    hipLaunchKernelGGL(centres_kernel, dim3((unsigned)((nhalf + 255) / 256)), dim3(256), 0, s, nside,
                       xyz, anti);
    return hipGetLastError();
}

}  // namespace sgwb

// Full Fisher information matrix of a band and the conjugate-gradient clean map
// (Eqs. eq_fisher, eq_ML_linear and its footnote; broadband H weighting of
// Sec. V), for weights of rank R, w(t,f) = sum_r a_r(t) b_r(f) (one pass per rank;
// the formulas below are one rank's):
//   G(p,q) = sum_{k in band} H_k sum_t w(t,k) gamma_p gamma_q cos 2 pi f_k (tau_p - tau_q)
//          = sum_t a_t gamma_p(t) gamma_q(t) W(tau_p(t) - tau_q(t)),
//   W(D)   = sum_{k in band} H_k b_k cos 2 pi f_k D.
// Route (not the paper's): the band sum is done once, in float64, into W and
// its derivative on a grid of delay differences D_j = j delta >= 0 (W is even)
// with 64 points per period of the band's highest frequency, up to 4 R / c, and
// from those into the cubic Hermite interpolant of each interval (relative
// error below (2 pi / 64)^4 / 384 = 2.4e-7 of sum |H b|).  Delays become 32-bit
// fixed-point table coordinates (17 fraction bits below 3 kHz), so a delay
// difference is an exact integer: its high bits pick the interval, its low
// bits the position in it, and (p,q) and (q,p) do the same arithmetic.
//
// Antipodal seeds (gamma(a(p)) = gamma(p), tau(a(p)) = -tau(p), a(p) the
// antipode) make the delays' fixed-point coordinates mirror exactly,
// U(a(p)) = 2^31 - U(p), and W is even, so the matrix has two distinct blocks
// over the northern pixels: G(p,q) = G(a(p),a(q)) with |U_p - U_q|, and
// G(p,a(q)) = G(q,a(p)) with |U_p - (2^31 - U_q)|.  Only the upper triangles of
// those two blocks are computed (half the table lookups of the whole upper
// triangle) and each value is written to its four places.
#include <cstdlib>
#include <cstring>

#include "fisher_general.h"

namespace sgwb {

constexpr int kFt = 64;      // matrix tile edge
constexpr int kFtSeg = 16;   // segments staged per step
constexpr int kFracBitsMax = 17;  // fixed-point fraction bits of a delay in table steps
constexpr int kFracBitsMin = 14;
constexpr uint32_t kDelayBias = 1u << 30;
constexpr uint32_t kDelayMirror = 2u * kDelayBias;  // U(a(p)) = kDelayMirror - U(p)
constexpr double kMaxDelay = 2.0 * kEarthRadius / kLightSpeed;  // |tau| bound on the Earth

// Table step, number of intervals J (|tau_p - tau_q| / delta < J - 1) and the
// fraction bits that keep |tau| / delta 2^fb + 2^30 inside 31 bits.
void fisher_table_geometry(double f_max, double *delta, int32_t *J, int32_t *fb)
{
    *delta = 1.0 / (64.0 * std::max(f_max, 1e-3));
    *J = (int32_t)std::ceil(2.0 * kMaxDelay / *delta) + 2;
    int32_t b = kFracBitsMax;
    while (b > 0 && (kMaxDelay / *delta + 1.0) * std::ldexp(1.0, b) >= (double)kDelayBias) --b;
    *fb = b;
}

// Delay bound of a seed set, for tables no longer than its delay differences
// need: max |tau| over all seeds (NaN counted as the Earth bound), as the bit
// pattern of a non-negative double (ordered like the value), reduced with an
// integer atomic max into *bound, which delay_bound_init_kernel zeroes first.
__global__ __launch_bounds__(64) void delay_bound_init_kernel(unsigned long long *__restrict__ bound)
{
    if (threadIdx.x == 0) *bound = 0ull;
}

__global__ __launch_bounds__(256) void delay_bound_kernel(const double *__restrict__ tau, int64_t n,
                                                          unsigned long long *__restrict__ bound)
{
    __shared__ double red[256];
    double m = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double v = tau[i];
        m = fmax(m, v != v ? kMaxDelay : fabs(v));
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(bound, (unsigned long long)__double_as_longlong(red[0]));
}

// Table intervals the seeds can reach: |tau_p - tau_q| <= 2 m with m their
// delay bound (clamped to the Earth bound, as the delays are), so an interval
// index (|U_p - U_q| >> fb, rounding included) stays <= ceil(2 m / delta) and
// ceil(2 m / delta) + 2 intervals suffice; J (the Earth bound's count) without
// a bound.
__device__ __forceinline__ int32_t table_intervals(const unsigned long long *__restrict__ bound, double delta,
                                                   int32_t J)
{
    if (!bound) return J;
    const double m = fmin(__longlong_as_double((long long)*bound), kMaxDelay);
    return min(J, (int32_t)ceil(2.0 * m / delta) + 2);
}

constexpr int kWaitVm0 = 0x0F70;  // s_waitcnt vmcnt(0), expcnt and lgkmcnt left at their maxima

// Pass 1, entry j <= J and one chunk of kTabChunk bins: the chunk's share of
// W(D_j) and delta dW/dD (D_j) in float64, D_j = j delta.  Phases are reduced
// in float64 at every 64th bin and advanced by a float64 rotation in between.
constexpr int kTabChunk = 2048;

__global__ __launch_bounds__(256) void delay_table_kernel(const float *__restrict__ H, const float *__restrict__ b,
                                                          int32_t clo, int32_t chi, double f0, double df, int64_t k0,
                                                          double delta, int32_t J, double2 *__restrict__ part)
{
    __shared__ double hb[kTabChunk], hbf[kTabChunk];
    const int32_t cb = clo + (int32_t)blockIdx.y * kTabChunk, ce = min(cb + kTabChunk, chi);
    for (int32_t c = cb + threadIdx.x; c < ce; c += 256) {
        const double h = (double)H[c] * (double)b[c];
        hb[c - cb] = h;
        hbf[c - cb] = h * kTwoPi * (f0 + (double)(k0 + c) * df);
    }
    __syncthreads();
    const int32_t j = blockIdx.x * 256 + threadIdx.x;
    if (j > J) return;
    const double D = (double)j * delta;
    double er, ei;
    sincospi(2.0 * df * D, &ei, &er);
    double sw = 0.0, sd = 0.0;
    for (int32_t c0 = cb; c0 < ce; c0 += 64) {
        const double fa = f0 + (double)(k0 + c0) * df;
        const double x = fa * D, r = x - rint(x);
        double zr, zi;
        sincospi(2.0 * r, &zi, &zr);
        const int32_t c1 = min(c0 + 64, ce);
        for (int32_t c = c0; c < c1; ++c) {
            sw += hb[c - cb] * zr;
            sd -= hbf[c - cb] * zi;
            const double nr = zr * er - zi * ei, ni = zr * ei + zi * er;
            zr = nr;
            zi = ni;
        }
    }
    part[(size_t)blockIdx.y * (J + 1) + j] = make_double2(sw, sd * delta);
}

// Cubic Hermite interpolant of W on [D_j, D_j+1] from (W, delta W') at both
// ends, written as a polynomial in x = 1 + s, s in [0, 1) the position inside
// the interval (x is what the assembly kernels build from the fraction bits).
__device__ __forceinline__ float4 hermite_cubic(double2 a, double2 b)
{
    // polynomial in s
    const double c0 = a.x, c1 = a.y, c2 = 3.0 * (b.x - a.x) - 2.0 * a.y - b.y, c3 = 2.0 * (a.x - b.x) + a.y + b.y;
    // re-expanded around s = x - 1
    return make_float4((float)(c0 - c1 + c2 - c3), (float)(c1 - 2.0 * c2 + 3.0 * c3), (float)(c2 - 3.0 * c3),
                       (float)c3);
}

// Pass 2, interval j < J: the chunk sums at both ends (chunk order fixed),
// then the interval's cubic.
__global__ __launch_bounds__(256) void delay_cubic_kernel(const double2 *__restrict__ part, int32_t nchunk, int32_t J,
                                                          float4 *__restrict__ cub)
{
    const int32_t j = blockIdx.x * 256 + threadIdx.x;
    if (j >= J) return;
    double2 a = make_double2(0.0, 0.0), b = a;
    for (int32_t q = 0; q < nchunk; ++q) {
        const double2 u = part[(size_t)q * (J + 1) + j], v = part[(size_t)q * (J + 1) + j + 1];
        a.x += u.x;
        a.y += u.y;
        b.x += v.x;
        b.y += v.y;
    }
    cub[j] = hermite_cubic(a, b);
}

// General weights (any w(t,c), not a sum of a few products): one table per
// segment,
//   Wd_t(D_j) = sum_{c in band} H_c w(t,c) cos 2 pi f_c D_j,   delta Wd_t'(D_j),
// for every segment t and grid point j <= Jv (the points the seeds' delay
// bound can reach) at once.  That is a dense contraction, run on the float64
// matrix cores (v_mfma_f64_16x16x4), in one of two bases:
//  * direct: over the band's bins, [nt x nbins] . [nbins x (Jv + 1)], twice
//    (cosine and sine), the weight operand H_c w(t,c) (and -2 pi delta f_c
//    times it for the derivative) built in registers from w;
//  * expanded: per strip of S bins (S >= 16, aligned to the absolute grid, f_c
//    = f_s + s_c (S - 1) df / 2 with f_s the strip centre, s_c in [-1, 1]),
//    the Jacobi-Anger expansion e^{i s eta} = sum_n eps_n i^n J_n(eta) T_n(s),
//    eta = pi (S - 1) df D, turns the band sum into one over (strip, term):
//      Wd_t(D) = sum_{s,n} mu_n(t,s) eps_n J_n(eta) Re[i^n e^{2 pi i f_s D}],
//      delta Wd_t'(D) = -2 pi delta sum_{s,n} nu_n(t,s) eps_n J_n(eta) Im[i^n e^{2 pi i f_s D}],
//    mu_n = sum_{c in s} H_c w(t,c) T_n(s_c), nu_n the same with H_c w(t,c) f_c
//    (table_moments_kernel): kTxTerms terms per strip instead of S bins.  S is
//    the widest power of two up to 64 with eta <= kTxEtaMax at the Earth bound
//    (S = 64 at 1/32 Hz), so the dropped remainder is below 2 (eta/2)^8 / 8! =
//    1.6e-9 of sum |H w|.
// Per work item a 64-segment x 64-point tile over one range of K (bins, or
// strip terms), the cosine / sine operand of each 32-deep chunk generated into
// LDS (float64 phases reduced exactly, then advanced by float64 rotations; the
// Bessel factors once per item), the other operand read per lane.  Workgroups
// walk the items persistently; K splits into as many ranges as fill the chip
// (their count, like Jv, is worked out on the device), whose float64 partial
// sums delay_cubic_general_kernel adds in a fixed order.
typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int kTgM = 64;          // segments per tile (16 per wave)
constexpr int kTgN = 64;          // grid points per tile (four 16-wide blocks)
constexpr int kTgK = 32;          // K per chunk (eight 4-deep matrix-core steps)
constexpr int kTgSplitsMax = 16;  // K ranges at most
constexpr int kTgSplitsBuf = 4;   // partial sums held: kTgSplitsBuf x nt x (J + 1) points
constexpr int kTgItems = 8192;    // work items aimed at
constexpr int kTxTerms = 8;       // Jacobi-Anger terms per strip (expanded basis)
constexpr double kTxEtaMax = 0.55;
static_assert(kTgK % kTxTerms == 0, "a chunk holds whole strips");

struct TableSplit {
    int32_t n;     // K ranges
    int32_t bins;  // K per range (a multiple of kTgK)
};

// Partial-sum buffer of the table contraction, in tables of J + 1 points per
// segment: kTgSplitsBuf, fewer for K of under 16 chunks a range.
__host__ __device__ __forceinline__ int32_t table_split_cap(int32_t nk)
{
    const int32_t c = ((nk + kTgK - 1) / kTgK) / 16;
    return c < 1 ? 1 : (c < kTgSplitsBuf ? c : kTgSplitsBuf);
}

// K ranges for a table of Jv intervals: about kTgItems work items, at least
// 16 chunks a range (unless there is one range), at most kTgSplitsMax, and no
// more partial sums than the buffer holds (n (Jv + 1) <= cap (J + 1)).
__host__ __device__ __forceinline__ TableSplit table_split(int32_t Jv, int32_t J, int32_t nt, int32_t nk)
{
    const int64_t tiles = (int64_t)((Jv + 1 + kTgN - 1) / kTgN) * ((nt + kTgM - 1) / kTgM);
    const int32_t nchunk = (nk + kTgK - 1) / kTgK;
    int64_t n = (kTgItems + tiles - 1) / tiles;
    n = n < nchunk / 16 ? n : nchunk / 16;
    const int64_t fit = (int64_t)table_split_cap(nk) * (J + 1) / (Jv + 1);
    n = n < fit ? n : fit;
    n = n < kTgSplitsMax ? n : kTgSplitsMax;
    n = n > 1 ? n : 1;
    TableSplit r;
    r.bins = (int32_t)((nchunk + n - 1) / n) * kTgK;
    r.n = (nk + r.bins - 1) / r.bins;
    return r;
}

// Strips of the expanded basis: S bins each (0: use the direct basis), the
// first strip's index (absolute bins first S ..) and the count touching the band.
struct StripGrid {
    int32_t S = 0;
    int64_t first = 0;
    int32_t n = 0;
};

static StripGrid strip_grid(double df, int64_t k0, int32_t clo, int32_t chi)
{
    StripGrid g;
    int32_t S = 64;
    while (S >= 16 && kTwoPi * 0.5 * (S - 1) * df * 2.0 * kMaxDelay > kTxEtaMax) S >>= 1;
    if (S < 16) return g;  // eight terms per strip would not save work
    g.S = S;
    const int64_t a = k0 + clo, b = k0 + chi - 1;
    g.first = a / S;
    g.n = (int32_t)(b / S - g.first + 1);
    return g;
}

// Strip moments: mu_n(t,s) = sum over the strip's band bins of H_c w(t,c)
// T_n(s_c), nu_n(t,s) the same with H_c w(t,c) f_c; [nt][nstrips kTxTerms]
// float64, T_n by the three-term recurrence.  A 256-thread workgroup takes 64
// strips of one segment: their H w (float64, zero outside the band) come into
// LDS with coalesced loads (rows padded by one word against bank conflicts);
// four threads share a strip, a quarter of its bins each, and their partial
// moments are added in a fixed order.
constexpr int kTxStrips = 64;  // strips per workgroup
constexpr int kTxSplit = 4;    // threads per strip

__global__ __launch_bounds__(256) void table_moments_kernel(const float *__restrict__ w, int64_t ldw,
                                                            const float *__restrict__ H, int32_t clo, int32_t chi,
                                                            double f0, double df, int64_t k0, int32_t S,
                                                            int64_t first, int32_t nstrips, double *__restrict__ mu,
                                                            double *__restrict__ nu)
{
    __shared__ double hw[kTxStrips][64 + 1];
    __shared__ double red[kTxSplit - 1][kTxStrips][2 * kTxTerms];
    const int32_t s0 = blockIdx.x * kTxStrips;
    const int32_t t = blockIdx.y;
    const float *wr = w + (int64_t)t * ldw;
    const int64_t kb0 = (first + s0) * S;  // absolute first bin of the workgroup's first strip
    const int32_t nsg = min(kTxStrips, nstrips - s0);
    for (int32_t e = threadIdx.x; e < nsg * S; e += 256) {
        const int64_t c = kb0 + e - k0;  // column
        hw[e / S][e % S] = c >= clo && c < chi ? (double)H[c] * (double)wr[c] : 0.0;
    }
    __syncthreads();
    const int ls = threadIdx.x % kTxStrips, part = threadIdx.x / kTxStrips;  // strip, quarter
    const int32_t sg = s0 + ls;
    const bool ok = sg < nstrips;
    const int64_t kb = kb0 + (int64_t)ls * S;
    const double half = 0.5 * (S - 1);
    const int32_t q = S / kTxSplit, i0 = part * q;
    double m[kTxTerms], v[kTxTerms];
#pragma unroll
    for (int n = 0; n < kTxTerms; ++n) m[n] = v[n] = 0.0;
    for (int32_t i = i0; ok && i < i0 + q; ++i) {
        const double h = hw[ls][i];
        const double hf = h * (f0 + (double)(kb + i) * df);
        const double s = ((double)i - half) / half;
        double tp = 1.0, tc = s;  // T_0, T_1
        m[0] += h;
        v[0] += hf;
        m[1] += h * s;
        v[1] += hf * s;
#pragma unroll
        for (int n = 2; n < kTxTerms; ++n) {
            const double tn = 2.0 * s * tc - tp;
            tp = tc;
            tc = tn;
            m[n] += h * tn;
            v[n] += hf * tn;
        }
    }
    if (part > 0) {
#pragma unroll
        for (int n = 0; n < kTxTerms; ++n) {
            red[part - 1][ls][n] = m[n];
            red[part - 1][ls][kTxTerms + n] = v[n];
        }
    }
    __syncthreads();
    if (part > 0 || !ok) return;
#pragma unroll
    for (int r = 0; r < kTxSplit - 1; ++r)
#pragma unroll
        for (int n = 0; n < kTxTerms; ++n) {
            m[n] += red[r][ls][n];
            v[n] += red[r][ls][kTxTerms + n];
        }
    const int64_t nk = (int64_t)nstrips * kTxTerms;
    double *mr = mu + (int64_t)t * nk + (int64_t)sg * kTxTerms, *vr = nu + (int64_t)t * nk + (int64_t)sg * kTxTerms;
#pragma unroll
    for (int n = 0; n < kTxTerms; ++n) {
        mr[n] = m[n];
        vr[n] = v[n];
    }
}

// eps_n J_n(eta) for n < kTxTerms (power series; eta <= kTxEtaMax, 12 terms
// leave less than 1e-17).
__device__ __forceinline__ void bessel_eps(double eta, double (&J)[kTxTerms])
{
    const double x = 0.5 * eta, x2 = -x * x;
    double lead = 1.0;  // x^n / n!
#pragma unroll
    for (int n = 0; n < kTxTerms; ++n) {
        double term = lead, sum = lead;
#pragma unroll
        for (int k = 1; k <= 12; ++k) {
            term *= x2 / (double)(k * (n + k));
            sum += term;
        }
        J[n] = n == 0 ? sum : 2.0 * sum;
        lead *= x / (double)(n + 1);
    }
}

// EXP = false: A = w, H (direct basis over the bins; nk = nbins); EXP = true:
// A = mu, nu (strip moments, nk = nstrips kTxTerms).
template <bool EXP>
__global__ __launch_bounds__(256) void delay_table_gemm_kernel(const float *__restrict__ w, int64_t ldw,
                                                               const float *__restrict__ H,
                                                               const double *__restrict__ mu,
                                                               const double *__restrict__ nu, int32_t nt,
                                                               int32_t clo, int32_t nk, double f0, double df,
                                                               int64_t k0, int32_t S, int64_t first, double delta,
                                                               int32_t J, const unsigned long long *__restrict__ bound,
                                                               double2 *__restrict__ part)
{
    __shared__ double bc[kTgK][kTgN], bs[kTgK][kTgN];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int kq = lane >> 4;
    const int gj = threadIdx.x & 63, gg = threadIdx.x >> 6;  // generation: point gj, K rows 8 gg .. 8 gg + 7
    const int32_t Jv = table_intervals(bound, delta, J);
    const TableSplit sp = table_split(Jv, J, nt, nk);
    const int32_t nx = (Jv + 1 + kTgN - 1) / kTgN, ny = (nt + kTgM - 1) / kTgM;
    const int64_t items = (int64_t)nx * ny * sp.n;
    const float *hr = H + clo;
    const double half = 0.5 * (S - 1);
    for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
        const int32_t bx = (int32_t)(it % nx);
        const int64_t rest = it / nx;
        const int32_t by = (int32_t)(rest % ny), bz = (int32_t)(rest / ny);
        const int32_t j0 = bx * kTgN, t0 = by * kTgM;
        const int32_t cbeg = bz * sp.bins, cend = min(nk, cbeg + sp.bins);
        const double D = (double)(j0 + gj) * delta;
        double er, ei, Jn[kTxTerms];
        if (EXP) {
            bessel_eps(kTwoPi * half * df * D, Jn);
        } else {
            sincospi(2.0 * df * D, &ei, &er);
        }
        // operand from memory: segment t0 + 16 wv + lane % 16, K index c0 + 4 ks + lane / 16
        const int32_t trow = t0 + 16 * wv + (lane & 15);
        const bool rok = trow < nt;
        const float *wr = w + (int64_t)(rok ? trow : 0) * ldw + clo;
        const double *mr = EXP ? mu + (int64_t)(rok ? trow : 0) * nk : nullptr;
        const double *vr = EXP ? nu + (int64_t)(rok ? trow : 0) * nk : nullptr;
        dbl4 av[4], ad[4];
#pragma unroll
        for (int n = 0; n < 4; ++n) av[n] = ad[n] = dbl4{0.0, 0.0, 0.0, 0.0};
        for (int32_t c0 = cbeg; c0 < cend; c0 += kTgK) {
            // this chunk's operand values first, so their loads overlap the generation
            double ak[kTgK / 4], dk[kTgK / 4];
#pragma unroll
            for (int ks = 0; ks < kTgK / 4; ++ks) {
                const int32_t c = c0 + 4 * ks + kq;
                const bool ok = rok && c < cend;
                if (EXP) {
                    ak[ks] = ok ? mr[c] : 0.0;
                    dk[ks] = ok ? vr[c] : 0.0;
                } else {
                    const double h = ok ? (double)hr[c] * (double)wr[c] : 0.0;
                    ak[ks] = h;
                    dk[ks] = -kTwoPi * delta * (f0 + (double)(k0 + clo + c) * df) * h;
                }
            }
            __syncthreads();  // the previous chunk's (or item's) operands are no longer read
            if (EXP) {
                // strip c0 / kTxTerms + gg, its kTxTerms terms
                const int64_t sgi = first + c0 / kTxTerms + gg;
                const double x = (f0 + ((double)(sgi * S) + half) * df) * D, r = x - rint(x);
                double zr, zi;
                sincospi(2.0 * r, &zi, &zr);
                const double sd = -kTwoPi * delta;
#pragma unroll
                for (int n = 0; n < kTxTerms; ++n) {
                    // i^n e^{i theta}: real and imaginary parts
                    const double re = (n & 3) == 0 ? zr : (n & 3) == 1 ? -zi : (n & 3) == 2 ? -zr : zi;
                    const double im = (n & 3) == 0 ? zi : (n & 3) == 1 ? zr : (n & 3) == 2 ? -zi : -zr;
                    bc[8 * gg + n][gj] = Jn[n] * re;
                    bs[8 * gg + n][gj] = sd * Jn[n] * im;
                }
            } else {
                const int32_t cs = c0 + 8 * gg;
                const double x = (f0 + (double)(k0 + clo + cs) * df) * D, r = x - rint(x);
                double zr, zi;
                sincospi(2.0 * r, &zi, &zr);
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    bc[8 * gg + i][gj] = zr;
                    bs[8 * gg + i][gj] = zi;
                    const double nr = zr * er - zi * ei, ni = zr * ei + zi * er;
                    zr = nr;
                    zi = ni;
                }
            }
            __syncthreads();
#pragma unroll
            for (int ks = 0; ks < kTgK / 4; ++ks) {
#pragma unroll
                for (int n = 0; n < 4; ++n) {
                    const double b1 = bc[4 * ks + kq][16 * n + (lane & 15)];
                    const double b2 = bs[4 * ks + kq][16 * n + (lane & 15)];
                    av[n] = __builtin_amdgcn_mfma_f64_16x16x4f64(ak[ks], b1, av[n], 0, 0, 0);
                    ad[n] = __builtin_amdgcn_mfma_f64_16x16x4f64(dk[ks], b2, ad[n], 0, 0, 0);
                }
            }
        }
        // result layout (measured): register r of a lane holds row lane / 16 + 4 r
        // of the wave's 16, column lane % 16 of each block; partial sums of range
        // bz at part + (bz nt + t) (Jv + 1) + j
#pragma unroll
        for (int n = 0; n < 4; ++n)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int32_t t = t0 + 16 * wv + kq + 4 * r, j = j0 + 16 * n + (lane & 15);
                if (t < nt && j <= Jv)
                    part[((size_t)bz * nt + t) * (Jv + 1) + j] = make_double2(av[n][r], ad[n][r]);
            }
    }
}

// Cubic of interval j < Jv of segment blockIdx.y's table, from the bin ranges'
// partial sums (range order fixed).  Tables are stored back to back, Jv
// intervals each (segment t's at cub + t Jv).
__global__ __launch_bounds__(256) void delay_cubic_general_kernel(const double2 *__restrict__ part, int32_t nt,
                                                                  int32_t nk, int32_t J,
                                                                  const unsigned long long *__restrict__ bound,
                                                                  double delta, float4 *__restrict__ cub)
{
    const int32_t j = blockIdx.x * 256 + threadIdx.x;
    const int32_t Jv = table_intervals(bound, delta, J);
    if (j >= Jv) return;
    const TableSplit sp = table_split(Jv, J, nt, nk);
    const size_t stride = (size_t)nt * (Jv + 1);
    part += (size_t)blockIdx.y * (Jv + 1);
    double2 a = make_double2(0.0, 0.0), b = a;
    for (int32_t q = 0; q < sp.n; ++q) {
        const double2 u = part[q * stride + j], v = part[q * stride + j + 1];
        a.x += u.x;
        a.y += u.y;
        b.x += v.x;
        b.y += v.y;
    }
    cub[(size_t)blockIdx.y * Jv + j] = hermite_cubic(a, b);
}

// Delays as biased fixed-point table coordinates: U = round(tau / delta 2^fb) + 2^30,
// tau clamped to the Earth bound, so that |U_p - U_q| >> fb < J - 1.
__global__ __launch_bounds__(256) void fixed_delay_kernel(const double *__restrict__ tau, int64_t n, double scale,
                                                          uint32_t *__restrict__ U)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double t = fmin(fmax(tau[i], -kMaxDelay), kMaxDelay);
    U[i] = (uint32_t)((int64_t)llrint(t * scale) + (int64_t)kDelayBias);
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

// G(p,q) and G(q,p) (once on the diagonal), overwritten or added to (the
// terms of a further rank of the weights).
__device__ __forceinline__ void store_pair(float *__restrict__ G, int64_t npix, int64_t p, int64_t q, float v,
                                           int32_t accumulate)
{
    float *e = G + p * npix + q;
    *e = accumulate ? *e + v : v;
    if (p != q) {
        float *m = G + q * npix + p;
        *m = accumulate ? *m + v : v;
    }
}

// Tile k of the computed triangles: with antipodal seeds (nside > 0) tiles
// [0, half) are the northern block's upper triangle and [half, 2 half) the
// northern x southern block's (columns mirrored, ns = true).
__device__ __forceinline__ void fisher_tile(int64_t k, int64_t nT, bool anti, int64_t &tr, int64_t &tc, bool &ns)
{
    const int64_t half = nT * (nT + 1) / 2;
    ns = anti && k >= half;
    tri_tile(ns ? k - half : k, nT, tr, tc);
}

// Matrix entries of the value computed for the pair (p, q), p <= q, of a tile:
// plain (p,q) and its mirror; antipodal also the antipodes' pair
// (northern block) or the mirrored-column pairs (p,a(q)) and (q,a(p)).
__device__ __forceinline__ void store_value(float *__restrict__ G, int64_t npix, int64_t nside, bool ns, int64_t p,
                                            int64_t q, float v, int32_t accumulate)
{
    if (nside == 0) {
        store_pair(G, npix, p, q, v, accumulate);
        return;
    }
    const int64_t ap = antipode_north(ring_of_north(p, nside), npix);
    const int64_t aq = antipode_north(ring_of_north(q, nside), npix);
    if (!ns) {
        store_pair(G, npix, p, q, v, accumulate);
        store_pair(G, npix, ap, aq, v, accumulate);
    } else {
        store_pair(G, npix, p, aq, v, accumulate);
        if (p != q) store_pair(G, npix, q, ap, v, accumulate);
    }
}

// Seeds failed the antipodal spot check (any of the kSymParts flags set).
__device__ __forceinline__ bool seeds_rejected(const double *__restrict__ flags)
{
    if (!flags) return false;
    bool bad = false;
    for (int i = 0; i < kSymParts; ++i) bad = bad || flags[i] != 0.0;
    return bad;
}

__device__ __forceinline__ uint32_t abs_diff(uint32_t x, uint32_t y)
{
    uint32_t d;
    asm("v_sad_u32 %0, %1, %2, 0" : "=v"(d) : "v"(x), "v"(y));
    return d;
}

// G tile (r, c) of the upper triangle; 256 threads, 4 x 4 entries each.  Per
// (t, p, q): |U_p - U_q| gives the table interval (high bits) and the position
// in it (low fb bits, placed in the mantissa of x in [1, 2)); three FMAs
// evaluate the cubic, two more weight and accumulate it.  With weights a[t],
// one table for all segments; with a null, one table per segment, Jv
// intervals each, back to back (Jv from the seeds' delay bound).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 4))) void fisher_full_kernel(const float *__restrict__ a, const float *__restrict__ gamma,
                                                          const uint32_t *__restrict__ U, int32_t nt, int32_t npix,
                                                          int64_t nside, const double *__restrict__ flags,
                                                          const float4 *__restrict__ cub, int32_t J,
                                                          const unsigned long long *__restrict__ bound,
                                                          double delta, int32_t fb, int32_t accumulate,
                                                          float *__restrict__ G)
{
    const int64_t seg_stride = a ? 0 : table_intervals(bound, delta, J);
    __shared__ float gP[kFtSeg][kFt], gQ[kFtSeg][kFt];
    __shared__ uint32_t uP[kFtSeg][kFt], uQ[kFtSeg][kFt];
    const int64_t nrow = nside > 0 ? npix / 2 : npix;  // rows and columns of the computed blocks
    const int64_t nT = (nrow + kFt - 1) / kFt;
    int64_t tr, tc;
    bool ns;
    fisher_tile(blockIdx.x, nT, nside > 0, tr, tc, ns);
    const int ty = threadIdx.x / 16, tx = threadIdx.x % 16;
    float acc[4][4] = {};
    const char *cb = reinterpret_cast<const char *>(cub);
    const int ntu = seeds_rejected(flags) ? 0 : nt;
    for (int t0 = 0; t0 < ntu; t0 += kFtSeg) {
        __syncthreads();
        for (int e = threadIdx.x; e < kFtSeg * kFt; e += 256) {
            const int tt = e / kFt, i = e % kFt, t = t0 + tt;
            const int64_t p = tr * kFt + i, q = tc * kFt + i;
            const bool ok = t < nt;
            const float at = ok ? (a ? a[t] : 1.0f) : 0.0f;
            gP[tt][i] = ok && p < nrow ? at * gamma[(int64_t)t * npix + p] : 0.0f;
            uP[tt][i] = ok && p < nrow ? U[(int64_t)t * npix + p] : kDelayBias;
            gQ[tt][i] = ok && q < nrow ? gamma[(int64_t)t * npix + q] : 0.0f;
            const uint32_t uq = ok && q < nrow ? U[(int64_t)t * npix + q] : kDelayBias;
            uQ[tt][i] = ns ? kDelayMirror - uq : uq;
        }
        __syncthreads();
        const int tn = min(kFtSeg, nt - t0);
        for (int tt = 0; tt < tn; ++tt) {
            const char *ct = cb + (size_t)(t0 + tt) * seg_stride * sizeof(float4);
            float gp[4], gq[4];
            uint32_t up[4], uq[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                gp[i] = gP[tt][ty * 4 + i];
                up[i] = uP[tt][ty * 4 + i];
                gq[i] = gQ[tt][tx * 4 + i];
                uq[i] = uQ[tt][tx * 4 + i];
            }
            // all sixteen table reads in flight before the first is used
            float4 c[4][4];
            float x[4][4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const uint32_t d = abs_diff(up[i], uq[jj]);
                    c[i][jj] = *reinterpret_cast<const float4 *>(ct + ((size_t)(d >> fb) << 4));
                    x[i][jj] = __uint_as_float(((d << (23 - fb)) & 0x007fffffu) | 0x3f800000u);
                }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const float4 cc = c[i][jj];
                    const float W = fmaf(fmaf(fmaf(cc.w, x[i][jj], cc.z), x[i][jj], cc.y), x[i][jj], cc.x);
                    acc[i][jj] = fmaf(gp[i] * gq[jj], W, acc[i][jj]);
                }
        }
    }
    if (ntu != nt) {  // rejected seeds: the matrix is NaN
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) acc[i][jj] = __builtin_nanf("");
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int64_t p = tr * kFt + ty * 4 + i, q = tc * kFt + tx * 4 + jj;
            // a diagonal tile writes its upper triangle and the mirror of it
            if (p < nrow && q < nrow && (tr != tc || p <= q))
                store_value(G, npix, nside, ns, p, q, acc[i][jj], accumulate);
        }
}

// LDS-resident form: one 512-thread workgroup per compute unit copies the
// whole cubic table into LDS (up to 10240 intervals = 160 KiB, enough for
// bands up to 1.88 kHz) and then walks the upper-triangle tiles persistently,
// two at a time (one per 256-thread half, halves independent).  Inputs come
// from global memory into registers one segment ahead.
constexpr int kLdsTable = 10240;

__global__ __launch_bounds__(512) void fisher_full_lds_kernel(const float *__restrict__ a,
                                                               const float *__restrict__ gamma,
                                                               const uint32_t *__restrict__ U, int32_t nt,
                                                               int32_t npix, int64_t nside,
                                                               const double *__restrict__ flags,
                                                               const float4 *__restrict__ cub,
                                                               int32_t J, int32_t fb, int64_t ntiles,
                                                               int32_t accumulate, float *__restrict__ G)
{
    __shared__ float4 tab[kLdsTable];
    for (int j = threadIdx.x; j < J; j += 512) tab[j] = cub[j];
    __syncthreads();
    const char *tb = reinterpret_cast<const char *>(tab);
    const int half = threadIdx.x >> 8, lt = threadIdx.x & 255;
    const int ty = lt / 16, tx = lt % 16;
    const int64_t nrow = nside > 0 ? npix / 2 : npix;  // rows and columns of the computed blocks
    const int32_t last = (int32_t)nrow - 1;
    const int64_t nT = (nrow + kFt - 1) / kFt;
    const int ntu = seeds_rejected(flags) ? 0 : nt;
    for (int64_t k = (int64_t)blockIdx.x * 2 + half; k < ntiles; k += (int64_t)gridDim.x * 2) {
        int64_t tr, tc;
        bool ns;
        fisher_tile(k, nT, nside > 0, tr, tc, ns);
        // the mirrored columns of the northern x southern block: U(a(q)) = kDelayMirror - U(q)
        const uint32_t qm = ns ? kDelayMirror : 0u, qs = ns ? 0u : 1u;
        auto ucol = [qm, qs](uint32_t u) { return qs ? u : qm - u; };
        int32_t pi[4], qi[4];
        bool pv[4], qv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t p = tr * kFt + ty * 4 + i, q = tc * kFt + tx * 4 + i;
            pv[i] = p < nrow;
            qv[i] = q < nrow;
            pi[i] = (int32_t)(pv[i] ? p : last);
            qi[i] = (int32_t)(qv[i] ? q : last);
        }
        float acc[4][4] = {};
        float gp[4], gq[4];
        uint32_t up[4], uq[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            gp[i] = pv[i] ? a[0] * gamma[pi[i]] : 0.0f;
            up[i] = U[pi[i]];
            gq[i] = qv[i] ? gamma[qi[i]] : 0.0f;
            uq[i] = ucol(U[qi[i]]);
        }
        for (int t = 0; t < ntu; ++t) {
            // next segment's inputs (the last iteration re-reads segment nt - 1)
            const int tn = min(t + 1, nt - 1);
            const int64_t o = (int64_t)tn * npix;
            const float an = a[tn];
            float gpn[4], gqn[4];
            uint32_t upn[4], uqn[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                gpn[i] = gamma[o + pi[i]];
                upn[i] = U[o + pi[i]];
                gqn[i] = gamma[o + qi[i]];
                uqn[i] = U[o + qi[i]];
            }
            float4 c[4][4];
            float x[4][4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const uint32_t d = abs_diff(up[i], uq[jj]);
                    c[i][jj] = *reinterpret_cast<const float4 *>(tb + ((d >> fb) << 4));
                    x[i][jj] = __uint_as_float(((d << (23 - fb)) & 0x007fffffu) | 0x3f800000u);
                }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const float4 cc = c[i][jj];
                    const float W = fmaf(fmaf(fmaf(cc.w, x[i][jj], cc.z), x[i][jj], cc.y), x[i][jj], cc.x);
                    acc[i][jj] = fmaf(gp[i] * gq[jj], W, acc[i][jj]);
                }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                gp[i] = pv[i] ? an * gpn[i] : 0.0f;
                up[i] = upn[i];
                gq[i] = qv[i] ? gqn[i] : 0.0f;
                uq[i] = ucol(uqn[i]);
            }
        }
        if (ntu != nt) {  // rejected seeds: the matrix is NaN
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) acc[i][jj] = __builtin_nanf("");
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const int64_t p = tr * kFt + ty * 4 + i, q = tc * kFt + tx * 4 + jj;
                if (pv[i] && q < nrow && (tr != tc || p <= q))
                    store_value(G, npix, nside, ns, p, q, acc[i][jj], accumulate);
            }
    }
}

// General weights, streaming form: each workgroup owns kStTiles consecutive
// tiles of the walk (two waves a tile, one per 32-column half; lane (ty, tx)
// of a wave the 8 x 4 entries rows 8 ty.., columns 4 tx.. of its half), keeps
// their sums in registers over every segment and streams the segments'
// tables through LDS, copied straight from global memory (global_load_lds, 16
// bytes a lane), a stage of as many segments as fit at a time.  Stages of
// tables up to kLdsTable / 2 intervals are double-buffered (stage s + 1 lands
// while stage s is read); longer tables take turns in one buffer.  Only the
// first Jv intervals of each table are copied: those the seeds' delay bound
// can reach.  Same term arithmetic as the other forms, so the same bits in the
// same segment order.
constexpr int kStTiles = 4;
constexpr int kStWaves = 2 * kStTiles;  // 512 threads

// n float4 from src into LDS at dst, 16 bytes a lane straight from global
// memory; lane l of a wave writes the l-th 16 bytes after the wave's base.
__device__ __forceinline__ void copy_lds(const float4 *__restrict__ src, float4 *dst, int32_t n)
{
    const int lane = threadIdx.x & 63;
    const char *base = reinterpret_cast<const char *>(src);
    for (int32_t e = threadIdx.x; e < n; e += kStWaves * 64)
        __builtin_amdgcn_global_load_lds(base + (size_t)e * sizeof(float4), dst + (e - lane), 16, 0, 0);
}

// kLdsTable / 2 float4 into LDS at dst (a half-size buffer), the first n of
// them from src: a fixed number of copy instructions per lane (lanes past n
// copy src[n - 1] into the buffer's unused tail), so the compiler can count
// them and wait for earlier loads without waiting for the copy.
__device__ __forceinline__ void copy_lds_half(const float4 *__restrict__ src, float4 *dst, int32_t n)
{
    const int lane = threadIdx.x & 63;
    const char *base = reinterpret_cast<const char *>(src);
#pragma unroll
    for (int r = 0; r < kLdsTable / 2 / (kStWaves * 64); ++r) {
        const int32_t e = r * kStWaves * 64 + (int32_t)threadIdx.x;
        __builtin_amdgcn_global_load_lds(base + (size_t)min(e, n - 1) * sizeof(float4), dst + (e - lane), 16, 0,
                                         0);
    }
}
static_assert((kLdsTable / 2) % (kStWaves * 64) == 0, "whole copy rounds");

// Buffer resource over one segment's npix 4-byte seeds (raw loads at byte
// offsets; out-of-range offsets read 0).  0x00020000: the gfx9 descriptor word
// for plain 32-bit raw access.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t seg_rsrc(const void *p, int32_t npix)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, npix * 4, 0x00020000);
}

// ONE = true: one table for every segment (weights a of rank-one terms),
// copied once, the segment's weight a[t] on the row seeds; accumulate adds to
// G (the later ranks).  ONE = false: per-segment tables streamed as above.
// The two stage buffers are distinct LDS arrays, and the stage loop is
// unrolled by two so that each step reads one and copies into the other by
// name: the compiler then orders the reads only after copies into the same
// array (with one array it waits for every copy before every read).  Tables
// longer than one buffer (single-buffered) span both arrays.
template <bool ONE>
__global__ __launch_bounds__(512) void fisher_full_stream_kernel(const float *__restrict__ a,
                                                                 const float *__restrict__ gamma,
                                                                 const uint32_t *__restrict__ U, int32_t nt,
                                                                 int32_t npix, int64_t nside,
                                                                 const double *__restrict__ flags,
                                                                 const float4 *__restrict__ cub, int32_t J,
                                                                 const unsigned long long *__restrict__ bound,
                                                                 double delta, int32_t fb, int64_t ntiles,
                                                                 int32_t accumulate, float *__restrict__ G)
{
    constexpr int32_t kHalf = kLdsTable / 2;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int ty = lane >> 3, tx = lane & 7;
    const int64_t nrow = nside > 0 ? npix / 2 : npix;
    const int64_t last_row = nrow - 1;
    const int64_t nT = (nrow + kFt - 1) / kFt;
    const int64_t k = (int64_t)blockIdx.x * kStTiles + (wv >> 1);
    const bool active = k < ntiles;
    int64_t tr = 0, tc = 0;
    bool ns = false;
    if (active) fisher_tile(k, nT, nside > 0, tr, tc, ns);
    const uint32_t qm = ns ? kDelayMirror : 0u, qs = ns ? 0u : 1u;
    auto ucol = [qm, qs](uint32_t u) { return qs ? u : qm - u; };
    const int64_t p0 = tr * kFt + ty * 8, q0 = tc * kFt + (wv & 1) * 32 + tx * 4;
    // byte offsets of the lane's rows and columns within a segment's seeds
    // (clamped into the matrix: entries past it are computed but never stored,
    // as are those of an idle wave)
    uint32_t po[8], qo[4];
#pragma unroll
    for (int i = 0; i < 8; ++i) po[i] = (uint32_t)min(p0 + i, last_row) * 4u;
#pragma unroll
    for (int j = 0; j < 4; ++j) qo[j] = (uint32_t)min(q0 + j, last_row) * 4u;
    const int32_t Jv = table_intervals(bound, delta, J);
    const bool rejected = seeds_rejected(flags);
    const int32_t ntu = rejected ? 0 : nt;
    float acc[8][4] = {};
    float gp[8], gq[4];
    uint32_t up[8], uq[4];
    {
        const __amdgpu_buffer_rsrc_t rg = seg_rsrc(gamma, npix), ru = seg_rsrc(U, npix);
        const float a0 = ONE ? a[0] : 1.0f;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            gp[i] = a0 * __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rg, po[i], 0, 0));
            up[i] = __builtin_amdgcn_raw_buffer_load_b32(ru, po[i], 0, 0);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            gq[j] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rg, qo[j], 0, 0));
            uq[j] = ucol(__builtin_amdgcn_raw_buffer_load_b32(ru, qo[j], 0, 0));
        }
    }
    // One segment t: the next segment's seeds are loaded, then hook() runs (it
    // may start a copy: issued after those loads, it is not waited for with
    // them), then the terms, with entry(i) the table interval i (byte offset
    // i * 16 given as off).
    auto segment = [&](int32_t t, auto hook, auto entry) {
        const int32_t tn = min(t + 1, nt - 1);
        const size_t o = (size_t)tn * (size_t)npix;
        const __amdgpu_buffer_rsrc_t rg = seg_rsrc(gamma + o, npix), ru = seg_rsrc(U + o, npix);
        const float an = ONE ? a[tn] : 1.0f;
        float gpn[8], gqn[4];
        uint32_t upn[8], uqn[4];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            gpn[i] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rg, po[i], 0, 0));
            upn[i] = __builtin_amdgcn_raw_buffer_load_b32(ru, po[i], 0, 0);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            gqn[j] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rg, qo[j], 0, 0));
            uqn[j] = __builtin_amdgcn_raw_buffer_load_b32(ru, qo[j], 0, 0);
        }
        hook();
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            float4 c[4];
            float x[4];
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const uint32_t d = abs_diff(up[i], uq[jj]);
                c[jj] = entry(d >> fb);
                x[jj] = __uint_as_float(((d << (23 - fb)) & 0x007fffffu) | 0x3f800000u);
            }
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const float4 cc = c[jj];
                const float W = fmaf(fmaf(fmaf(cc.w, x[jj], cc.z), x[jj], cc.y), x[jj], cc.x);
                acc[i][jj] = fmaf(gp[i] * gq[jj], W, acc[i][jj]);
            }
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            gp[i] = ONE ? an * gpn[i] : gpn[i];
            up[i] = upn[i];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            gq[j] = gqn[j];
            uq[j] = ucol(uqn[j]);
        }
    };
    auto none = [] {};
    if constexpr (ONE) {
        __shared__ float4 tab[kLdsTable];
        if (ntu > 0) {
            copy_lds(cub, tab, Jv);
            __builtin_amdgcn_s_waitcnt(kWaitVm0);
            __syncthreads();
        }
        for (int32_t t = 0; t < ntu; ++t) segment(t, none, [](uint32_t i) { return tab[i]; });
    } else {
    __shared__ float4 tab0[kHalf], tab1[kHalf];
    // a table longer than one array: intervals [0, kHalf) in tab0, the rest in tab1
    auto split_entry = [](uint32_t i) { return i < (uint32_t)kHalf ? tab0[i] : tab1[i - kHalf]; };
    auto copy_split = [&](const float4 *src) {
        copy_lds(src, tab0, min(Jv, kHalf));
        if (Jv > kHalf) copy_lds(src + kHalf, tab1, Jv - kHalf);
    };
    if (2 * Jv <= kLdsTable) {
        // double-buffered stages of g tables each, tab0 and tab1 by turns
        const int32_t g = kHalf / Jv;
        auto stage = [&](int32_t s0, const float4 *cur, float4 *nxt) {
            const int32_t s1 = min(s0 + g, nt);
            __builtin_amdgcn_s_waitcnt(kWaitVm0);  // this stage's tables have landed (this lane's share)
            __syncthreads();                        // ... every lane's; the previous stage is no longer read
            // the stage's first segment copies the next stage in, always (the
            // last stage copies table 0 into the idle buffer), so that the
            // count of copy instructions after its loads is known
            const int32_t cs = s1 < nt ? s1 : 0, cn = s1 < nt ? min(g, nt - s1) * Jv : Jv;
            segment(s0, [&] { copy_lds_half(cub + (size_t)cs * Jv, nxt, cn); }, [cur](uint32_t i) { return cur[i]; });
            for (int32_t t = s0 + 1; t < s1; ++t) {
                const float4 *tt = cur + (size_t)(t - s0) * Jv;
                segment(t, none, [tt](uint32_t i) { return tt[i]; });
            }
        };
        if (ntu > 0) copy_lds(cub, tab0, min(g, nt) * Jv);
        for (int32_t s0 = 0; s0 < ntu; s0 += 2 * g) {
            stage(s0, tab0, tab1);
            if (s0 + g < ntu) stage(s0 + g, tab1, tab0);
        }
    } else {
        // one table at a time, spanning both arrays
        for (int32_t t = 0; t < ntu; ++t) {
            if (t > 0) __syncthreads();  // the previous table is no longer read
            copy_split(cub + (size_t)t * Jv);
            __builtin_amdgcn_s_waitcnt(kWaitVm0);
            __syncthreads();
            segment(t, none, split_entry);
        }
    }
    }
    if (!active) return;
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int64_t p = p0 + i, q = q0 + jj;
            // rejected seeds: the matrix is NaN
            const float v = rejected ? __builtin_nanf("") : acc[i][jj];
            if (p < nrow && q < nrow && (tr != tc || p <= q)) store_value(G, npix, nside, ns, p, q, v, accumulate);
        }
}

bool fisher_full_band_ok(double f_max)
{
    double delta;
    int32_t J, fb;
    fisher_table_geometry(f_max, &delta, &J, &fb);
    return fb >= kFracBitsMin;
}

// SGWB_FISHER_TABLE=global keeps the table in global memory (both forms give
// bitwise the same matrix).
static bool fisher_full_table_in_lds()
{
    const char *e = std::getenv("SGWB_FISHER_TABLE");
    return !(e && std::strcmp(e, "global") == 0);
}

// Separable weights go through the streaming kernel (one table, 8 x 4
// entries a lane: 25 % faster); SGWB_FISHER_ONE_TABLE=persistent selects the
// persistent LDS kernel (4 x 4 a thread).  Both give the same bits.
static bool fisher_full_one_table_stream()
{
    const char *e = std::getenv("SGWB_FISHER_ONE_TABLE");
    return !(e && std::strcmp(e, "persistent") == 0);
}

static size_t up256(size_t n) { return (n + 255) & ~(size_t)255; }

// nbins bounds the band width (the chunk count of the table pass).
size_t fisher_full_workspace_bytes(double f_max, int32_t nbins, int32_t nt, int32_t npix)
{
    double delta;
    int32_t J, fb;
    fisher_table_geometry(f_max, &delta, &J, &fb);
    const size_t nchunk = ((size_t)nbins + kTabChunk - 1) / kTabChunk;
    return up256(nchunk * (J + 1) * sizeof(double2)) + up256((size_t)J * sizeof(float4)) +
           up256((size_t)nt * npix * sizeof(uint32_t)) + up256(kSymParts * sizeof(double));
}

hipError_t launch_fisher_full(const float *a, const float *b, int32_t rank, const float *H, int32_t nf, int32_t clo,
                              int32_t chi, double f0, double df, int64_t k0, const float *gamma, const double *tau,
                              int32_t nt, int32_t npix, int64_t nside, float *G, void *work, hipStream_t s)
{
    const double f_max = f0 + (double)(k0 + chi - 1) * df;
    double delta;
    int32_t J, fb;
    fisher_table_geometry(f_max, &delta, &J, &fb);
    if (fb < kFracBitsMin) return hipErrorInvalidValue;
    const int32_t nchunk = (chi - clo + kTabChunk - 1) / kTabChunk;
    if (nchunk > 65535) return hipErrorInvalidValue;
    char *w = reinterpret_cast<char *>(work);
    double2 *part = reinterpret_cast<double2 *>(w);
    w += up256((size_t)nchunk * (J + 1) * sizeof(double2));
    float4 *cub = reinterpret_cast<float4 *>(w);
    w += up256((size_t)J * sizeof(float4));
    uint32_t *U = reinterpret_cast<uint32_t *>(w);
    w += up256((size_t)nt * npix * sizeof(uint32_t));
    double *flags = nullptr;
    if (nside > 0) {
        flags = reinterpret_cast<double *>(w);
        const hipError_t e = launch_antipodal_check(gamma, tau, nt, npix, nside, flags, s);
        if (e != hipSuccess) return e;
    }
    const int64_t n = (int64_t)nt * npix;
    hipLaunchKernelGGL(fixed_delay_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, tau, n,
                       std::ldexp(1.0, fb) / delta, U);
    // antipodal: the two triangles of the northern blocks; otherwise the whole upper triangle
    const int64_t nrow = nside > 0 ? npix / 2 : npix;
    const int64_t nT = (nrow + kFt - 1) / kFt, ntiles = (nside > 0 ? 2 : 1) * (nT * (nT + 1) / 2);
    if (ntiles > 0x7fffffff) return hipErrorInvalidValue;
    const bool lds = J <= kLdsTable && fisher_full_table_in_lds();
    int cus = 256;
    if (lds) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
    }
    // one delay table and one pass over the matrix per rank of the weights,
    // the later passes adding to G
    for (int32_t r = 0; r < rank; ++r) {
        const float *ar = a + (int64_t)r * nt, *br = b + (int64_t)r * nf;
        hipLaunchKernelGGL(delay_table_kernel, dim3((unsigned)((J + 1 + 255) / 256), (unsigned)nchunk), dim3(256), 0,
                           s, H, br, clo, chi, f0, df, k0, delta, J, part);
        hipLaunchKernelGGL(delay_cubic_kernel, dim3((unsigned)((J + 255) / 256)), dim3(256), 0, s, part, nchunk, J,
                           cub);
        if (lds && fisher_full_one_table_stream()) {
            hipLaunchKernelGGL(fisher_full_stream_kernel<true>, dim3((unsigned)((ntiles + kStTiles - 1) / kStTiles)),
                               dim3(kStWaves * 64), 0, s, ar, gamma, U, nt, npix, nside, flags, cub, J,
                               (const unsigned long long *)nullptr, delta, fb, ntiles, (int32_t)(r > 0), G);
        } else if (lds) {
            const int64_t grid = std::min<int64_t>(cus, (ntiles + 1) / 2);
            hipLaunchKernelGGL(fisher_full_lds_kernel, dim3((unsigned)grid), dim3(512), 0, s, ar, gamma, U, nt, npix,
                               nside, flags, cub, J, fb, ntiles, (int32_t)(r > 0), G);
        } else {
            hipLaunchKernelGGL(fisher_full_kernel, dim3((unsigned)ntiles), dim3(256), 0, s, ar, gamma, U, nt, npix,
                               nside, flags, cub, J, (const unsigned long long *)nullptr, delta, fb, (int32_t)(r > 0),
                               G);
        }
    }
    return hipGetLastError();
}

// ---- general weights: workspace layout and launch ----
struct GeneralLayout {
    int32_t J = 0, fb = 0;
    StripGrid sg;     // expanded basis (sg.S > 0) or direct
    int32_t nk = 0;   // K of the table contraction
    int64_t ntiles = 0;
    size_t part = 0, cub = 0, U = 0, flags = 0, bound = 0, mu = 0, nu = 0, total = 0;  // byte offsets (total: size)
};

static GeneralLayout general_layout(double f0, double df, int64_t k0, int32_t clo, int32_t chi, int32_t nt,
                                    int32_t npix, int64_t nside)
{
    GeneralLayout L;
    double delta;
    fisher_table_geometry(f0 + (double)(k0 + chi - 1) * df, &delta, &L.J, &L.fb);
    L.sg = strip_grid(df, k0, clo, chi);
    L.nk = L.sg.S > 0 ? L.sg.n * kTxTerms : chi - clo;
    const int64_t nrow = nside > 0 ? npix / 2 : npix;
    const int64_t nT = (nrow + kFt - 1) / kFt;
    L.ntiles = (nside > 0 ? 2 : 1) * (nT * (nT + 1) / 2);
    size_t o = 0;
    L.part = o;
    o += up256((size_t)table_split_cap(L.nk) * nt * (L.J + 1) * sizeof(double2));
    L.cub = o;
    o += up256((size_t)nt * L.J * sizeof(float4));
    L.U = o;
    o += up256((size_t)nt * npix * sizeof(uint32_t));
    L.flags = o;
    o += up256(kSymParts * sizeof(double));
    L.bound = o;
    o += 256;
    if (L.sg.S > 0) {
        L.mu = o;
        o += up256((size_t)nt * L.nk * sizeof(double));
        L.nu = o;
        o += up256((size_t)nt * L.nk * sizeof(double));
    }
    L.total = o;
    return L;
}

size_t fisher_full_general_workspace_bytes(double f0, double df, int64_t k0, int32_t clo, int32_t chi, int32_t nt,
                                           int32_t npix, int64_t nside)
{
    return general_layout(f0, df, k0, clo, chi, nt, npix, nside).total;
}

hipError_t launch_fisher_full_general(const float *w, int64_t ldw, const float *H, int32_t clo, int32_t chi,
                                      double f0, double df, int64_t k0, const float *gamma, const double *tau,
                                      int32_t nt, int32_t npix, int64_t nside, float *G, void *work, hipStream_t s)
{
    const GeneralLayout L = general_layout(f0, df, k0, clo, chi, nt, npix, nside);
    if (L.fb < kFracBitsMin || L.ntiles > 0x7fffffff) return hipErrorInvalidValue;
    double delta;
    int32_t J, fb;
    fisher_table_geometry(f0 + (double)(k0 + chi - 1) * df, &delta, &J, &fb);
    char *base = reinterpret_cast<char *>(work);
    double2 *part = reinterpret_cast<double2 *>(base + L.part);
    float4 *cub = reinterpret_cast<float4 *>(base + L.cub);
    uint32_t *U = reinterpret_cast<uint32_t *>(base + L.U);
    unsigned long long *bound = reinterpret_cast<unsigned long long *>(base + L.bound);
    double *flags = nullptr;
    if (nside > 0) {
        flags = reinterpret_cast<double *>(base + L.flags);
        const hipError_t e = launch_antipodal_check(gamma, tau, nt, npix, nside, flags, s);
        if (e != hipSuccess) return e;
    }
    const int64_t n = (int64_t)nt * npix;
    hipLaunchKernelGGL(delay_bound_init_kernel, dim3(1), dim3(64), 0, s, bound);
    hipLaunchKernelGGL(delay_bound_kernel, dim3((unsigned)std::min<int64_t>(2048, (n + 255) / 256)), dim3(256), 0,
                       s, tau, n, bound);
    hipLaunchKernelGGL(fixed_delay_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, tau, n,
                       std::ldexp(1.0, fb) / delta, U);
    int cus = 256, dev = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    // persistent: two workgroups per compute unit (their registers allow two)
    if (L.sg.S > 0) {
        double *mu = reinterpret_cast<double *>(base + L.mu), *nu = reinterpret_cast<double *>(base + L.nu);
        hipLaunchKernelGGL(table_moments_kernel, dim3((unsigned)((L.sg.n + kTxStrips - 1) / kTxStrips), (unsigned)nt),
                           dim3(kTxStrips * kTxSplit), 0, s, w,
                           ldw, H, clo, chi, f0, df, k0, L.sg.S, L.sg.first, L.sg.n, mu, nu);
        hipLaunchKernelGGL(delay_table_gemm_kernel<true>, dim3((unsigned)(2 * cus)), dim3(256), 0, s, w, ldw, H,
                           (const double *)mu, (const double *)nu, nt, clo, L.nk, f0, df, k0, L.sg.S, L.sg.first,
                           delta, J, (const unsigned long long *)bound, part);
    } else {
        hipLaunchKernelGGL(delay_table_gemm_kernel<false>, dim3((unsigned)(2 * cus)), dim3(256), 0, s, w, ldw, H,
                           (const double *)nullptr, (const double *)nullptr, nt, clo, L.nk, f0, df, k0, (int32_t)0,
                           (int64_t)0, delta, J, (const unsigned long long *)bound, part);
    }
    hipLaunchKernelGGL(delay_cubic_general_kernel, dim3((unsigned)((J + 255) / 256), (unsigned)nt), dim3(256), 0, s,
                       part, nt, L.nk, J, (const unsigned long long *)bound, delta, cub);
    if (J <= kLdsTable && fisher_full_table_in_lds()) {
        const int64_t grid = (L.ntiles + kStTiles - 1) / kStTiles;
        hipLaunchKernelGGL(fisher_full_stream_kernel<false>, dim3((unsigned)grid), dim3(kStWaves * 64), 0, s,
                           (const float *)nullptr, gamma, U, nt, npix, nside, flags, cub, J,
                           (const unsigned long long *)bound, delta, fb, L.ntiles, (int32_t)0, G);
    } else {
        hipLaunchKernelGGL(fisher_full_kernel, dim3((unsigned)L.ntiles), dim3(256), 0, s, (const float *)nullptr,
                           gamma, U, nt, npix, nside, flags, cub, J, (const unsigned long long *)bound, delta, fb,
                           (int32_t)0, G);
    }
    return hipGetLastError();
}

// ---- conjugate gradient on G P = X (float64 vectors, fixed-order sums) ----
// Three kernels per iteration: q = G p with the partial sums of p.q; the step
// (every block adds the p.q partials itself, in one fixed order, so all agree
// on alpha) with the partial sums of r.r; the new direction (likewise for
// beta).  The scalars never leave the device.

// q = G p for kCgRows rows per workgroup: each p[j] is read once for all of
// them; per-thread partial sums over a fixed column stride, then a fixed tree;
// the workgroup's share of p.q goes to pq_part[blockIdx.x].
// VEC: four consecutive columns per load (n % 4 == 0, G 16-byte aligned).
constexpr int kCgRows = 4;

template <bool VEC>
__global__ __launch_bounds__(256) void cg_matvec_kernel(const float *__restrict__ G, const double *__restrict__ p,
                                                        int32_t n, double *__restrict__ q,
                                                        double *__restrict__ pq_part)
{
    __shared__ double red[kCgRows][256];
    const int64_t r0 = (int64_t)blockIdx.x * kCgRows;
    const int nr = (int)min<int64_t>(kCgRows, n - r0);
    const float *row[kCgRows];
#pragma unroll
    for (int r = 0; r < kCgRows; ++r) row[r] = G + (r0 + min(r, nr - 1)) * n;  // tail rows repeat the last
    double acc[kCgRows] = {};
    if (VEC) {
        const int32_t n4 = n / 4;
        for (int32_t j4 = threadIdx.x; j4 < n4; j4 += 256) {
            const double2 pa = reinterpret_cast<const double2 *>(p)[2 * j4];
            const double2 pb = reinterpret_cast<const double2 *>(p)[2 * j4 + 1];
#pragma unroll
            for (int r = 0; r < kCgRows; ++r) {
                const float4 g = reinterpret_cast<const float4 *>(row[r])[j4];
                acc[r] += (double)g.x * pa.x + (double)g.y * pa.y + (double)g.z * pb.x + (double)g.w * pb.y;
            }
        }
    } else {
        for (int32_t j = threadIdx.x; j < n; j += 256) {
            const double pj = p[j];
#pragma unroll
            for (int r = 0; r < kCgRows; ++r) acc[r] += (double)row[r][j] * pj;
        }
    }
#pragma unroll
    for (int r = 0; r < kCgRows; ++r) red[r][threadIdx.x] = acc[r];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
#pragma unroll
            for (int r = 0; r < kCgRows; ++r) red[r][threadIdx.x] += red[r][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double d = 0.0;
        for (int r = 0; r < nr; ++r) {
            q[r0 + r] = red[r][0];
            d += p[r0 + r] * red[r][0];
        }
        pq_part[blockIdx.x] = d;
    }
}

// Sum of part[0..np) in a fixed order (per-thread strides, then a fixed tree),
// the same in every block; called by all 256 threads.
__device__ __forceinline__ double cg_block_sum(const double *__restrict__ part, int32_t np, double *red)
{
    double acc = 0.0;
    for (int32_t j = threadIdx.x; j < np; j += 256) acc += part[j];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    const double v = red[0];
    __syncthreads();
    return v;
}

// Partial sums of x.y, one per block of 256 elements.
__device__ __forceinline__ void cg_block_dot(double v, double *__restrict__ part, double *red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// x = 0, r = p = X, partial sums of r.r
__global__ __launch_bounds__(256) void cg_init_kernel(const float *__restrict__ X, int32_t n, double *__restrict__ x,
                                                      double *__restrict__ r, double *__restrict__ p,
                                                      double *__restrict__ rr_part)
{
    __shared__ double red[256];
    const int32_t j = blockIdx.x * 256 + threadIdx.x;
    double v = 0.0;
    if (j < n) {
        const double xj = (double)X[j];
        x[j] = 0.0;
        r[j] = p[j] = xj;
        v = xj * xj;
    }
    cg_block_dot(v, rr_part, red);
}

// alpha = rr / pq (0 once the residual or the curvature vanishes); x += alpha p;
// r -= alpha q; partial sums of the new r.r.  rr = sum of rr_part (nb blocks).
__global__ __launch_bounds__(256) void cg_step_kernel(double *__restrict__ x, double *__restrict__ r,
                                                      const double *__restrict__ p, const double *__restrict__ q,
                                                      const double *__restrict__ rr_part,
                                                      const double *__restrict__ pq_part, int32_t nb, int32_t nm,
                                                      int32_t n, double *__restrict__ rr_new_part)
{
    __shared__ double red[256];
    const double rr = cg_block_sum(rr_part, nb, red), pq = cg_block_sum(pq_part, nm, red);
    const double alpha = (rr != 0.0 && pq != 0.0) ? rr / pq : 0.0;
    const int32_t j = blockIdx.x * 256 + threadIdx.x;
    double v = 0.0;
    if (j < n) {
        x[j] += alpha * p[j];
        const double rj = r[j] - alpha * q[j];
        r[j] = rj;
        v = rj * rj;
    }
    cg_block_dot(v, rr_new_part, red);
}

// p = r + (rr_new / rr) p
__global__ __launch_bounds__(256) void cg_dir_kernel(double *__restrict__ p, const double *__restrict__ r,
                                                     const double *__restrict__ rr_part,
                                                     const double *__restrict__ rr_new_part, int32_t nb, int32_t n)
{
    __shared__ double red[256];
    const double rr = cg_block_sum(rr_part, nb, red), rr_new = cg_block_sum(rr_new_part, nb, red);
    const double beta = rr != 0.0 ? rr_new / rr : 0.0;
    const int32_t j = blockIdx.x * 256 + threadIdx.x;
    if (j < n) p[j] = r[j] + beta * p[j];
}

__global__ __launch_bounds__(256) void cg_out_kernel(const double *__restrict__ x, int32_t n, float *__restrict__ P)
{
    const int32_t j = blockIdx.x * 256 + threadIdx.x;
    if (j < n) P[j] = (float)x[j];
}

size_t cg_workspace_bytes(int32_t n)
{
    const size_t nb = ((size_t)n + 255) / 256, nm = ((size_t)n + kCgRows - 1) / kCgRows;
    return (4 * (size_t)n + nm + 2 * nb) * sizeof(double);
}

hipError_t launch_clean_map_cg(const float *G, const float *X, int32_t n, int32_t niter, float *P, void *work,
                               hipStream_t s)
{
    const int32_t nb = (n + 255) / 256, nm = (n + kCgRows - 1) / kCgRows;
    double *x = reinterpret_cast<double *>(work), *r = x + n, *p = r + n, *q = p + n;
    double *pq_part = q + n, *rr_a = pq_part + nm, *rr_b = rr_a + nb;  // r.r partials, this and the next iterate
    const bool vec = n % 4 == 0 && reinterpret_cast<uintptr_t>(G) % 16 == 0;
    hipLaunchKernelGGL(cg_init_kernel, dim3((unsigned)nb), dim3(256), 0, s, X, n, x, r, p, rr_a);
    for (int32_t it = 0; it < niter; ++it) {
        double *rr = (it & 1) ? rr_b : rr_a, *rr_new = (it & 1) ? rr_a : rr_b;
        if (vec)
            hipLaunchKernelGGL(cg_matvec_kernel<true>, dim3((unsigned)nm), dim3(256), 0, s, G, p, n, q, pq_part);
        else
            hipLaunchKernelGGL(cg_matvec_kernel<false>, dim3((unsigned)nm), dim3(256), 0, s, G, p, n, q, pq_part);
        hipLaunchKernelGGL(cg_step_kernel, dim3((unsigned)nb), dim3(256), 0, s, x, r, p, q, rr, pq_part, nb, nm, n,
                           rr_new);
        hipLaunchKernelGGL(cg_dir_kernel, dim3((unsigned)nb), dim3(256), 0, s, p, r, rr, rr_new, nb, n);
    }
    hipLaunchKernelGGL(cg_out_kernel, dim3((unsigned)nb), dim3(256), 0, s, x, n, P);
    return hipGetLastError();
}

}  // namespace sgwb

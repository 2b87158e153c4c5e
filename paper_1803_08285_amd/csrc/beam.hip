// Per-bin Fisher diagonal ("beam") Gam(k,p) = sum_t w(t,k) gamma(t,p)^2
// (Eq. eq_fisher with p = p', split per bin as in Sec. III.A) on gfx950.
//
// It is a dense contraction Gam = W^T G2 with M = bins, N = pixels, K = segments,
// so it runs on the matrix cores:
//   * prep kernels split the float32 operands W and G2 = gamma^2 into
//     bfloat16 hi + lo (x = hi + lo + O(2^-17 x)) and store them in MFMA
//     fragment order: for a 32-row (or 32-column) block and a 16-segment
//     K-step, lane l holds the 8 consecutive segments 8 (l / 32) .. +7 of row
//     32 * block + l % 32, exactly the operand layout of
//     v_mfma_f32_32x32x16_bf16, so the GEMM loads each fragment with one
//     16-byte load per lane;
//   * the GEMM accumulates hi.hi + hi.lo + lo.hi in float32 (lo.lo, below
//     2^-16 relative, is dropped) in a fixed K order;
//   * with antipodal seeds only the northern half of the pixels is computed
//     and each result is also written to the antipode column.
// A float64 vector-unit kernel serves the float64 path.
#include "sgwb_internal.h"

namespace sgwb {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kBlk = 32;  // rows/columns per MFMA block
constexpr int kKs = 16;   // segments per MFMA K-step

// float32 -> bfloat16 bits, round to nearest even (finite inputs).
__device__ inline uint32_t bf16_bits(float x)
{
    const uint32_t u = __float_as_uint(x);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
__device__ inline float bf16_value(uint32_t b) { return __uint_as_float(b << 16); }

// Pack 8 values into hi and lo bf16 fragments.
__device__ inline void split8(const float v[8], uint4 *hi, uint4 *lo)
{
    uint32_t h[8], l[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        h[e] = bf16_bits(v[e]);
        l[e] = bf16_bits(v[e] - bf16_value(h[e]));
    }
    *hi = make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16));
    *lo = make_uint4(l[0] | (l[1] << 16), l[2] | (l[3] << 16), l[4] | (l[5] << 16), l[6] | (l[7] << 16));
}

struct FragDims {
    int64_t nblk;  // 32-wide blocks
    int64_t nks;   // 16-deep K steps
};
__host__ __device__ inline FragDims frag_dims(int64_t n, int64_t nt)
{
    return FragDims{(n + kBlk - 1) / kBlk, (nt + kKs - 1) / kKs};
}
// Fragment array: [blk][ks][part 0 = hi, 1 = lo][64 lanes] of uint4.
__host__ __device__ inline int64_t frag_index(int64_t blk, int64_t ks, int part, int lane, int64_t nks)
{
    return ((blk * nks + ks) * 2 + part) * 64 + lane;
}

// W[t][ldc] (row t, column = bin) -> fragments; SQUARE squares the value first
// (used for gamma -> gamma^2).
template <bool SQUARE>
__global__ __launch_bounds__(256) void prep_frag_kernel(const float *__restrict__ src, int64_t ld,
                                                         int32_t nt, int64_t n, FragDims fd,
                                                         uint4 *__restrict__ dst)
{
    const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t total = fd.nblk * fd.nks * 64;
    if (gid >= total) return;
    const int lane = (int)(gid & 63);
    const int64_t ks = (gid >> 6) % fd.nks;
    const int64_t blk = (gid >> 6) / fd.nks;
    const int64_t col = blk * kBlk + (lane & 31);
    const int64_t t0 = ks * kKs + (lane >> 5) * 8;
    float v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int64_t t = t0 + e;
        float x = 0.0f;
        if (col < n && t < nt) x = src[t * ld + col];
        v[e] = SQUARE ? x * x : x;
    }
    uint4 hi, lo;
    split8(v, &hi, &lo);
    dst[frag_index(blk, ks, 0, lane, fd.nks)] = hi;
    dst[frag_index(blk, ks, 1, lane, fd.nks)] = lo;
}

// Each wave computes a (WM x 32) x (WN x 32) tile of Gam; waves are independent
// and read their operand fragments straight from L2 (the fragment arrays are
// small: every fragment is reused by all waves of its tile row or column).
// The next K-step's fragments are loaded while the current step's MFMAs run.
constexpr int WM = 4, WN = 4;

struct Frags {
    uint4 a[WM][2], b[WN][2];
};

__device__ inline void load_frags(Frags &f, const uint4 *__restrict__ Wf, const uint4 *__restrict__ Gf,
                                  int64_t tm, int64_t tn, int64_t ks, const FragDims &fm, const FragDims &fn,
                                  int lane)
{
    const uint4 zero4 = make_uint4(0, 0, 0, 0);
#pragma unroll
    for (int i = 0; i < WM; ++i) {
        const int64_t mb = tm * WM + i;
#pragma unroll
        for (int part = 0; part < 2; ++part)
            f.a[i][part] = mb < fm.nblk ? Wf[frag_index(mb, ks, part, lane, fm.nks)] : zero4;
    }
#pragma unroll
    for (int j = 0; j < WN; ++j) {
        const int64_t nb = tn * WN + j;
#pragma unroll
        for (int part = 0; part < 2; ++part)
            f.b[j][part] = nb < fn.nblk ? Gf[frag_index(nb, ks, part, lane, fn.nks)] : zero4;
    }
}

// Wave-tile order.  Workgroups are dispatched round-robin over the 8 XCDs
// (each with its own L2), so workgroup b runs on XCD b % 8.  The tile grid is
// cut into patches of kPatch x kPatch wave tiles; XCD x works through patches
// x, x + 8, x + 16, ... and the 16 workgroups (64 waves) of a patch share its
// 8 bin tiles and 8 pixel tiles through that XCD's L2.
constexpr int kXcds = 8;
constexpr int kPatch = 8;
constexpr int kWavesPerWg = 4;
constexpr int kWgPerPatch = kPatch * kPatch / kWavesPerWg;

__device__ inline bool patch_tile(int64_t b, int w, int64_t tiles_m, int64_t tiles_n, int64_t *tm, int64_t *tn)
{
    const int64_t pm = (tiles_m + kPatch - 1) / kPatch, pn = (tiles_n + kPatch - 1) / kPatch;
    const int64_t xcd = b % kXcds, l = b / kXcds;
    const int64_t patch = xcd + kXcds * (l / kWgPerPatch);
    if (patch >= pm * pn) return false;
    const int64_t in = (l % kWgPerPatch) * kWavesPerWg + w;  // 0 .. 63 inside the patch
    // patches walk the bin direction fastest, so neighbouring patches share pixel tiles
    const int64_t pi = patch % pm, pj = patch / pm;
    *tm = pi * kPatch + in % kPatch;
    *tn = pj * kPatch + in / kPatch;
    return *tm < tiles_m && *tn < tiles_n;
}

// Number of workgroups that covers every patch for the XCD-striped order.
__host__ inline int64_t patch_grid(int64_t tiles_m, int64_t tiles_n)
{
    const int64_t pm = (tiles_m + kPatch - 1) / kPatch, pn = (tiles_n + kPatch - 1) / kPatch;
    const int64_t patches = pm * pn;
    const int64_t per_xcd = (patches + kXcds - 1) / kXcds;
    return per_xcd * kWgPerPatch * kXcds;
}

__global__ __launch_bounds__(256) void beam_gemm_kernel(const uint4 *__restrict__ Wf,
                                                         const uint4 *__restrict__ Gf, FragDims fm,
                                                         FragDims fn, int32_t nf, int64_t ncol,
                                                         int32_t npix, int64_t nside,
                                                         float *__restrict__ Gam)
{
    const int lane = threadIdx.x & 63;
    const int64_t tiles_m = (fm.nblk + WM - 1) / WM;
    const int64_t tiles_n = (fn.nblk + WN - 1) / WN;
    int64_t tm, tn;
    if (!patch_tile(blockIdx.x, threadIdx.x >> 6, tiles_m, tiles_n, &tm, &tn)) return;
    const int64_t nks = fm.nks;

    f32x16 acc[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

    Frags cur, nxt;
    load_frags(cur, Wf, Gf, tm, tn, 0, fm, fn, lane);
    for (int64_t ks = 0; ks < nks; ++ks) {
        if (ks + 1 < nks) load_frags(nxt, Wf, Gf, tm, tn, ks + 1, fm, fn, lane);
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
            for (int j = 0; j < WN; ++j) {
                const bf16x8 ah = __builtin_bit_cast(bf16x8, cur.a[i][0]);
                const bf16x8 al = __builtin_bit_cast(bf16x8, cur.a[i][1]);
                const bf16x8 bh = __builtin_bit_cast(bf16x8, cur.b[j][0]);
                const bf16x8 bl = __builtin_bit_cast(bf16x8, cur.b[j][1]);
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc[i][j], 0, 0, 0);
            }
        if (ks + 1 < nks) cur = nxt;
    }

    // Accumulator layout of the 32x32 MFMA: lane l holds column l % 32 and rows
    // 8 (r / 4) + 4 (l / 32) + r % 4 for r = 0..15.
#pragma unroll
    for (int j = 0; j < WN; ++j) {
        const int64_t n = (tn * WN + j) * kBlk + (lane & 31);
        if (n >= ncol) continue;
        int64_t nB = -1;
        if (nside > 0) nB = antipode_north(ring_of_north(n, nside), npix);
#pragma unroll
        for (int i = 0; i < WM; ++i) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t m = (tm * WM + i) * kBlk + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                if (m >= nf) continue;
                float *row = Gam + m * (int64_t)npix;
                row[n] = acc[i][j][r];
                if (nB >= 0) row[nB] = acc[i][j][r];
            }
        }
    }
}

size_t beam_workspace_bytes(int32_t nt, int32_t nf, int32_t ncol)
{
    const FragDims fm = frag_dims(nf, nt), fn = frag_dims(ncol, nt);
    return (size_t)(fm.nblk + fn.nblk) * (size_t)fm.nks * 2 * 64 * sizeof(uint4);
}

hipError_t launch_beam_bf16x3(const MapArgs &a, const float *w, const float *gamma, float *Gam,
                              void *work, hipStream_t s)
{
    const bool pair = a.nside > 0;
    const int64_t ncol = pair ? a.npix / 2 : a.npix;
    const FragDims fm = frag_dims(a.nf, a.nt), fn = frag_dims(ncol, a.nt);
    uint4 *Wf = reinterpret_cast<uint4 *>(work);
    uint4 *Gf = Wf + fm.nblk * fm.nks * 2 * 64;
    const int64_t nw = fm.nblk * fm.nks * 64, ng = fn.nblk * fn.nks * 64;
    // the bins of this call start at column 0 of w (the caller offsets w by k0)
    hipLaunchKernelGGL(prep_frag_kernel<false>, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s, w,
                       a.ldc, a.nt, (int64_t)a.nf, fm, Wf);
    hipLaunchKernelGGL(prep_frag_kernel<true>, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, s, gamma,
                       (int64_t)a.npix, a.nt, ncol, fn, Gf);
    const int64_t grid = patch_grid((fm.nblk + WM - 1) / WM, (fn.nblk + WN - 1) / WN);
    hipLaunchKernelGGL(beam_gemm_kernel, dim3((unsigned)grid), dim3(256), 0, s, Wf, Gf, fm, fn,
                       a.nf, ncol, a.npix, pair ? a.nside : (int64_t)0, Gam);
    return hipGetLastError();
}

// float64 path: one thread per (bin, pixel column), sequential sum over t.
__global__ __launch_bounds__(256) void beam_f64_kernel(MapArgs a, const double *__restrict__ w,
                                                        const double *__restrict__ gamma,
                                                        double *__restrict__ Gam)
{
    const bool pair = a.nside > 0;
    const int64_t ncol = pair ? a.npix / 2 : a.npix;
    const int64_t col = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t k = blockIdx.y;
    if (col >= ncol || k >= a.nf) return;
    double acc = 0.0;
    for (int t = 0; t < a.nt; ++t) {
        const double g = gamma[(int64_t)t * a.npix + col];
        acc = fma(w[(int64_t)t * a.ldc + k], g * g, acc);
    }
    double *row = Gam + k * (int64_t)a.npix;
    row[col] = acc;
    if (pair) row[antipode_north(ring_of_north(col, a.nside), a.npix)] = acc;
}

hipError_t launch_beam_f64(const MapArgs &a, const double *w, const double *gamma, double *Gam,
                           hipStream_t s)
{
    const int64_t ncol = a.nside > 0 ? a.npix / 2 : a.npix;
    for (int64_t k0 = 0; k0 < a.nf; k0 += 65535) {
        MapArgs b = a;
        b.nf = (int32_t)(a.nf - k0 < 65535 ? a.nf - k0 : 65535);
        hipLaunchKernelGGL(beam_f64_kernel, dim3((unsigned)((ncol + 255) / 256), (unsigned)b.nf), dim3(256),
                           0, s, b, w + k0, gamma, Gam + k0 * (int64_t)a.npix);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace sgwb

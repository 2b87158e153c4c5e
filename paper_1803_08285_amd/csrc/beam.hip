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
//     16-byte load per lane (with 2 x 4 wave tiles the four waves of a
//     workgroup share each K-step's pixel-side fragments through LDS); the
//     arrays are padded to whole 4-block tiles with zero blocks, so no load
//     needs a bounds condition;
//   * the GEMM accumulates hi.hi + hi.lo + lo.hi in float32 (lo.lo, below
//     2^-16 relative, is dropped) in a fixed K order;
//   * with antipodal seeds only the northern half of the pixels is computed
//     and each result is also written to the antipode column, with streaming
//     (nontemporal) stores.
// A float64 vector-unit kernel serves the float64 path.
#include "sgwb_internal.h"

namespace sgwb {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));


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
#pragma clang fp contract(off)  // the residual uses the same rounded value as hi
    uint32_t h[8], l[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        h[e] = bf16_bits(v[e]);
        l[e] = bf16_bits(v[e] - bf16_value(h[e]));
    }
    *hi = make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16));
    *lo = make_uint4(l[0] | (l[1] << 16), l[2] | (l[3] << 16), l[4] | (l[5] << 16), l[6] | (l[7] << 16));
}

// Fragment array: [blk][ks][part 0 = hi, 1 = lo][64 lanes] of uint4, with
// the block count padded to whole 4-block tiles; the padding blocks are zero.
constexpr int64_t kTileBlocks = 4;
__host__ __device__ inline int64_t padded_blocks(int64_t nblk)
{
    return (nblk + kTileBlocks - 1) / kTileBlocks * kTileBlocks;
}
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

// The three products of a K-step are issued part by part over all WM x WN
// accumulators so that consecutive MFMAs never depend on each other.

template <int WM, int WN>
struct Frags {
    uint4 a[WM][2], b[WN][2];
};

// The fragment arrays arrive through a by-value job descriptor, so the
// compiler cannot tell that they live in global memory and would read them
// with flat loads, which also count against the LDS counter and must wait for
// the direct global -> LDS copies.  Reading through an explicit global
// pointer keeps those loads on the vector-memory counter alone.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__device__ inline const __attribute__((address_space(1))) u32x4 *as_global(const uint4 *p)
{
    return (const __attribute__((address_space(1))) u32x4 *)p;
}

// Fragment (blk, ks, part) for this lane.  The arrays hold whole tiles
// (padded_blocks), so every block a wave tile touches exists and the loads
// need no condition: a condition would turn into a branch around each load
// and keep the compiler from counting loads in flight.
__device__ inline uint4 fetch_frag(const uint4 *F, int64_t blk, int64_t ks, int part, int lane, int64_t nks)
{
    const u32x4 v = as_global(F)[frag_index(blk, ks, part, lane, nks)];
    return make_uint4(v.x, v.y, v.z, v.w);
}

template <int WM, int WN>
__device__ inline void load_frags(Frags<WM, WN> &f, const uint4 *__restrict__ Wf, const uint4 *__restrict__ Gf,
                                  int64_t tm, int64_t tn, int64_t ks, const FragDims &fm, const FragDims &fn,
                                  int lane)
{
#pragma unroll
    for (int i = 0; i < WM; ++i) {
        const int64_t mb = tm * WM + i;
#pragma unroll
        for (int part = 0; part < 2; ++part)
            f.a[i][part] = fetch_frag(Wf, mb, ks, part, lane, fm.nks);
    }
#pragma unroll
    for (int j = 0; j < WN; ++j) {
        const int64_t nb = tn * WN + j;
#pragma unroll
        for (int part = 0; part < 2; ++part)
            f.b[j][part] = fetch_frag(Gf, nb, ks, part, lane, fn.nks);
    }
}

// Wave-tile order.  Workgroups are dispatched round-robin over the 8 XCDs
// (each with its own L2), so workgroup b runs on XCD b % 8.  The tile grid is
// cut into patches of kPatch x kPatch wave tiles; XCD x works through patches
// x, x + 8, x + 16, ... and the 16 workgroups (64 waves) of a patch share its
// bin tiles and pixel tiles through that XCD's L2.
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
    *tn = pj * kPatch + in / kPatch;  // the same for the four waves of a workgroup
    return *tn < tiles_n;             // uniform over the workgroup; tm may lie past the last tile
}

// Number of workgroups that covers every patch in the XCD-striped order.
__host__ inline int64_t patch_grid(int64_t tiles_m, int64_t tiles_n)
{
    const int64_t pm = (tiles_m + kPatch - 1) / kPatch, pn = (tiles_n + kPatch - 1) / kPatch;
    const int64_t patches = pm * pn;
    const int64_t per_xcd = (patches + kXcds - 1) / kXcds;
    return per_xcd * kWgPerPatch * kXcds;
}

// 4 x 4 wave tiles (256 accumulators) leave no registers for staging: each wave
// reads both operands straight from L2, one K-step ahead in registers.
template <int WM, int WN>
__device__ inline void beam_wave_tile_direct(const BJob &jb, int64_t tm, int64_t tn, int lane)
{
    const FragDims fm = jb.fm, fn = jb.fn;
    const int64_t nks = fm.nks;
    f32x16 acc[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

    Frags<WM, WN> cur, nxt;
    load_frags<WM, WN>(cur, jb.Wf, jb.Gf, tm, tn, 0, fm, fn, lane);
    for (int64_t ks = 0; ks < nks; ++ks) {
        if (ks + 1 < nks) load_frags<WM, WN>(nxt, jb.Wf, jb.Gf, tm, tn, ks + 1, fm, fn, lane);
        // lo.hi, then hi.lo, then hi.hi: smallest terms first, fixed order
#pragma unroll
        for (int part = 0; part < 3; ++part)
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int j = 0; j < WN; ++j) {
                    const bf16x8 av = __builtin_bit_cast(bf16x8, cur.a[i][part == 0 ? 1 : 0]);
                    const bf16x8 bv = __builtin_bit_cast(bf16x8, cur.b[j][part == 1 ? 1 : 0]);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[i][j], 0, 0, 0);
                }
        if (ks + 1 < nks) cur = nxt;
    }

    // Accumulator layout of the 32x32 MFMA: lane l holds column l % 32 and rows
    // 8 (r / 4) + 4 (l / 32) + r % 4 for r = 0..15.
#pragma unroll
    for (int j = 0; j < WN; ++j) {
        const int64_t n = (tn * WN + j) * kBlk + (lane & 31);
        if (n >= jb.ncol) continue;
        int64_t nB = -1;
        if (jb.nside > 0) nB = antipode_north(ring_of_north(n, jb.nside), jb.npix);
#pragma unroll
        for (int i = 0; i < WM; ++i) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t m = (tm * WM + i) * kBlk + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                if (m >= jb.nf) continue;
                // streaming stores: the map is not read back here, and the
                // whole grid writes at once when its tiles end together
                float *row = jb.Gam + m * (int64_t)jb.npix;
                __builtin_nontemporal_store(acc[i][j][r], &row[n]);
                if (nB >= 0) __builtin_nontemporal_store(acc[i][j][r], &row[nB]);
            }
        }
    }
}

constexpr int kVmcnt0 = 0x0F70;  // s_waitcnt vmcnt(0), expcnt and lgkmcnt left at their maxima
constexpr int kVmcnt2 = 0x0F72;  // s_waitcnt vmcnt(2)

// The pixel-side fragments of one K-step for the workgroup's column tile tn
// (2 WN fragments of 64 x 16 B: blocks tn WN + j, hi and lo), copied global ->
// LDS directly into slot part WN + j (the hi parts, which the first products
// use, first); wave w moves fragments w, w + 4, ... (the same number per wave;
// the padding blocks past the last are zero).
template <int WN>
__device__ inline void stage_bfrags(const uint4 *__restrict__ Gf, int64_t tn, int64_t ks, const FragDims &fn,
                                    int wave, int lane, uint4 (*dst)[64])
{
    static_assert(2 * WN % kWavesPerWg == 0, "every wave moves the same number of fragments");
#pragma unroll
    for (int r = 0; r < 2 * WN / kWavesPerWg; ++r) {
        const int f = wave + r * kWavesPerWg;
        const int j = f / 2, part = f % 2;
        __builtin_amdgcn_global_load_lds(Gf + frag_index(tn * WN + j, ks, part, lane, fn.nks), &dst[part * WN + j][0],
                                         16, 0, 0);
    }
}

// One wave's (WM x 32) x (WN x 32) tile.  The four waves of a workgroup share
// the column tile tn (the patch order makes it uniform), so its fragments are
// staged once per K-step in LDS (three distinct buffers, K loop unrolled by
// three, so that reads of one need not wait for the copies into the others);
// each wave reads its own bin-side fragments from L2, one K-step ahead in
// registers.  Every wave of the workgroup runs the K loop (it holds
// barriers): a wave whose bin tile lies past the last multiplies the last
// tile's fragments and stores nothing.
template <int WM, int WN>
__device__ inline void beam_wave_tile(const BJob &jb, int64_t tm, int64_t tn, int lane, uint4 (*Bs0)[64],
                                      uint4 (*Bs1)[64], uint4 (*Bs2)[64])
{
    const FragDims fm = jb.fm, fn = jb.fn;
    const int64_t nks = fm.nks;
    const int wave = threadIdx.x >> 6;
    f32x16 acc[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

    // a wave past the last bin tile multiplies the last tile's fragments
    const int64_t tml = min(tm, (fm.nblk + WM - 1) / WM - 1);
    uint4 a[WM][2], an[WM][2];
    auto load_a = [&](int64_t ks, uint4 (&d)[WM][2]) {
#pragma unroll
        for (int i = 0; i < WM; ++i) {
            const int64_t mb = tml * WM + i;
#pragma unroll
            for (int part = 0; part < 2; ++part)
                d[i][part] = fetch_frag(jb.Wf, mb, ks, part, lane, fm.nks);
        }
    };
    __syncthreads();  // the previous tile's readers of the buffers are done
    load_a(0, a);
    stage_bfrags<WN>(jb.Gf, tn, 0, fn, wave, lane, Bs0);
    if (nks > 1) stage_bfrags<WN>(jb.Gf, tn, 1, fn, wave, lane, Bs1);
    __builtin_amdgcn_s_waitcnt(kVmcnt0);
    __syncthreads();
    // Three pixel-side buffers: step ks reads Bcur (K-step ks) while the copy
    // of K-step ks + 2 goes into Bnext2 (read last in step ks - 1, before the
    // previous barrier); the bin-side fragments of ks + 1 are loaded first, so
    // waiting until only that step's own copies (kStageOps per wave, issued
    // last) are in flight leaves everything of ks + 1 landed.
    constexpr int kStageOps = (2 * WN + kWavesPerWg - 1) / kWavesPerWg;
    static_assert(kStageOps == 2, "the wait below counts two copies per wave");
    auto step = [&](int64_t ks, uint4 (*Bcur)[64], uint4 (*Bnext2)[64]) {
        // past the end the loads repeat the last K-step into registers and a
        // buffer that nothing reads any more, so every step issues the same
        // operations and the wait below is one fixed count
        load_a(min(ks + 1, nks - 1), an);
        stage_bfrags<WN>(jb.Gf, tn, min(ks + 2, nks - 1), fn, wave, lane, Bnext2);
        __builtin_amdgcn_sched_barrier(0);  // the loads go out before the products
        // hi parts first: the first products (lo.hi) need only those
        uint4 b[WN][2];
#pragma unroll
        for (int part = 0; part < 2; ++part)
#pragma unroll
            for (int j = 0; j < WN; ++j) b[j][part] = Bcur[part * WN + j][lane];
        // lo.hi, then hi.lo, then hi.hi: smallest terms first, fixed order
#pragma unroll
        for (int part = 0; part < 3; ++part)
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int j = 0; j < WN; ++j) {
                    const bf16x8 av = __builtin_bit_cast(bf16x8, a[i][part == 0 ? 1 : 0]);
                    const bf16x8 bv = __builtin_bit_cast(bf16x8, b[j][part == 1 ? 1 : 0]);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[i][j], 0, 0, 0);
                }
#pragma unroll
        for (int i = 0; i < WM; ++i) {
            a[i][0] = an[i][0];
            a[i][1] = an[i][1];
        }
        // the next K-step's fragments have landed (those of ks + 2 may still
        // fly); the reads of Bcur are done before any wave copies into it again
        __builtin_amdgcn_sched_barrier(0);  // the wait stays after the products
        __builtin_amdgcn_s_waitcnt(kVmcnt2);
        asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
    };
    int64_t ks = 0;
    for (; ks + 3 <= nks; ks += 3) {
        step(ks, Bs0, Bs2);
        step(ks + 1, Bs1, Bs0);
        step(ks + 2, Bs2, Bs1);
    }
    if (ks < nks) step(ks, Bs0, Bs2);
    if (ks + 1 < nks) step(ks + 1, Bs1, Bs0);
    __builtin_amdgcn_s_waitcnt(kVmcnt0);  // the repeated copies of the last steps

    // Accumulator layout of the 32x32 MFMA: lane l holds column l % 32 and rows
    // 8 (r / 4) + 4 (l / 32) + r % 4 for r = 0..15.
#pragma unroll
    for (int j = 0; j < WN; ++j) {
        const int64_t n = (tn * WN + j) * kBlk + (lane & 31);
        if (n >= jb.ncol) continue;
        int64_t nB = -1;
        if (jb.nside > 0) nB = antipode_north(ring_of_north(n, jb.nside), jb.npix);
#pragma unroll
        for (int i = 0; i < WM; ++i) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t m = (tm * WM + i) * kBlk + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                if (m >= jb.nf) continue;
                // streaming stores: the map is not read back here, and the
                // whole grid writes at once when its tiles end together
                float *row = jb.Gam + m * (int64_t)jb.npix;
                __builtin_nontemporal_store(acc[i][j][r], &row[n]);
                if (nB >= 0) __builtin_nontemporal_store(acc[i][j][r], &row[nB]);
            }
        }
    }
}

template <int WM, int WN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WM == 2 ? 2 : 1))) void beam_gemm_kernel(BJob jb)
{
    static_assert(kTileBlocks % WM == 0 && kTileBlocks % WN == 0, "wave tiles stay inside the padded arrays");
    __shared__ uint4 Bs0[2 * WN][64], Bs1[2 * WN][64], Bs2[2 * WN][64];
    const int64_t tiles_m = (jb.fm.nblk + WM - 1) / WM;
    const int64_t tiles_n = (jb.fn.nblk + WN - 1) / WN;
    int64_t tm, tn;
    if (!patch_tile(blockIdx.x, threadIdx.x >> 6, tiles_m, tiles_n, &tm, &tn)) return;
    if constexpr (WM == 4) {
        if (tm < tiles_m) beam_wave_tile_direct<WM, WN>(jb, tm, tn, threadIdx.x & 63);
    } else {
        beam_wave_tile<WM, WN>(jb, tm, tn, threadIdx.x & 63, Bs0, Bs1, Bs2);
    }
}

// Persistent multi-job form: workgroup g of the concatenated per-job patch
// grids (each job's range starts at a multiple of 8 workgroups, so the XCD
// striping of every job is kept when the grid size is a multiple of 8).
template <int WM, int WN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WM == 2 ? 2 : 1))) void beam_gemm_batched_kernel(const BJob *__restrict__ jobs, int32_t njobs,
                                                                int64_t nwg)
{
    __shared__ uint4 Bs0[2 * WN][64], Bs1[2 * WN][64], Bs2[2 * WN][64];
    for (int64_t g = blockIdx.x; g < nwg; g += gridDim.x) {
        int j = 0;
        while (j + 1 < njobs && g >= jobs[j + 1].wg_begin) ++j;
        const BJob &jb = jobs[j];
        const int64_t tiles_m = (jb.fm.nblk + WM - 1) / WM;
        const int64_t tiles_n = (jb.fn.nblk + WN - 1) / WN;
        int64_t tm, tn;
        if (patch_tile(g - jb.wg_begin, threadIdx.x >> 6, tiles_m, tiles_n, &tm, &tn)) {
            if constexpr (WM == 4) {
                if (tm < tiles_m) beam_wave_tile_direct<WM, WN>(jb, tm, tn, threadIdx.x & 63);
            } else {
                beam_wave_tile<WM, WN>(jb, tm, tn, threadIdx.x & 63, Bs0, Bs1, Bs2);
            }
        }
    }
}

size_t beam_workspace_bytes(int32_t nt, int32_t nf, int32_t ncol)
{
    const FragDims fm = frag_dims(nf, nt), fn = frag_dims(ncol, nt);
    return (size_t)(padded_blocks(fm.nblk) + padded_blocks(fn.nblk)) * (size_t)fm.nks * 2 * 64 * sizeof(uint4);
}

void fill_bjob(BJob *jb, const MapArgs &a, const float *w, const float *gamma, float *Gam, void *work)
{
    const bool pair = a.nside > 0;
    jb->ncol = pair ? a.npix / 2 : a.npix;
    jb->fm = frag_dims(a.nf, a.nt);
    jb->fn = frag_dims(jb->ncol, a.nt);
    jb->Wf = reinterpret_cast<uint4 *>(work);
    jb->Gf = const_cast<uint4 *>(jb->Wf) + padded_blocks(jb->fm.nblk) * jb->fm.nks * 2 * 64;
    jb->nf = a.nf;
    jb->npix = a.npix;
    jb->nside = pair ? a.nside : 0;
    jb->Gam = Gam;
    jb->w = w;
    jb->gamma = gamma;
    jb->ldw = a.ldc;
    jb->nt = a.nt;
    jb->wg_begin = 0;
}

int64_t bjob_workgroups(const BJob &jb, int shape)
{
    const int wm = shape == kBeamShape2x4 ? 2 : 4, wn = 4;
    return patch_grid((jb.fm.nblk + wm - 1) / wm, (jb.fn.nblk + wn - 1) / wn);
}

hipError_t launch_beam_prep(const BJob &jb, hipStream_t s)
{
    // the padding blocks are written too (their columns lie past the data: zeros)
    const FragDims pm{padded_blocks(jb.fm.nblk), jb.fm.nks}, pn{padded_blocks(jb.fn.nblk), jb.fn.nks};
    const int64_t nw = pm.nblk * pm.nks * 64, ng = pn.nblk * pn.nks * 64;
    hipLaunchKernelGGL(prep_frag_kernel<false>, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s, jb.w, jb.ldw,
                       jb.nt, (int64_t)jb.nf, pm, const_cast<uint4 *>(jb.Wf));
    hipLaunchKernelGGL(prep_frag_kernel<true>, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, s, jb.gamma,
                       (int64_t)jb.npix, jb.nt, jb.ncol, pn, const_cast<uint4 *>(jb.Gf));
    return hipGetLastError();
}

hipError_t launch_beam_gemm(const BJob &jb, int shape, hipStream_t s)
{
    const unsigned grid = (unsigned)bjob_workgroups(jb, shape);
    if (shape == kBeamShape2x4)
        hipLaunchKernelGGL((beam_gemm_kernel<2, 4>), dim3(grid), dim3(256), 0, s, jb);
    else
        hipLaunchKernelGGL((beam_gemm_kernel<4, 4>), dim3(grid), dim3(256), 0, s, jb);
    return hipGetLastError();
}

hipError_t launch_beam_gemm_batched(const BJob *jobs_dev, int32_t njobs, int64_t nwg, int64_t grid, int shape,
                                    hipStream_t s)
{
    if (shape == kBeamShape2x4)
        hipLaunchKernelGGL((beam_gemm_batched_kernel<2, 4>), dim3((unsigned)grid), dim3(256), 0, s, jobs_dev, njobs,
                           nwg);
    else
        hipLaunchKernelGGL((beam_gemm_batched_kernel<4, 4>), dim3((unsigned)grid), dim3(256), 0, s, jobs_dev, njobs,
                           nwg);
    return hipGetLastError();
}

hipError_t launch_beam_bf16x3(const MapArgs &a, const float *w, const float *gamma, float *Gam, void *work,
                              int shape, hipStream_t s)
{
    BJob jb;
    fill_bjob(&jb, a, w, gamma, Gam, work);
    hipError_t e = launch_beam_prep(jb, s);
    if (e != hipSuccess) return e;
    return launch_beam_gemm(jb, shape, s);
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

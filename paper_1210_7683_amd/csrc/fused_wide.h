// The two-piece split-BF16 fused contraction + solve with wide per-wave
// register blocks (p <= 4).
//
// Each wave holds 2 x 4 blocks of 16 x 16 problems (32 SNPs x 64 traits) for
// all p+1 sums (160 FP32 accumulators at p = 4) and reads 4 SNP-side and
// 8 (p+1) trait-side fragments per 32-sample stage for 24 (p+1) MFMAs, where
// the 2 x 2 blocks of dma_tile read 24 fragments for 60 MFMAs; the split of
// x'^2, formed in registers from the staged pieces of x' (square_split), costs
// VALU work per SNP fragment, so the wider trait side also halves it per MFMA.
// A workgroup of 8 waves (two per SIMD) computes 256 SNPs x 64 traits.
//
// Staging: both operands go to LDS by direct global->LDS loads (lds_dma16),
// each block one contiguous 1 KB copy of the fragment-ordered planes, into two
// stage buffers that are distinct LDS objects, so the compiler can tell the
// buffer being filled from the one being read and its own LDS reads need no
// wait for the copies in flight: plain loads, scheduled between the MFMAs. Per
// stage: wait for this wave's copies of the stage, barrier (every wave's copies
// landed, every wave done with the other buffer), issue the next stage's
// copies into the other buffer, compute from this one.
//
// Each problem's sums take the same MFMAs in the same order as in dma_tile
// (per stage: lo*hi, hi*lo, hi*hi), so b is bitwise that of the other tiles.
#pragma once

#include "fused.h"
#include "lds_dma.h"

namespace gw {

// 8 waves of 2 x 4 blocks: 256 SNPs x 64 traits per workgroup (measured at
// n = 1000, p = 4, m = 1e5 against 4 x 1 waves of 4 x 3 and 4 x 2 blocks,
// 4 x 2 waves of 4 x 2 and 2 x 2, 2 x 2 waves of 4 x 2, 8 x 1 waves of 2 x 2
// and 2 x 3: 2.85 ms against 2.98-3.86 ms).
template <int P>
struct WideCfg {
    static constexpr int WM = 8, WN = 1, FM = 2, FN = 4;
    static constexpr int NW = WM * WN;
    static constexpr int NT = 64 * NW;
    static constexpr int TM = WM * FM * 16, TN = WN * FN * 16;
    static constexpr int NQ = P + 1;
    static constexpr int GA = 2 * (TM / 16);                 // SNP blocks of a stage: hi, lo planes
    static constexpr int GB = 2 * NQ * (TN / 16);            // trait blocks: hi, lo of each sum's panel
    static constexpr int BLK = GA + GB;
    static constexpr int STAGE = BLK * 1024;
    static constexpr int LPW = (BLK + NW - 1) / NW;          // block copies per wave and stage
    static_assert(2 * STAGE <= 160 * 1024, "two stages must fit a CU's LDS");
};

// One tile with the two stage buffers buf0, buf1 (distinct LDS objects). The
// planes are fragment-ordered (bf_frag_index), so every block is a contiguous
// 1 KB copy: a wave-uniform source (the 16-row or 16-trait group, clamped to
// the last group in range; a.i0 + m_base is a multiple of 16) plus 16 bytes per
// lane. Rows and traits past the range only feed outputs that are never stored.
template <int P>
__device__ __forceinline__ void wide_tile(const FusedArgs &a, int64_t m_base, int n_base, uint8_t *buf0,
                                          uint8_t *buf1) {
    using C = WideCfg<P>;
    constexpr int NQ = C::NQ, TM = C::TM, TN = C::TN, FM = C::FM, FN = C::FN, GA = C::GA;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave % C::WM, wn = wave / C::WM;
    const int l16 = lane & 15, g = lane >> 4;

    const int nkg = a.n_pad / 32;                             // 32-sample groups per row
    // one group per stage, up to the pair holding sample n - 1 (the rest of
    // the row is zeros); even, at most nkg (n_pad % 64 == 0)
    const int nstages = 2 * ((a.n + 63) / 64);
    const int64_t a_plane = a.a_plane_rows * (int64_t)a.n_pad * 2;
    const int64_t b_plane = (int64_t)a.tcap * a.n_pad * 2;
    const int64_t g0 = (a.i0 + m_base) / 16, g_last = (a.i0 + a.mi - 1) / 16;
    const int t0 = n_base / 16, t_last = (a.tb - 1) / 16;

    // Block b = wave + NW u of a stage: a SNP block (plane b / (TM/16), row group
    // b mod (TM/16)) for b < GA, else a trait block (plane, 16-trait group).
    auto issue = [&](int c, uint8_t *buf) {
#pragma unroll
        for (int u = 0; u < C::LPW; ++u) {
            const int blk = wave + u * C::NW;
            if (blk >= C::BLK) continue;
            const uint8_t *src;
            if (blk < GA) {
                const int pl = blk / (TM / 16), rg = blk % (TM / 16);
                src = (const uint8_t *)a.a + pl * a_plane + (min(g0 + rg, g_last) * nkg + c) * 1024;
            } else {
                const int pl = (blk - GA) / (TN / 16), cg = (blk - GA) % (TN / 16);
                src = (const uint8_t *)a.panels + pl * b_plane + ((int64_t)min(t0 + cg, t_last) * nkg + c) * 1024;
            }
            lds_dma16(src + lane * 16, buf + blk * 1024);
        }
    };

    f4 acc[NQ][FM][FN];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int x = 0; x < FM; ++x)
#pragma unroll
            for (int y = 0; y < FN; ++y) acc[q][x][y] = f4{0, 0, 0, 0};

    auto stage = [&](int c, const uint8_t *cur, uint8_t *nxt) {
        __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));   // this wave's copies of stage c landed
        __syncthreads();                            // ... every wave's; every wave is done with nxt
        if (c + 1 < nstages) issue(c + 1, nxt);
        const uint8_t *base = cur + lane * 16;
        bf16x8 xh[FM], xl[FM], sh[FM], sl[FM];
#pragma unroll
        for (int x = 0; x < FM; ++x) {
            xh[x] = *(const bf16x8 *)(base + (wm * FM + x) * 1024);
            xl[x] = *(const bf16x8 *)(base + (TM / 16 + wm * FM + x) * 1024);
            square_split(xh[x], xl[x], sh[x], sl[x]);
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            bf16x8 bh[FN], bl[FN];
#pragma unroll
            for (int y = 0; y < FN; ++y) {
                bh[y] = *(const bf16x8 *)(base + (GA + (2 * q) * (TN / 16) + wn * FN + y) * 1024);
                bl[y] = *(const bf16x8 *)(base + (GA + (2 * q + 1) * (TN / 16) + wn * FN + y) * 1024);
            }
#pragma unroll
            for (int x = 0; x < FM; ++x) {
                // q = 0 pairs the split square with the weights; q >= 1 the split value
                const bf16x8 ah = q == 0 ? sh[x] : xh[x], al = q == 0 ? sl[x] : xl[x];
#pragma unroll
                for (int y = 0; y < FN; ++y) {
                    f4 v = acc[q][x][y];
                    v = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[y], v, 0, 0, 0);
                    v = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[y], v, 0, 0, 0);
                    acc[q][x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[y], v, 0, 0, 0);
                }
            }
        }
    };

    issue(0, buf0);
    for (int c = 0; c < nstages; c += 2) {
        stage(c, buf0, buf1);
        stage(c + 1, buf1, buf0);
    }
    fused_epilogue<GWAS_FORM_BF16X3, P, FM, FN>(
        a, [&](int q, int x, int y, int r) { return (double)acc[q][x][y][r]; }, m_base, n_base, wm, wn, l16, g);
}

template <int P>
__global__ __launch_bounds__(WideCfg<P>::NT) void fused_bf16_wide_kernel(FusedArgs a) {
    using C = WideCfg<P>;
    __shared__ __attribute__((aligned(1024))) uint8_t buf0[C::STAGE];
    __shared__ __attribute__((aligned(1024))) uint8_t buf1[C::STAGE];
    const int ntn = (a.tb + C::TN - 1) / C::TN;
    const int64_t ntm = (a.mi + C::TM - 1) / C::TM;
    const int64_t tile = tile_order(blockIdx.x, ntm, ntn);
    wide_tile<P>(a, (tile / ntn) * C::TM, (int)(tile % ntn) * C::TN, buf0, buf1);
}

template <int P>
hipError_t launch_bf16_wide(const FusedArgs &a, hipStream_t s) {
    using C = WideCfg<P>;
    if (a.mi <= 0 || a.tb <= 0) return hipSuccess;
    if (a.n_pad % 64 || a.i0 % 16 || a.tcap % 16) return hipErrorInvalidValue;
    const int64_t tiles = ((a.mi + C::TM - 1) / C::TM) * ((a.tb + C::TN - 1) / C::TN);
    hipLaunchKernelGGL((fused_bf16_wide_kernel<P>), dim3((unsigned)tiles), dim3(C::NT), 0, s, a);
    return hipGetLastError();
}

}  // namespace gw

// The fused contraction + solve of fused.h with the operands staged by direct
// global->LDS loads (global_load_lds_dwordx4), for all four forms.
//
// LDS layout: the staging buffer is a sequence of 1 KB blocks, each holding one
// MFMA operand fragment in lane order: lane l of a wave owns bytes
// 16 l .. 16 l + 15, which are bytes 16 (l / 16) .. + 15 of a 64-byte group of
// operand row l % 16. One wave-wide 16-byte load fills a block (64 lanes x 16
// bytes), and the wave that consumes it reads the same 16 bytes per lane back
// with one ds_read_b128: no staging registers, no LDS bank conflicts, no
// ds_write. A 64-byte group holds 8 doubles, 16 floats or 32 bf16 per row, so
// the 16 bytes of lane l are 2, 4 or 8 consecutive samples; lane l supplies
// them as the k = l / 16 element of 2 (FP64), 4 (FP32) or 1 (BF16, k-block of
// 8) MFMAs, the same way for both operands, so every product pairs equal k.
//
// One stage holds KB groups of every operand row (KB * 64 bytes per row). With
// one LDS buffer the loop per stage is: wait for the stage's loads, barrier,
// read the fragments of the whole stage into registers, barrier, issue the
// next stage's loads into the same LDS (they run under this stage's MFMAs),
// compute. With two (PIPE): wait, barrier, issue the next stage's loads into
// the other buffer, read this stage's fragments (inline-assembly reads, see
// lds_dma.h), compute.
//
// Split BF16: only the pieces of x' are staged (hi, lo; or hi, mid, lo); the
// split of x'^2 is formed from them in registers (square_split,
// square_split3), which halves the SNP-side bytes. Their planes are stored in
// fragment order (bf_frag_index), so every block is one contiguous 1 KB copy.
// FP64 folds (FLUSH): FP32 accumulators are added to FP64 sums at the end of
// each window and the next window's first MFMA starts from zero. FP32 form
// (KB = 2, 8 MFMAs of 4 samples per sum and stage): b_B, the sum that cancels,
// in four chains per stage, one per MFMA slot e of the two 16-sample groups, so
// each chain adds 8 products in 2 MFMAs (the rounding of 8-sample windows); the
// chains run one after another after the stage's other MFMAs, each folded as
// it ends, so one chain is live at a time; the other p sums in windows of
// kF32LongWindow stages. Three-piece BF16 (KB = 1): every sum in windows of
// one stage (32 samples).
#pragma once

#include "fused.h"
#include "lds_dma.h"

namespace gw {

template <int WM_, int WN_, int FM_, int FN_, int KB_, bool PIPE_ = false, bool PERSIST_ = false>
struct DmaTile {
    static constexpr int WM = WM_, WN = WN_, FM = FM_, FN = FN_, KB = KB_;
    static constexpr bool PIPE = PIPE_;       // two LDS buffers
    static constexpr bool PERSIST = PERSIST_; // persistent workgroups, one per CU
};

template <int FORM, int P, class T>
struct DmaCfg {
    static constexpr int WM = T::WM, WN = T::WN, FM = T::FM, FN = T::FN, KB = T::KB;
    static constexpr bool BF6 = FORM == GWAS_FORM_BF16X6;
    static constexpr bool BF = FORM == GWAS_FORM_BF16X3 || BF6;
    static constexpr int PIECES = FORM == GWAS_FORM_BF16X3 ? 2 : (BF6 ? 3 : 1);   // BF16 pieces per value
    static constexpr int NW = WM * WN;
    static constexpr int NT = 64 * NW;
    static constexpr int TM = WM * FM * 16, TN = WN * FN * 16;
    static constexpr int NQ = P + 1;
    static constexpr int ESZ = FORM == GWAS_FORM_F64 ? 8 : (FORM == GWAS_FORM_F32 ? 4 : 2);
    static constexpr int NA = PIECES;                   // staged SNP-side planes
    static constexpr int NB = PIECES * NQ;              // staged trait-side planes
    static constexpr int GA = NA * (TM / 16);           // blocks of one 64-byte group
    static constexpr int GBK = GA + NB * (TN / 16);
    static constexpr int BLK = KB * GBK;                // blocks per stage
    static constexpr bool PIPE = T::PIPE;
    static constexpr int LDS = (PIPE ? 2 : 1) * BLK * 1024;
    static constexpr int LPW = (BLK + NW - 1) / NW;     // block loads per wave and stage
    static_assert(KB == 1 || KB == 2, "one or two 64-byte groups per stage");
    static_assert(LDS <= 160 * 1024, "LDS stage too large");
    // the fragments one wave reads per stage, in order: per group kb, the SNP
    // fragments (plane, x) then the trait fragments (plane, y); offsets are
    // from the wave's SNP base (stage + lane * 16 + wm * FM KB) or trait base
    // (stage + lane * 16 + (GA + wn * FN) KB)
    static constexpr int NBP = NB;
    static constexpr int NFA = NA * FM, NFK = NFA + NBP * FN, NF = KB * NFK;
    static constexpr bool frag_is_b(int i) { return (i % NFK) >= NFA; }
    static constexpr int frag_off(int i) {
        return (i % NFK) < NFA
                   ? ((i / NFK) * GBK + ((i % NFK) / FM) * (TM / 16) + (i % NFK) % FM) * 1024
                   : ((i / NFK) * GBK + (((i % NFK) - NFA) / FN) * (TN / 16) + ((i % NFK) - NFA) % FN) * 1024;
    }
    static_assert(!PIPE || BLK * 1024 <= 65536, "fragment offsets must fit the 16-bit LDS offset field");
};


template <int FORM>
struct DmaFrag;
template <> struct DmaFrag<GWAS_FORM_F64> { using type = double2; using acc = d4; };
template <> struct DmaFrag<GWAS_FORM_F32> { using type = float4; using acc = f4; };
template <> struct DmaFrag<GWAS_FORM_BF16X3> { using type = bf16x8; using acc = f4; };
template <> struct DmaFrag<GWAS_FORM_BF16X6> { using type = bf16x8; using acc = f4; };

// FP32 form: stages (32 samples each) per FP64 fold window of the sums other than b_B
constexpr int kF32LongWindow = 2;

// One TM x TN tile of problems (tile index over the tiles of a, traits fastest),
// computed by a whole workgroup of C::NT threads with `lds` (C::LDS bytes,
// 1 KB aligned) as its staging memory. Every thread of the workgroup calls it
// with the same arguments (it contains workgroup barriers); on return all of
// its global->LDS loads have completed and its LDS is no longer read.
template <int FORM, int P, bool FLUSH, class T>
__device__ __forceinline__ void dma_tile(const FusedArgs &a, int64_t tile, uint8_t *lds) {
    using C = DmaCfg<FORM, P, T>;
    using frag = typename DmaFrag<FORM>::type;
    using acc_t = typename DmaFrag<FORM>::acc;
    constexpr int NQ = C::NQ, TM = C::TM, TN = C::TN, FM = C::FM, FN = C::FN, KB = C::KB, NA = C::NA;
    constexpr bool BF = C::BF;
    static_assert(!FLUSH || (FORM == GWAS_FORM_F32 && KB == 2) || (FORM == GWAS_FORM_BF16X6 && KB == 1),
                  "the FP64 fold is per 32-sample stage");

    const int ntn = (a.tb + TN - 1) / TN;
    const int tn = (int)(tile % ntn);
    const int64_t tm = tile / ntn;
    const int64_t m_base = tm * TM;
    const int n_base = tn * TN;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform
    const int wm = wave % C::WM, wn = wave / C::WM;
    const int l16 = lane & 15, g = lane >> 4;

    const int64_t row_bytes = (int64_t)a.n_pad * C::ESZ;
    // stages up to the one holding sample n - 1 (the rest of the row is zeros)
    const int nstages = (int)(((int64_t)a.n * C::ESZ + KB * 64 - 1) / (KB * 64));
    const uint8_t *A = (const uint8_t *)a.a;
    const uint8_t *B = (const uint8_t *)a.panels;
    const int64_t a_plane = a.a_plane_rows * row_bytes;
    const int64_t b_plane = (int64_t)a.tcap * row_bytes;

    // Source of every block this wave loads: a wave-uniform base (plane, tile
    // origin, group) plus a per-lane 32-bit offset (row within the tile, lane
    // group), so the loads use scalar base addresses and the stage advance is
    // scalar arithmetic. Block b of a stage is group kb = b / GBK; within the
    // group, blocks [0, GA) are the SNP planes (plane-major, 16-row groups), the
    // rest the trait planes. Rows past the tile's range are clamped into it:
    // they only feed outputs that are never stored.
    // The split-BF16 planes are fragment-ordered (bf_frag_index): a block is one
    // contiguous 1 KB source, the 16-row (16-trait) group clamped to the last
    // group in range (a.i0 + m_base is a multiple of 16, see launch_fused), the
    // same per-lane offset for every block, and a stage advances by KB blocks.
    const int nkg = a.n_pad / 32;
    const uint8_t *sbase[C::LPW];
    uint32_t voff[C::LPW];
#pragma unroll
    for (int u = 0; u < C::LPW; ++u) {
        const int blk = wave + u * C::NW;
        sbase[u] = A;
        voff[u] = 0;
        if (blk < C::BLK) {
            const int kb = blk / C::GBK, r = blk % C::GBK;
            if (r < C::GA) {
                const int pl = r / (TM / 16), rg = r % (TM / 16);
                if constexpr (BF) {
                    const int64_t grp = min((a.i0 + m_base) / 16 + rg, (a.i0 + a.mi - 1) / 16);
                    sbase[u] = A + pl * a_plane + (grp * nkg + kb) * 1024;
                    voff[u] = lane * 16;
                } else {
                    int64_t i = m_base + rg * 16 + l16;
                    if (i >= a.mi) i = a.mi - 1;
                    sbase[u] = A + pl * a_plane + (a.i0 + m_base) * row_bytes + kb * 64;
                    voff[u] = (uint32_t)((i - m_base) * row_bytes) + g * 16;
                }
            } else {
                const int rb = r - C::GA;
                const int pl = rb / (TN / 16), cg = rb % (TN / 16);
                if constexpr (BF) {
                    const int grp = min(n_base / 16 + cg, (a.tb - 1) / 16);
                    sbase[u] = B + pl * b_plane + ((int64_t)grp * nkg + kb) * 1024;
                    voff[u] = lane * 16;
                } else {
                    int j = n_base + cg * 16 + l16;
                    if (j >= a.tb) j = a.tb - 1;
                    sbase[u] = B + pl * b_plane + (int64_t)n_base * row_bytes + kb * 64;
                    voff[u] = (uint32_t)((j - n_base) * row_bytes) + g * 16;
                }
            }
        }
    }
    constexpr int STAGE_STRIDE = BF ? KB * 1024 : KB * 64;   // source bytes from one stage to the next
    auto issue = [&](int c) {
        uint8_t *stage = lds + (C::PIPE ? (c & 1) * (C::BLK * 1024) : 0);
#pragma unroll
        for (int u = 0; u < C::LPW; ++u) {
            const int blk = wave + u * C::NW;
            if (blk < C::BLK) lds_dma16(sbase[u] + (int64_t)c * STAGE_STRIDE + voff[u], stage + blk * 1024);
        }
    };
    auto afrag = [&](int kb, int plane, int x) -> frag {
        return *(const frag *)(lds + (kb * C::GBK + plane * (TM / 16) + wm * FM + x) * 1024 + lane * 16);
    };
    auto bfrag = [&](int kb, int plane, int y) -> frag {
        return *(const frag *)(lds + (kb * C::GBK + C::GA + plane * (TN / 16) + wn * FN + y) * 1024 + lane * 16);
    };

    acc_t acc[NQ][FM][FN];
    d4 acc64[FLUSH ? NQ : 1][FLUSH ? FM : 1][FLUSH ? FN : 1];
    // FP32 with FLUSH: b_B in four chains per stage (MFMA slot e), each run
    // and folded on its own after the stage's other MFMAs
    constexpr bool SPLIT_BB = FLUSH && FORM == GWAS_FORM_F32;
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int x = 0; x < FM; ++x)
#pragma unroll
            for (int y = 0; y < FN; ++y) {
                acc[q][x][y] = acc_t{0, 0, 0, 0};
                if constexpr (FLUSH) acc64[q][x][y] = d4{0, 0, 0, 0};
            }

    issue(0);
    for (int c = 0; c < nstages; ++c) {
        frag xa[KB][NA][FM], yb[KB][C::NBP][FN];
        if constexpr (C::PIPE) {
            // two LDS buffers, one barrier per stage: after it, stage c has
            // landed for every wave and every wave has read stage c - 1, whose
            // buffer then takes stage c + 1 while stage c is read and computed
            __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this wave's loads of stage c landed
            __syncthreads();
            if (c + 1 < nstages) issue(c + 1);
            const uint32_t sb = lds_addr(lds) + (c & 1) * (C::BLK * 1024) + lane * 16;
            i4v fr[C::NF];
            lds_read_frags<C, 0, C::NF>(fr, sb + wm * FM * 1024, sb + (C::GA + wn * FN) * 1024);
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
                for (int pl = 0; pl < NA; ++pl)
#pragma unroll
                    for (int x = 0; x < FM; ++x) xa[kb][pl][x] = __builtin_bit_cast(frag, fr[kb * C::NFK + pl * FM + x]);
#pragma unroll
                for (int pl = 0; pl < C::NBP; ++pl)
#pragma unroll
                    for (int y = 0; y < FN; ++y)
                        yb[kb][pl][y] = __builtin_bit_cast(frag, fr[kb * C::NFK + C::NFA + pl * FN + y]);
            }
        } else {
            __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this wave's loads of stage c landed
            __syncthreads();                      // ... and every other wave's
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
                for (int pl = 0; pl < NA; ++pl)
#pragma unroll
                    for (int x = 0; x < FM; ++x) xa[kb][pl][x] = afrag(kb, pl, x);
#pragma unroll
                for (int pl = 0; pl < C::NBP; ++pl)
#pragma unroll
                    for (int y = 0; y < FN; ++y) yb[kb][pl][y] = bfrag(kb, pl, y);
            }
            __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0): the fragments are in registers
            __syncthreads();                      // every wave is done with the stage
            if (c + 1 < nstages) issue(c + 1);    // the next stage's loads run under the MFMAs
        }

        // stages per window of the sums folded at stage ends
        constexpr int WS = FORM == GWAS_FORM_F32 ? kF32LongWindow : 1;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
            const bool fresh = FLUSH && kb == 0 && c % WS == 0;   // an FP32 window starts at zero
#pragma unroll
            for (int x = 0; x < FM; ++x) {
                if constexpr (FORM == GWAS_FORM_F64) {
                    const double2 xv = xa[kb][0][x];
#pragma unroll
                    for (int y = 0; y < FN; ++y) {
                        acc[0][x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(xv.x * xv.x, yb[kb][0][y].x, acc[0][x][y], 0, 0, 0);
                        acc[0][x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(xv.y * xv.y, yb[kb][0][y].y, acc[0][x][y], 0, 0, 0);
#pragma unroll
                        for (int q = 1; q < NQ; ++q) {
                            acc[q][x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(xv.x, yb[kb][q][y].x, acc[q][x][y], 0, 0, 0);
                            acc[q][x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(xv.y, yb[kb][q][y].y, acc[q][x][y], 0, 0, 0);
                        }
                    }
                } else if constexpr (FORM == GWAS_FORM_F32) {
                    const float4 xv = xa[kb][0][x];
                    const float xs[4] = {xv.x, xv.y, xv.z, xv.w};
#pragma unroll
                    for (int y = 0; y < FN; ++y) {
#pragma unroll
                        for (int q = 0; q < NQ; ++q) {
                            const float4 bv = yb[kb][q][y];
                            const float bs[4] = {bv.x, bv.y, bv.z, bv.w};
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                const float av = q == 0 ? xs[e] * xs[e] : xs[e];
                                if constexpr (SPLIT_BB) {
                                    if (q == NQ - 1) continue;   // b_B: after the kb loop
                                }
                                acc[q][x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                                    av, bs[e], (fresh && e == 0) ? acc_t{0, 0, 0, 0} : acc[q][x][y], 0, 0, 0);
                            }
                        }
                    }
                } else if constexpr (C::BF6) {
                    // x = h + m + l; six products per pair, smallest first
                    const bf16x8 xh = xa[kb][0][x], xm = xa[kb][1][x], xl = xa[kb][2][x];
                    bf16x8 sh, sm, sl;
                    square_split3(xh, xm, xl, sh, sm, sl);
#pragma unroll
                    for (int y = 0; y < FN; ++y)
#pragma unroll
                        for (int q = 0; q < NQ; ++q) {
                            const bf16x8 ah = q == 0 ? sh : xh, am = q == 0 ? sm : xm, al = q == 0 ? sl : xl;
                            const bf16x8 bh = yb[kb][3 * q][y], bm = yb[kb][3 * q + 1][y], bl = yb[kb][3 * q + 2][y];
                            f4 v = fresh ? f4{0, 0, 0, 0} : acc[q][x][y];
                            v = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, v, 0, 0, 0);
                            v = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, v, 0, 0, 0);
                            v = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bm, v, 0, 0, 0);
                            v = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bh, v, 0, 0, 0);
                            v = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bm, v, 0, 0, 0);
                            acc[q][x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, v, 0, 0, 0);
                        }
                } else {
                    const bf16x8 xh = xa[kb][0][x], xl = xa[kb][1][x];
                    bf16x8 sh, sl;
                    square_split(xh, xl, sh, sl);
#pragma unroll
                    for (int y = 0; y < FN; ++y) {
                        // q = 0 pairs the split square with the weights; q >= 1 the split value
                        acc[0][x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(sl, yb[kb][0][y], acc[0][x][y], 0, 0, 0);
                        acc[0][x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(sh, yb[kb][1][y], acc[0][x][y], 0, 0, 0);
                        acc[0][x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(sh, yb[kb][0][y], acc[0][x][y], 0, 0, 0);
#pragma unroll
                        for (int q = 1; q < NQ; ++q) {
                            acc[q][x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl, yb[kb][2 * q][y], acc[q][x][y], 0, 0, 0);
                            acc[q][x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, yb[kb][2 * q + 1][y], acc[q][x][y], 0, 0, 0);
                            acc[q][x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, yb[kb][2 * q][y], acc[q][x][y], 0, 0, 0);
                        }
                    }
                }
            }
        }
        if constexpr (SPLIT_BB) {
            // b_B: chain e = the MFMAs of slot e of both 16-sample groups (8
            // products), folded at once, so one chain is live at a time
            static_assert(KB == 2, "two groups per stage");
#pragma unroll
            for (int x = 0; x < FM; ++x) {
                const float4 x0 = xa[0][0][x], x1 = xa[1][0][x];
                const float a0[4] = {x0.x, x0.y, x0.z, x0.w}, a1[4] = {x1.x, x1.y, x1.z, x1.w};
#pragma unroll
                for (int y = 0; y < FN; ++y) {
                    const float4 y0 = yb[0][NQ - 1][y], y1 = yb[1][NQ - 1][y];
                    const float b0[4] = {y0.x, y0.y, y0.z, y0.w}, b1[4] = {y1.x, y1.y, y1.z, y1.w};
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        acc_t v = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[e], b0[e], acc_t{0, 0, 0, 0}, 0, 0, 0);
                        v = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[e], b1[e], v, 0, 0, 0);
#pragma unroll
                        for (int r = 0; r < 4; ++r) acc64[NQ - 1][x][y][r] += (double)v[r];
                    }
                }
            }
        }
        if constexpr (FLUSH) {
            if (c % WS == WS - 1 || c == nstages - 1) {   // the window ends with this stage
#pragma unroll
                for (int q = 0; q < (SPLIT_BB ? NQ - 1 : NQ); ++q)   // FP32 b_B: folded above
#pragma unroll
                    for (int x = 0; x < FM; ++x)
#pragma unroll
                        for (int y = 0; y < FN; ++y)
#pragma unroll
                            for (int r = 0; r < 4; ++r) acc64[q][x][y][r] += (double)acc[q][x][y][r];
            }
        }
    }

    if constexpr (FLUSH)
        fused_epilogue<FORM, P, FM, FN>(a, [&](int q, int x, int y, int r) { return acc64[q][x][y][r]; }, m_base,
                                        n_base, wm, wn, l16, g);
    else
        fused_epilogue<FORM, P, FM, FN>(a, [&](int q, int x, int y, int r) { return (double)acc[q][x][y][r]; },
                                        m_base, n_base, wm, wn, l16, g);
}

// One workgroup per tile. Workgroups are dispatched round-robin over the
// chip's 8 XCDs (workgroup b on XCD b mod 8), each with its own L2; with
// xcd_order, XCD x takes a contiguous eighth of the trait tiles and walks every
// SNP tile, so its trait panels stay in its L2 while the SNP rows stream.
// tile_order applies it to the largest multiple of 8 trait tiles and runs the
// rest (fewer than 8 per SNP tile) after them, all of a SNP tile's on one XCD.
template <int FORM, int P, bool FLUSH, class T>
__global__ __launch_bounds__((DmaCfg<FORM, P, T>::NT)) void fused_dma_kernel(FusedArgs a) {
    using C = DmaCfg<FORM, P, T>;
    extern __shared__ __attribute__((aligned(1024))) uint8_t lds[];
    const int ntn = (a.tb + C::TN - 1) / C::TN;
    const int64_t ntm = (a.mi + C::TM - 1) / C::TM;
    dma_tile<FORM, P, FLUSH, T>(a, tile_order(blockIdx.x, ntm, ntn), lds);
}

// Persistent variant: one workgroup per CU; workgroup b (on XCD b mod 8) takes
// the tiles x + 8 l of the order above (x = b mod 8) from its XCD's counter
// until they run out, so each XCD still covers its eighth of the trait tiles.
// Every workgroup reaches the exit once its counter passes the tile count.
template <int FORM, int P, bool FLUSH, class T>
__global__ __launch_bounds__((DmaCfg<FORM, P, T>::NT)) void fused_dma_persistent_kernel(FusedArgs a) {
    using C = DmaCfg<FORM, P, T>;
    extern __shared__ __attribute__((aligned(1024))) uint8_t lds[];
    __shared__ unsigned next;
    const int ntn = (a.tb + C::TN - 1) / C::TN;
    const int64_t ntm = (a.mi + C::TM - 1) / C::TM;
    const int64_t total = ntm * ntn;
    const int x = blockIdx.x % 8;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(a.tile_counters + x, 1u);
        __syncthreads();
        const int64_t b = (int64_t)next * 8 + x;
        __syncthreads();   // every thread has read `next` before it is overwritten
        if (b >= total) return;
        dma_tile<FORM, P, FLUSH, T>(a, tile_order(b, ntm, ntn), lds);
    }
}

// Clears the persistent launch's 8 tile counters with a kernel (a memset node
// is not what a caller capturing the stream into a graph should get).
template <int N>
__global__ void zero_words_kernel(unsigned *w) {
    if (threadIdx.x < N) w[threadIdx.x] = 0u;
}

template <int FORM, int P, bool FLUSH, class T>
hipError_t launch_dma_t(const FusedArgs &a, hipStream_t s) {
    using C = DmaCfg<FORM, P, T>;
    const int64_t tiles = ((a.mi + C::TM - 1) / C::TM) * ((a.tb + C::TN - 1) / C::TN);
    if (a.mi <= 0 || a.tb <= 0) return hipSuccess;
    if ((a.n_pad * C::ESZ) % (C::KB * 64)) return hipErrorInvalidValue;
    if (C::BF && (a.i0 % 16 || a.tcap % 16)) return hipErrorInvalidValue;   // whole fragment-ordered groups
    if constexpr (T::PERSIST) {
        if (!a.tile_counters) return hipErrorInvalidValue;
        static bool attr_set = false;   // per instantiation
        if (C::LDS > 65536 && !attr_set) {
            hipError_t e = hipFuncSetAttribute((const void *)fused_dma_persistent_kernel<FORM, P, FLUSH, T>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, C::LDS);
            if (e != hipSuccess) return e;
            attr_set = true;
        }
        int dev = 0, cus = 256;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(zero_words_kernel<8>, dim3(1), dim3(64), 0, s, a.tile_counters);
        const int64_t grid = std::max<int64_t>(8, std::min<int64_t>(cus, (tiles + 7) / 8 * 8));
        hipLaunchKernelGGL((fused_dma_persistent_kernel<FORM, P, FLUSH, T>), dim3((unsigned)grid), dim3(C::NT),
                           C::LDS, s, a);
        return hipGetLastError();
    }
    if (C::LDS > 65536) {
        static bool attr_set = false;   // per instantiation
        if (!attr_set) {
            hipError_t e = hipFuncSetAttribute((const void *)fused_dma_kernel<FORM, P, FLUSH, T>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, C::LDS);
            if (e != hipSuccess) return e;
            attr_set = true;
        }
    }
    hipLaunchKernelGGL((fused_dma_kernel<FORM, P, FLUSH, T>), dim3((unsigned)tiles), dim3(C::NT), C::LDS, s, a);
    return hipGetLastError();
}

// Per-form tiles, chosen by timing sweeps on the MI355X at n = 1000, p = 4
// (m = 1e5, t = 1000): one 16x16 block of problems per wave for FP64 and FP32,
// 32x32 per wave for split BF16 (more reuse of its larger operands). FP64 at
// m = 1e6: 8 waves in a column (128 SNPs x 16 traits) took 143.0-143.5 ms
// against 145.3-146.2 ms for 4 x 2 waves (64 x 32), 144.1-144.5 ms for 4 x 2
// waves of 32 x 16 blocks and 143.1 ms for 8 waves of 32 x 16 blocks; it is
// also 2.6% faster at p = 8 but 1.3% slower at p = 2, which keeps 4 x 2. FP32 and
// split BF16 run two LDS buffers (PIPE); for FP64 the single buffer with a
// smaller LDS footprint measured faster. Persistent workgroups measured 2-6%
// faster than one workgroup per tile for split BF16 at p <= 4 (varying
// between runs) and no faster for FP32 and FP64. Larger p narrows the split-BF16 tile,
// and from p = 10 (FP32: 12) the workgroup drops to 4 waves, one per SIMD, so
// a wave may hold up to 512 registers of p + 1 accumulator sets and fragments.
template <int FORM, int P>
struct DmaDefault {
    using F64T = typename std::conditional<(P == 2), DmaTile<4, 2, 1, 1, 1>,
                 typename std::conditional<(P <= 9), DmaTile<8, 1, 1, 1, 1>, DmaTile<4, 1, 1, 1, 1>>::type>::type;
    using F32T = typename std::conditional<(P <= 11), DmaTile<8, 1, 1, 1, 2, true>,
                                           DmaTile<4, 1, 1, 1, 2, true>>::type;
    using BF16T = typename std::conditional<(P <= 4), DmaTile<8, 1, 2, 2, 1, true, true>,
                  typename std::conditional<(P <= 9), DmaTile<8, 1, 2, 1, 1, true>,
                                            DmaTile<4, 1, 1, 1, 1, true>>::type>::type;
    // six-product form: three planes a side; the two-stage pipeline's 16-bit
    // fragment offsets bound the stage to 64 blocks
    using BF6T = typename std::conditional<(P <= 4), DmaTile<8, 1, 1, 2, 1, true>,
                 typename std::conditional<(P <= 9), DmaTile<8, 1, 1, 1, 1, true>,
                 typename std::conditional<(P <= 16), DmaTile<4, 1, 1, 1, 1, true>,
                                           DmaTile<4, 1, 1, 1, 1>>::type>::type>::type;
    using type = typename std::conditional<FORM == GWAS_FORM_F64, F64T,
                 typename std::conditional<FORM == GWAS_FORM_F32, F32T,
                 typename std::conditional<FORM == GWAS_FORM_BF16X3, BF16T, BF6T>::type>::type>::type;
};

template <int FORM, bool FLUSH>
hipError_t dispatch_dma(const FusedArgs &a, hipStream_t s) {
    switch (a.p) {
#define GW_CASE(PP) case PP: return launch_dma_t<FORM, PP, FLUSH, typename DmaDefault<FORM, PP>::type>(a, s);
        GW_CASE(2) GW_CASE(3) GW_CASE(4) GW_CASE(5) GW_CASE(6) GW_CASE(7) GW_CASE(8) GW_CASE(9)
        GW_CASE(10) GW_CASE(11) GW_CASE(12) GW_CASE(13) GW_CASE(14) GW_CASE(15) GW_CASE(16)
        GW_CASE(17) GW_CASE(18) GW_CASE(19) GW_CASE(20)
#undef GW_CASE
    default: return hipErrorInvalidValue;
    }
}

}  // namespace gw

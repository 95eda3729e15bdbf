// The fused inner loop of Algorithm 5 for a tile of (SNP, trait) problems.
//
// For every (i, j) of a TM x TN tile the p+1 length-n contractions
//   q = 0:        S_BR   = sum_k x'_ki^2   d_jk
//   q = 1..p-1:   S_BL_q = sum_k x'_ki     d_jk x'_L,k(q-1)
//   q = p:        b_B    = sum_k x'_ki     d_jk y'_kj
// are p+1 MFMA GEMM tiles that share the SNP operand (staged once per K chunk
// in LDS) and read one trait panel each. All p+1 accumulator tiles use one
// operand mapping, so the p+1 values of a problem land in the same lane and
// register slot; the epilogue is lane-local and FP64:
//   u = L_j^{-1} S_BL;  s = S_BR - u.u;  beta = (b_B - u.z_j) / s;
//   b_top = L_j^{-T} (z_j - u beta);  b_ij = [b_top; beta]
// which is the Cholesky solve of S_ij b = [b_T; b_B] (Algorithm 2's
// partitioned S_ij) with the factor of S_TL_j reused across the trait's SNPs.
//
// Forms (template FORM):
//   F64:    double operands, v_mfma_f64_16x16x4f64
//   F32:    float operands,  v_mfma_f32_16x16x4f32 (optional FP64 folding)
//   BF16X3: bf16 hi/lo operands, v_mfma_f32_16x16x32_bf16, three products
//           hi*hi + hi*lo + lo*hi per pair, FP32 accumulation
//
// K chunking: each chunk stages CB bytes of every operand row in LDS (row
// stride CB + 16 bytes, so 16-byte reads of 16 consecutive rows fall on
// distinct banks). Within a 64-byte group, lane (l16, g) of a wave reads the
// 16-byte segment g of row l16 of a 16-row fragment (2 doubles, 4 floats or 8
// bf16); the same segment->k mapping is used for both operands, so every
// product pairs equal k.
//
// fused_tile is the tile code of the persistent serving loop (register-staged
// LDS chunks); the direct solve uses the LDS-DMA kernel of fused_dma.h. Both
// end in fused_epilogue.
#pragma once

#include <type_traits>

#include "gwas_internal.h"

namespace gw {

// Tile shape of the fused kernel: WM x WN waves, each holding FM x FN 16x16
// MFMA blocks per contraction; CB bytes of every operand row staged per K
// chunk (64, 128 or 256); DB = 1 double-buffers the LDS stage (one barrier per
// chunk, the next chunk's global loads in flight during the MFMAs).
template <int WM_, int WN_, int FM_, int FN_, int CB_, int DB_>
struct Tile {
    static constexpr int WM = WM_, WN = WN_, FM = FM_, FN = FN_, CB = CB_, DB = DB_;
};

template <int FORM, int P, class T>
struct FusedCfg {
    static constexpr int WM = T::WM, WN = T::WN, FM = T::FM, FN = T::FN, CB = T::CB, DB = T::DB;
    static constexpr int NT = 64 * WM * WN;
    static constexpr int TM = WM * FM * 16;
    static constexpr int TN = WN * FN * 16;
    static constexpr int NQ = P + 1;
    static constexpr int NA = (FORM == GWAS_FORM_BF16X3) ? 2 : 1;        // SNP-side planes
    static constexpr int NB = (FORM == GWAS_FORM_BF16X3) ? 2 * NQ : NQ;  // trait-side planes
    static constexpr int ESZ = (FORM == GWAS_FORM_F64) ? 8 : (FORM == GWAS_FORM_F32 ? 4 : 2);
    static constexpr int SPR = CB / 16;          // 16-byte segments per row per chunk
    static constexpr int RS = CB + 16;           // LDS row stride
    static constexpr int SEG_A = NA * TM * SPR;
    static constexpr int SEG_B = NB * TN * SPR;
    static constexpr int LA = (SEG_A + NT - 1) / NT;
    static constexpr int LB = (SEG_B + NT - 1) / NT;
    static constexpr int STAGE = (NA * TM + NB * TN) * RS;
    static constexpr int LDS = STAGE * (DB ? 2 : 1);
    static_assert(LDS <= 160 * 1024, "LDS tile too large");
};

template <typename T>
__device__ __forceinline__ T load16(const uint8_t *p) { return *(const T *)p; }

// Split-BF16 square: the hi/lo split of x'^2 from the split of x' (8 values per
// lane): x' = hi + lo is exact in FP32, its square is rounded to FP32 and split.
__device__ __forceinline__ void square_split(const bf16x8 &h, const bf16x8 &l, bf16x8 &sh, bf16x8 &sl) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const float x = (float)h[e] + (float)l[e];
        const float s = x * x;
        const __bf16 s_hi = (__bf16)s;
        sh[e] = s_hi;
        sl[e] = (__bf16)(s - (float)s_hi);
    }
}

// FP64 epilogue: Gram assembly and the p x p solve, lane-local. get(q, x, y,
// r) returns contraction q of register slot r of the wave's MFMA block (x, y).
template <int FORM, int P, int FM, int FN, class Get>
__device__ __forceinline__ void fused_epilogue(const FusedArgs &a, Get get, int64_t m_base, int n_base, int wm,
                                               int wn, int l16, int g) {
    constexpr int Q = P - 1;
    constexpr int NTL = Q * (Q + 1) / 2;
    unsigned bad = 0;
#pragma unroll
    for (int x = 0; x < FM; ++x)
#pragma unroll
        for (int y = 0; y < FN; ++y) {
            const int j = n_base + wn * FN * 16 + y * 16 + l16;
            if (j >= a.tb) continue;
            const double *F = a.fac + (int64_t)j * a.fac_stride;
            // small p: the trait's factor is cached in registers; large p reads it
            // from memory (L1/L2-resident) to keep the epilogue free of spills
            constexpr bool CACHE = NTL <= 36;
            double Lc[CACHE ? NTL : 1], z[Q];
            if constexpr (CACHE) {
#pragma unroll
                for (int u = 0; u < NTL; ++u) Lc[u] = F[u];
            }
            auto Lf = [&](int u) -> double {
                if constexpr (CACHE) return Lc[u];
                else return F[u];
            };
#pragma unroll
            for (int u = 0; u < Q; ++u) z[u] = F[NTL + u];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = m_base + wm * FM * 16 + x * 16 + mfma16_row<FORM == GWAS_FORM_F64>(g, r);
                if (i >= a.mi) continue;
                double cq[P + 1];
#pragma unroll
                for (int q = 0; q <= P; ++q) cq[q] = get(q, x, y, r);
                double u[Q];
                double s = cq[0];
#pragma unroll
                for (int aa = 0; aa < Q; ++aa) {
                    double v = 0.0;
#pragma unroll
                    for (int bb = 0; bb <= aa; ++bb) v += Lf(aa * (aa + 1) / 2 + bb) * cq[1 + bb];
                    u[aa] = v;
                    s -= v * v;
                }
                double num = cq[P];
#pragma unroll
                for (int aa = 0; aa < Q; ++aa) num -= u[aa] * z[aa];
                const bool ok = (s > a.rank_rtol * cq[0]) && isfinite(s) && isfinite(num);
                const double beta = num / s;
                double out[P];
#pragma unroll
                for (int aa = 0; aa < Q; ++aa) u[aa] = z[aa] - u[aa] * beta;
#pragma unroll
                for (int bb = 0; bb < Q; ++bb) {
                    double v = 0.0;
#pragma unroll
                    for (int aa = bb; aa < Q; ++aa) v += Lf(aa * (aa + 1) / 2 + bb) * u[aa];
                    out[bb] = v;
                }
                out[Q] = beta;
                const int64_t o = (i * a.ldt + j) * P;
                if constexpr (FORM == GWAS_FORM_F64) {
                    double *bo = (double *)a.b + o;
#pragma unroll
                    for (int v = 0; v < P; ++v) bo[v] = ok ? out[v] : __builtin_nan("");
                } else {
                    float *bo = (float *)a.b + o;
#pragma unroll
                    for (int v = 0; v < P; ++v) bo[v] = ok ? (float)out[v] : __builtin_nanf("");
                }
                bad += ok ? 0u : 1u;
            }
        }
    if (bad) atomicAdd(a.non_spd, (unsigned long long)bad);
}
// One TM x TN tile of problems (tile index over the tiles of a, traits fastest),
// computed by a whole workgroup of C::NT threads with `lds` (C::LDS bytes) as
// its staging memory. Every thread of the workgroup must call it with the same
// arguments (it contains workgroup barriers).
template <int FORM, int P, bool FLUSH, class T>
__device__ __forceinline__ void fused_tile(const FusedArgs &a, int64_t tile, uint8_t *lds) {
    using C = FusedCfg<FORM, P, T>;
    constexpr int NQ = C::NQ, TM = C::TM, TN = C::TN, NT = C::NT;
    constexpr int FM = C::FM, FN = C::FN, WM = C::WM;
    constexpr int SPR = C::SPR, RS = C::RS, CB = C::CB;
    using acc_t = typename std::conditional<FORM == GWAS_FORM_F64, d4, f4>::type;

    const int ntn = (a.tb + TN - 1) / TN;
    const int tn = (int)(tile % ntn);
    const int64_t tm = tile / ntn;
    const int64_t m_base = tm * TM;
    const int n_base = tn * TN;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;
    const int l16 = lane & 15, g = lane >> 4;

    const int64_t row_bytes = (int64_t)a.n_pad * C::ESZ;
    const int nchunks = (int)(row_bytes / CB);
    const uint8_t *A = (const uint8_t *)a.a;
    const uint8_t *B = (const uint8_t *)a.panels;
    const int64_t a_plane = a.a_plane_rows * row_bytes;
    const int64_t b_plane = (int64_t)a.tcap * row_bytes;

    uint4 ra[C::LA], rb[C::LB];
    auto gload = [&](int c) {
#pragma unroll
        for (int u = 0; u < C::LA; ++u) {
            const int seg = tid + u * NT;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (seg < C::SEG_A) {
                const int pl = seg / (TM * SPR), rem = seg % (TM * SPR);
                const int row = rem / SPR, sg = rem % SPR;
                const int64_t i = m_base + row;
                if (i < a.mi)
                    v = load16<uint4>(A + pl * a_plane + (a.i0 + i) * row_bytes + (int64_t)c * CB + sg * 16);
            }
            ra[u] = v;
        }
#pragma unroll
        for (int u = 0; u < C::LB; ++u) {
            const int seg = tid + u * NT;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (seg < C::SEG_B) {
                const int pl = seg / (TN * SPR), rem = seg % (TN * SPR);
                const int row = rem / SPR, sg = rem % SPR;
                const int j = n_base + row;
                if (j < a.tb)
                    v = load16<uint4>(B + pl * b_plane + (int64_t)j * row_bytes + (int64_t)c * CB + sg * 16);
            }
            rb[u] = v;
        }
    };
    auto sstore = [&](uint8_t *stage) {
        uint8_t *lA = stage;
        uint8_t *lB = stage + C::NA * TM * RS;
#pragma unroll
        for (int u = 0; u < C::LA; ++u) {
            const int seg = tid + u * NT;
            if (seg < C::SEG_A) {
                const int pl = seg / (TM * SPR), rem = seg % (TM * SPR);
                const int row = rem / SPR, sg = rem % SPR;
                *(uint4 *)(lA + (pl * TM + row) * RS + sg * 16) = ra[u];
            }
        }
#pragma unroll
        for (int u = 0; u < C::LB; ++u) {
            const int seg = tid + u * NT;
            if (seg < C::SEG_B) {
                const int pl = seg / (TN * SPR), rem = seg % (TN * SPR);
                const int row = rem / SPR, sg = rem % SPR;
                *(uint4 *)(lB + (pl * TN + row) * RS + sg * 16) = rb[u];
            }
        }
    };

    acc_t acc[NQ][FM][FN];
    d4 acc64[FLUSH ? NQ : 1][FLUSH ? FM : 1][FLUSH ? FN : 1];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int x = 0; x < FM; ++x)
#pragma unroll
            for (int y = 0; y < FN; ++y) {
                acc[q][x][y] = acc_t{0, 0, 0, 0};
                if constexpr (FLUSH) acc64[q][x][y] = d4{0, 0, 0, 0};
            }
    // FLUSH: the FP32 accumulators hold one 32-sample window (one 128-byte
    // chunk); after the window's last MFMA they are added to the FP64 sums, and
    // the next window's first MFMA starts from zero (no register clearing).
    auto fold = [&]() {
        if constexpr (FLUSH) {
#pragma unroll
            for (int q = 0; q < NQ; ++q)
#pragma unroll
                for (int x = 0; x < FM; ++x)
#pragma unroll
                    for (int y = 0; y < FN; ++y)
#pragma unroll
                        for (int r = 0; r < 4; ++r) acc64[q][x][y][r] += (double)acc[q][x][y][r];
        }
    };
    static_assert(!FLUSH || (FORM == GWAS_FORM_F32 && CB == 128), "the FP64 fold is per 128-byte FP32 chunk");

    const int arow0 = wm * FM * 16 + l16;
    const int brow0 = wn * FN * 16 + l16;

    // MFMAs of one 64-byte group of a staged chunk: lane group g reads the
    // 16-byte segment sg of its rows (the same segment of A and B rows).
    auto compute = [&](const uint8_t *stage, int sg, auto first_group) {
        constexpr bool FRESH = FLUSH && decltype(first_group)::value;   // window starts at zero
        const uint8_t *lA = stage;
        const uint8_t *lB = stage + C::NA * TM * RS;
        const int off = sg * 16;
        if constexpr (FORM == GWAS_FORM_F64) {
            double2 av[FM];
#pragma unroll
            for (int x = 0; x < FM; ++x) av[x] = load16<double2>(lA + (arow0 + x * 16) * RS + off);
#pragma unroll
            for (int y = 0; y < FN; ++y) {
                double2 bv[NQ];
#pragma unroll
                for (int q = 0; q < NQ; ++q) bv[q] = load16<double2>(lB + (q * TN + brow0 + y * 16) * RS + off);
#pragma unroll
                for (int x = 0; x < FM; ++x) {
                    const double x0 = av[x].x, x1 = av[x].y;
                    acc[0][x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0 * x0, bv[0].x, acc[0][x][y], 0, 0, 0);
                    acc[0][x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1 * x1, bv[0].y, acc[0][x][y], 0, 0, 0);
#pragma unroll
                    for (int q = 1; q < NQ; ++q) {
                        acc[q][x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, bv[q].x, acc[q][x][y], 0, 0, 0);
                        acc[q][x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, bv[q].y, acc[q][x][y], 0, 0, 0);
                    }
                }
            }
        } else if constexpr (FORM == GWAS_FORM_F32) {
            float4 av[FM];
#pragma unroll
            for (int x = 0; x < FM; ++x) av[x] = load16<float4>(lA + (arow0 + x * 16) * RS + off);
#pragma unroll
            for (int y = 0; y < FN; ++y) {
                float4 bv[NQ];
#pragma unroll
                for (int q = 0; q < NQ; ++q) bv[q] = load16<float4>(lB + (q * TN + brow0 + y * 16) * RS + off);
#pragma unroll
                for (int x = 0; x < FM; ++x) {
                    const float xs[4] = {av[x].x, av[x].y, av[x].z, av[x].w};
                    const float b0[4] = {bv[0].x, bv[0].y, bv[0].z, bv[0].w};
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        acc[0][x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                            xs[e] * xs[e], b0[e], (FRESH && e == 0) ? acc_t{0, 0, 0, 0} : acc[0][x][y], 0, 0, 0);
#pragma unroll
                    for (int q = 1; q < NQ; ++q) {
                        const float bq[4] = {bv[q].x, bv[q].y, bv[q].z, bv[q].w};
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            acc[q][x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                                xs[e], bq[e], (FRESH && e == 0) ? acc_t{0, 0, 0, 0} : acc[q][x][y], 0, 0, 0);
                    }
                }
            }
        } else {
            bf16x8 av[4][FM];   // x' hi, lo (staged), x'^2 hi, lo (formed here)
#pragma unroll
            for (int pl = 0; pl < 2; ++pl)
#pragma unroll
                for (int x = 0; x < FM; ++x) av[pl][x] = load16<bf16x8>(lA + (pl * TM + arow0 + x * 16) * RS + off);
#pragma unroll
            for (int x = 0; x < FM; ++x) square_split(av[0][x], av[1][x], av[2][x], av[3][x]);
#pragma unroll
            for (int y = 0; y < FN; ++y) {
                bf16x8 bh[NQ], bl[NQ];
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    bh[q] = load16<bf16x8>(lB + ((2 * q) * TN + brow0 + y * 16) * RS + off);
                    bl[q] = load16<bf16x8>(lB + ((2 * q + 1) * TN + brow0 + y * 16) * RS + off);
                }
#pragma unroll
                for (int x = 0; x < FM; ++x) {
                    // q = 0 uses the split square (planes 2, 3); q >= 1 the split value (planes 0, 1)
                    acc[0][x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[3][x], bh[0], acc[0][x][y], 0, 0, 0);
                    acc[0][x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[2][x], bl[0], acc[0][x][y], 0, 0, 0);
                    acc[0][x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[2][x], bh[0], acc[0][x][y], 0, 0, 0);
#pragma unroll
                    for (int q = 1; q < NQ; ++q) {
                        acc[q][x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[1][x], bh[q], acc[q][x][y], 0, 0, 0);
                        acc[q][x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[0][x], bl[q], acc[q][x][y], 0, 0, 0);
                        acc[q][x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[0][x], bh[q], acc[q][x][y], 0, 0, 0);
                    }
                }
            }
        }
    };

    // one staged chunk: CB / 64 groups of 64 bytes per row, then the fold
    auto compute_chunk = [&](const uint8_t *stage) {
        compute(stage, g, std::true_type{});
        if constexpr (CB >= 128) compute(stage, 4 + g, std::false_type{});
        if constexpr (CB >= 256) {
            compute(stage, 8 + g, std::false_type{});
            compute(stage, 12 + g, std::false_type{});
        }
        fold();
    };

    if constexpr (C::DB) {
        gload(0);
        sstore(lds);
        __syncthreads();
        for (int c = 0; c < nchunks; ++c) {
            uint8_t *cur = lds + (c & 1) * C::STAGE;
            if (c + 1 < nchunks) gload(c + 1);
            compute_chunk(cur);
            if (c + 1 < nchunks) sstore(lds + ((c + 1) & 1) * C::STAGE);
            __syncthreads();
        }
    } else {
        gload(0);
        for (int c = 0; c < nchunks; ++c) {
            __syncthreads();
            sstore(lds);
            __syncthreads();
            if (c + 1 < nchunks) gload(c + 1);
            compute_chunk(lds);
        }
    }
    if constexpr (FLUSH)
        fused_epilogue<FORM, P, FM, FN>(a, [&](int q, int x, int y, int r) { return acc64[q][x][y][r]; }, m_base,
                                        n_base, wm, wn, l16, g);
    else
        fused_epilogue<FORM, P, FM, FN>(a, [&](int q, int x, int y, int r) { return (double)acc[q][x][y][r]; },
                                        m_base, n_base, wm, wn, l16, g);
}

}  // namespace gw

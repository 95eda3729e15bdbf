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
//   F32:    float operands,  v_mfma_f32_16x16x4f32, FP32 accumulation added to
//           FP64 sums (b_B in chains of 8 samples, the others every 64)
//   BF16X3: bf16 hi/lo operands, v_mfma_f32_16x16x32_bf16, three products
//           hi*hi + hi*lo + lo*hi per pair, FP32 accumulation
//   BF16X6: bf16 hi/mid/lo operands, six products (all but mid*lo, lo*mid,
//           lo*lo), FP32 accumulation added to FP64 sums every 32 samples
//
// The tile kernels (operand staging, MFMA loops) are in fused_dma.h; this
// header holds what every form shares: the split-BF16 square and the FP64
// epilogue.
#pragma once

#include <type_traits>

#include "gwas_internal.h"

namespace gw {

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

// The p x p solve of one problem (i, j) from its p+1 contractions cq (FP64):
//   u = L_j^{-1} S_BL;  s = S_BR - u.u;  beta = (b_B - u.z_j) / s;
//   b_top = L_j^{-T} (z_j - u beta)
// with Lf(k) the packed lower triangle of L_j^{-1} and z = z_j. Stores b_ij
// (NaN when the pivot s falls below rank_rtol * S_BR or is not finite) at row
// i - row_lo of b and returns whether it was finite.
template <int FORM, int P, class LF>
__device__ __forceinline__ bool gls_solve_store(const FusedArgs &a, const double *cq, LF Lf, const double *z,
                                                int64_t i, int j) {
    constexpr int Q = P - 1;
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
    const int64_t o = ((i - a.row_lo) * a.ldt + j) * P;
    if constexpr (FORM == GWAS_FORM_F64) {
        double *bo = (double *)a.b + o;
#pragma unroll
        for (int v = 0; v < P; ++v) bo[v] = ok ? out[v] : __builtin_nan("");
    } else {
        float *bo = (float *)a.b + o;
#pragma unroll
        for (int v = 0; v < P; ++v) bo[v] = ok ? (float)out[v] : __builtin_nanf("");
    }
    return ok;
}

// Three-piece square: the hi/mid/lo split of x'^2 from x' = hi + mid + lo
// (exact in FP32), its square rounded to FP32 and split in three.
__device__ __forceinline__ void square_split3(const bf16x8 &h, const bf16x8 &m, const bf16x8 &l, bf16x8 &sh,
                                              bf16x8 &sm, bf16x8 &sl) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const float x = (float)h[e] + (float)m[e] + (float)l[e];
        const float s = x * x;
        const __bf16 s_hi = (__bf16)s;
        const float r = s - (float)s_hi;
        const __bf16 s_md = (__bf16)r;
        sh[e] = s_hi;
        sm[e] = s_md;
        sl[e] = (__bf16)(r - (float)s_md);
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
                if (i >= a.mi || i < a.row_lo) continue;
                double cq[P + 1];
#pragma unroll
                for (int q = 0; q <= P; ++q) cq[q] = get(q, x, y, r);
                bad += gls_solve_store<FORM, P>(a, cq, Lf, z, i, j) ? 0u : 1u;
            }
        }
    if (bad) atomicAdd(a.non_spd, (unsigned long long)bad);
}
}  // namespace gw

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
// K chunking: each chunk stages 64 bytes of every operand row (8 doubles,
// 16 floats or 32 bf16). Lane (l16, g) of a wave reads the 16-byte segment g
// of row l16 of a 16-row fragment; the same segment->k mapping is used for
// both operands, so every product pairs equal k.
#pragma once

#include <type_traits>

#include "gwas_internal.h"

namespace gw {

template <int FORM, int P, bool FLUSH>
struct FusedCfg {
    // waves along M and N, 16x16 MFMA blocks per wave along M and N
    static constexpr int WM = (FORM == GWAS_FORM_BF16X3) ? (P <= 4 ? 2 : (P <= 9 ? 4 : 2)) : 2;
    static constexpr int WN = (FORM == GWAS_FORM_BF16X3) ? (P <= 4 ? 2 : 1) : 2;
    static constexpr int FM = (FORM == GWAS_FORM_BF16X3) ? (P <= 4 ? 2 : 1) : (P <= 9 ? 2 : 1);
    static constexpr int FN = (FORM == GWAS_FORM_BF16X3) ? 1
                            : (FORM == GWAS_FORM_F64)    ? (P <= 4 ? 2 : 1)
                            : (FLUSH ? (P <= 4 ? 2 : 1) : (P <= 9 ? 2 : 1));
    static constexpr int NT = 64 * WM * WN;
    static constexpr int TM = WM * FM * 16;
    static constexpr int TN = WN * FN * 16;
    static constexpr int NQ = P + 1;
    static constexpr int NA = (FORM == GWAS_FORM_BF16X3) ? 4 : 1;        // SNP-side planes
    static constexpr int NB = (FORM == GWAS_FORM_BF16X3) ? 2 * NQ : NQ;  // trait-side planes
    static constexpr int ESZ = (FORM == GWAS_FORM_F64) ? 8 : (FORM == GWAS_FORM_F32 ? 4 : 2);
    static constexpr int SEG_A = NA * TM * (kChunkBytes / 16);
    static constexpr int SEG_B = NB * TN * (kChunkBytes / 16);
    static constexpr int LA = (SEG_A + NT - 1) / NT;
    static constexpr int LB = (SEG_B + NT - 1) / NT;
    static constexpr int LDS = (NA * TM + NB * TN) * kRowStride;
    static_assert(LDS <= 65536, "LDS tile too large");
};

template <typename T>
__device__ __forceinline__ T load16(const uint8_t *p) { return *(const T *)p; }

template <int FORM, int P, bool FLUSH>
__global__ __launch_bounds__((FusedCfg<FORM, P, FLUSH>::NT)) void fused_kernel(FusedArgs a) {
    using C = FusedCfg<FORM, P, FLUSH>;
    constexpr int NQ = C::NQ, TM = C::TM, TN = C::TN, NT = C::NT;
    constexpr int FM = C::FM, FN = C::FN, WM = C::WM;
    constexpr int SPR = kChunkBytes / 16;   // 16-byte segments per row per chunk
    using acc_t = typename std::conditional<FORM == GWAS_FORM_F64, d4, f4>::type;

    __shared__ __attribute__((aligned(16))) uint8_t lds[C::LDS];
    uint8_t *lA = lds;
    uint8_t *lB = lds + C::NA * TM * kRowStride;

    const int ntn = (a.tb + TN - 1) / TN;
    const int64_t tile = blockIdx.x;
    const int tn = (int)(tile % ntn);
    const int64_t tm = tile / ntn;
    const int64_t m_base = tm * TM;
    const int n_base = tn * TN;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;
    const int l16 = lane & 15, g = lane >> 4;

    const int64_t row_bytes = (int64_t)a.n_pad * C::ESZ;
    const int nchunks = (int)(row_bytes / kChunkBytes);
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
                    v = load16<uint4>(A + pl * a_plane + (a.i0 + i) * row_bytes +
                                      (int64_t)c * kChunkBytes + sg * 16);
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
                    v = load16<uint4>(B + pl * b_plane + (int64_t)j * row_bytes +
                                      (int64_t)c * kChunkBytes + sg * 16);
            }
            rb[u] = v;
        }
    };
    auto sstore = [&]() {
#pragma unroll
        for (int u = 0; u < C::LA; ++u) {
            const int seg = tid + u * NT;
            if (seg < C::SEG_A) {
                const int pl = seg / (TM * SPR), rem = seg % (TM * SPR);
                const int row = rem / SPR, sg = rem % SPR;
                *(uint4 *)(lA + (pl * TM + row) * kRowStride + sg * 16) = ra[u];
            }
        }
#pragma unroll
        for (int u = 0; u < C::LB; ++u) {
            const int seg = tid + u * NT;
            if (seg < C::SEG_B) {
                const int pl = seg / (TN * SPR), rem = seg % (TN * SPR);
                const int row = rem / SPR, sg = rem % SPR;
                *(uint4 *)(lB + (pl * TN + row) * kRowStride + sg * 16) = rb[u];
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

    const int arow0 = wm * FM * 16 + l16;
    const int brow0 = wn * FN * 16 + l16;

    gload(0);
    for (int c = 0; c < nchunks; ++c) {
        __syncthreads();
        sstore();
        __syncthreads();
        if (c + 1 < nchunks) gload(c + 1);

        if constexpr (FORM == GWAS_FORM_F64) {
            double2 av[FM];
#pragma unroll
            for (int x = 0; x < FM; ++x) av[x] = load16<double2>(lA + (arow0 + x * 16) * kRowStride + g * 16);
#pragma unroll
            for (int y = 0; y < FN; ++y) {
                double2 bv[NQ];
#pragma unroll
                for (int q = 0; q < NQ; ++q)
                    bv[q] = load16<double2>(lB + (q * TN + brow0 + y * 16) * kRowStride + g * 16);
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
            for (int x = 0; x < FM; ++x) av[x] = load16<float4>(lA + (arow0 + x * 16) * kRowStride + g * 16);
#pragma unroll
            for (int y = 0; y < FN; ++y) {
                float4 bv[NQ];
#pragma unroll
                for (int q = 0; q < NQ; ++q)
                    bv[q] = load16<float4>(lB + (q * TN + brow0 + y * 16) * kRowStride + g * 16);
#pragma unroll
                for (int x = 0; x < FM; ++x) {
                    const float xs[4] = {av[x].x, av[x].y, av[x].z, av[x].w};
                    const float b0[4] = {bv[0].x, bv[0].y, bv[0].z, bv[0].w};
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        acc[0][x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(xs[e] * xs[e], b0[e], acc[0][x][y], 0, 0, 0);
#pragma unroll
                    for (int q = 1; q < NQ; ++q) {
                        const float bq[4] = {bv[q].x, bv[q].y, bv[q].z, bv[q].w};
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            acc[q][x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(xs[e], bq[e], acc[q][x][y], 0, 0, 0);
                    }
                }
            }
            if constexpr (FLUSH) {
                if (((c + 1) % a.f32_flush) == 0 || c + 1 == nchunks) {
#pragma unroll
                    for (int q = 0; q < NQ; ++q)
#pragma unroll
                        for (int x = 0; x < FM; ++x)
#pragma unroll
                            for (int y = 0; y < FN; ++y) {
#pragma unroll
                                for (int r = 0; r < 4; ++r) acc64[q][x][y][r] += (double)acc[q][x][y][r];
                                acc[q][x][y] = acc_t{0, 0, 0, 0};
                            }
                }
            }
        } else {
            bf16x8 av[4][FM];
#pragma unroll
            for (int pl = 0; pl < 4; ++pl)
#pragma unroll
                for (int x = 0; x < FM; ++x)
                    av[pl][x] = load16<bf16x8>(lA + (pl * TM + arow0 + x * 16) * kRowStride + g * 16);
#pragma unroll
            for (int y = 0; y < FN; ++y) {
                bf16x8 bh[NQ], bl[NQ];
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    bh[q] = load16<bf16x8>(lB + ((2 * q) * TN + brow0 + y * 16) * kRowStride + g * 16);
                    bl[q] = load16<bf16x8>(lB + ((2 * q + 1) * TN + brow0 + y * 16) * kRowStride + g * 16);
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
    }

    // FP64 epilogue: Gram assembly and the p x p solve, lane-local.
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
            double Lf[NTL], z[Q];
#pragma unroll
            for (int u = 0; u < NTL; ++u) Lf[u] = F[u];
#pragma unroll
            for (int u = 0; u < Q; ++u) z[u] = F[NTL + u];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = m_base + wm * FM * 16 + x * 16 + mfma16_row<FORM == GWAS_FORM_F64>(g, r);
                if (i >= a.mi) continue;
                double cq[NQ];
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    if constexpr (FLUSH) cq[q] = acc64[q][x][y][r];
                    else cq[q] = (double)acc[q][x][y][r];
                }
                double u[Q];
                double s = cq[0];
#pragma unroll
                for (int aa = 0; aa < Q; ++aa) {
                    double v = 0.0;
#pragma unroll
                    for (int bb = 0; bb <= aa; ++bb) v += Lf[aa * (aa + 1) / 2 + bb] * cq[1 + bb];
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
                    for (int aa = bb; aa < Q; ++aa) v += Lf[aa * (aa + 1) / 2 + bb] * u[aa];
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

template <int FORM, int P, bool FLUSH>
hipError_t launch_fused_t(const FusedArgs &a, hipStream_t s) {
    using C = FusedCfg<FORM, P, FLUSH>;
    const int64_t tiles = ((a.mi + C::TM - 1) / C::TM) * ((a.tb + C::TN - 1) / C::TN);
    if (tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL((fused_kernel<FORM, P, FLUSH>), dim3((unsigned)tiles), dim3(C::NT), 0, s, a);
    return hipGetLastError();
}

template <int FORM, bool FLUSH>
hipError_t dispatch_p(const FusedArgs &a, hipStream_t s) {
    switch (a.p) {
#define GW_CASE(PP) case PP: return launch_fused_t<FORM, PP, FLUSH>(a, s);
        GW_CASE(2) GW_CASE(3) GW_CASE(4) GW_CASE(5) GW_CASE(6) GW_CASE(7) GW_CASE(8) GW_CASE(9)
        GW_CASE(10) GW_CASE(11) GW_CASE(12) GW_CASE(13) GW_CASE(14) GW_CASE(15) GW_CASE(16)
        GW_CASE(17) GW_CASE(18) GW_CASE(19) GW_CASE(20)
#undef GW_CASE
    default: return hipErrorInvalidValue;
    }
}

}  // namespace gw

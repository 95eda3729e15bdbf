// The fused contraction + solve for calls with few traits (t <= kSmallT),
// FP64 and FP32 forms.
//
// With few traits, the p+1 contractions of Algorithm 5's inner loop are dot
// products that read each rotated SNP row once for all t traits: about
// 2 (p+1) t flops per SNP-row element loaded, so the work is bound by HBM
// bandwidth, not by the MFMAs (a 16-trait MFMA tile would compute 16 / t times
// the useful work). Each wave takes R SNP rows at a time with L = 64 / R lanes
// per row (FP64: L = 16; FP32: L = 4); lane (k, rr) = (l mod L, l / L)
// multiplies row rr's samples 8L w + 4L h + 4k + {0..3} (h = 0, 1) of each
// 8L-sample window w with the trait panels, which the workgroup copies into LDS
// once, so one load instruction reads 16L contiguous elements of each of R rows
// (FP64: 512 bytes, whole cache lines; FP32: 64 bytes, with the panel reads of
// a lane position shared by the R rows). The L lanes' partial sums of a row are
// added with log2 L cross-lane exchanges; lane k then solves trait k.
//
// Occupancy: the panels take (p+1) t n_pad elements of LDS per workgroup (up to
// the 160 KB of a CU). A bandwidth-bound kernel needs many loads in flight, so
// the workgroup is sized for 16 waves per CU: 256 threads while four panel
// copies fit a CU, else 1024 threads (one workgroup per CU). Each panel value
// read from LDS serves one row per lane and costs an LDS read per product; with
// FP64 and t >= 2 the LDS reads, not HBM, would bound the kernel, so there each
// lane takes two rows at the same samples (and a workgroup 512 threads, as its
// registers double).
//
// Arithmetic: FP64 form in FP64. The FP32 form multiplies and adds in FP32
// within each window (8 products per lane) and adds the window sums in FP64.
#pragma once

#include <algorithm>
#include <type_traits>

#include "fused.h"

namespace gw {

template <int FORM>
struct GemvType { using type = float; };
template <>
struct GemvType<GWAS_FORM_F64> { using type = double; };

// 4 consecutive values of a row (element e0) of a form's store, as the compute type.
template <int FORM>
__device__ __forceinline__ void gemv_load4(const void *base, int64_t e0, typename GemvType<FORM>::type *v) {
    if constexpr (FORM == GWAS_FORM_F64) {
        const double2 a = *(const double2 *)((const double *)base + e0);
        const double2 b = *(const double2 *)((const double *)base + e0 + 2);
        v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    } else {
        static_assert(FORM == GWAS_FORM_F32, "FP64 and FP32 forms only");
        const float4 a = *(const float4 *)((const float *)base + e0);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    }
}

// 4 consecutive panel values from LDS (16-byte aligned).
template <int FORM>
__device__ __forceinline__ void gemv_lds4(const typename GemvType<FORM>::type *p, typename GemvType<FORM>::type *v) {
    if constexpr (FORM == GWAS_FORM_F64) {
        const double2 a = *(const double2 *)p, b = *(const double2 *)(p + 2);
        v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    } else {
        const float4 a = *(const float4 *)p;
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    }
}

// LDS bytes of a workgroup's panels (p+1 contractions x T traits x n_pad samples).
template <int FORM>
constexpr int64_t gemv_lds(int p, int t, int n_pad) {
    return (int64_t)(p + 1) * t * n_pad * (FORM == GWAS_FORM_F64 ? 8 : 4);
}

// Rows per lane: an FP64 lane with two or more traits takes two rows at the
// same sample positions, so every panel value it reads from LDS serves both
// (LDS reads, not HBM, bound the FP64 kernel as t grows).
template <int FORM, int T>
constexpr int gemv_rows_per_lane() { return FORM == GWAS_FORM_F64 && T >= 2 ? 2 : 1; }

// Threads per workgroup for a panel copy of `lds` bytes (see the header comment).
template <int FORM, int T>
constexpr int gemv_threads(int64_t lds) {
    return lds <= 40 * 1024 ? 256 : (gemv_rows_per_lane<FORM, T>() == 2 ? 512 : 1024);
}

template <int FORM, int P, int T, int NTH>
__global__ __launch_bounds__(NTH) void fused_gemv_kernel(FusedArgs a) {
    using ct = typename GemvType<FORM>::type;
    constexpr int NQ = P + 1;
    extern __shared__ __attribute__((aligned(16))) uint8_t gemv_lds_raw[];
    ct *pan = (ct *)gemv_lds_raw;   // [q][j][n_pad], in the compute type
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // L consecutive lanes per row, R row groups per wave: 16 x 4 for FP64 (whole
    // cache lines per row and load), 4 x 16 for FP32 (measured best at n = 1000);
    // each lane takes RPL rows, R apart
    constexpr int L = FORM == GWAS_FORM_F64 ? 16 : 4, R = 64 / L;
    constexpr int RPL = gemv_rows_per_lane<FORM, T>(), RW = R * RPL;   // rows per wave
    const int k = lane % L, rr = lane / L;   // lane k of row group rr
    const int n_pad = a.n_pad;
    constexpr int esz = FORM == GWAS_FORM_F64 ? 8 : 4;
    constexpr int NWV = NTH / 64;                     // waves per workgroup
    const int64_t b_plane = (int64_t)a.tcap * n_pad;  // panel plane stride (elements)

    // the workgroup's copy of the T traits' panels
    for (int e = threadIdx.x * 4; e < NQ * T * n_pad; e += NTH * 4) {
        const int q = e / (T * n_pad), j = (e / n_pad) % T, s = e % n_pad;
        ct v[4];
        gemv_load4<FORM>((const uint8_t *)a.panels + ((int64_t)q * b_plane + (int64_t)j * n_pad) * esz, s, v);
#pragma unroll
        for (int k = 0; k < 4; ++k) pan[e + k] = v[k];
    }
    __syncthreads();

    const int64_t nblk = (a.mi + NWV * RW - 1) / (NWV * RW);
    for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const int64_t r0 = (blk * NWV + wave) * RW + rr;   // rows r0 + R u
        const uint8_t *xrow[RPL];
#pragma unroll
        for (int u = 0; u < RPL; ++u) {
            const int64_t i = r0 + R * u;
            const int64_t ic = i < a.mi ? i : a.mi - 1;   // rows past the range load a valid row, store nothing
            xrow[u] = (const uint8_t *)a.a + (a.i0 + ic) * n_pad * esz;
        }

        double acc[RPL][T][NQ];
#pragma unroll
        for (int u = 0; u < RPL; ++u)
#pragma unroll
            for (int j = 0; j < T; ++j)
#pragma unroll
                for (int q = 0; q < NQ; ++q) acc[u][j][q] = 0.0;

        // lane k takes samples s0 .. s0 + 3 and s0 + 4L .. s0 + 4L + 3 of each
        // 8L-sample window (s0 = 8L w + 4k): the L lanes of a row read 16L
        // contiguous elements per load. n_pad is a multiple of 64, so only an
        // FP64 window (128 samples) can end the row half full, the same for
        // every lane: that last window runs as a separate half-window step, so
        // the loop body carries no run-time test.
        auto window = [&](int s0, auto two_c) {
            constexpr bool TWO = decltype(two_c)::value;
            constexpr int NE = TWO ? 8 : 4;
            ct x[RPL][8];
#pragma unroll
            for (int u = 0; u < RPL; ++u) {
                gemv_load4<FORM>(xrow[u], s0, x[u]);
                if constexpr (TWO) gemv_load4<FORM>(xrow[u], s0 + 4 * L, x[u] + 4);
            }
#pragma unroll
            for (int j = 0; j < T; ++j)
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    const ct *pp = pan + (q * T + j) * n_pad + s0;
                    ct pv[8];
                    gemv_lds4<FORM>(pp, pv);
                    if constexpr (TWO) gemv_lds4<FORM>(pp + 4 * L, pv + 4);
#pragma unroll
                    for (int u = 0; u < RPL; ++u) {
                        ct w = 0;
#pragma unroll
                        for (int e = 0; e < NE; ++e) {
                            const ct xs = q == 0 ? x[u][e] * x[u][e] : x[u][e];   // S_BR takes x'^2
                            w += xs * pv[e];
                        }
                        acc[u][j][q] += (double)w;
                    }
                }
        };
        const int nfull = n_pad / (8 * L);
#pragma unroll 2
        for (int w = 0; w < nfull; ++w) window(8 * L * w + 4 * k, std::true_type{});
        if (n_pad % (8 * L)) window(8 * L * nfull + 4 * k, std::false_type{});
        // sum the L lanes of each row
#pragma unroll
        for (int u = 0; u < RPL; ++u)
#pragma unroll
            for (int j = 0; j < T; ++j)
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    double v = acc[u][j][q];
#pragma unroll
                    for (int o = 1; o < L; o <<= 1) v += __shfl_xor(v, o);
                    acc[u][j][q] = v;
                }
        // lane k solves trait k of each of its rows
        const int j = k;
        if (j < T) {
            constexpr int Q = P - 1, NTL = Q * (Q + 1) / 2;
            const double *F = a.fac + (int64_t)j * a.fac_stride;
            double z[Q];
#pragma unroll
            for (int u = 0; u < Q; ++u) z[u] = F[NTL + u];
            auto Lf = [&](int u) -> double { return F[u]; };
#pragma unroll
            for (int u = 0; u < RPL; ++u) {
                const int64_t i = r0 + R * u;
                if (i >= a.mi) continue;
                double cq[NQ];
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    double v = acc[u][0][q];
#pragma unroll
                    for (int jj = 1; jj < T; ++jj)
                        if (j == jj) v = acc[u][jj][q];
                    cq[q] = v;
                }
                if (!gls_solve_store<FORM, P>(a, cq, Lf, z, i, j)) atomicAdd(a.non_spd, 1ull);
            }
        }
    }
}

template <int FORM, int P, int T, int NTH>
hipError_t launch_gemv_tn(const FusedArgs &a, int64_t lds, hipStream_t s) {
    static bool attr_set = false;   // per instantiation
    if (lds > 65536 && !attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)fused_gemv_kernel<FORM, P, T, NTH>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)kGemvLdsMax);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    // rows per wave, as in the kernel
    constexpr int RW = 64 / (FORM == GWAS_FORM_F64 ? 16 : 4) * gemv_rows_per_lane<FORM, T>();
    const int64_t nblk = (a.mi + (NTH / 64) * RW - 1) / ((NTH / 64) * RW);
    // 256-thread groups: up to 8 per CU; larger groups: up to 2 (512) or 1 (1024) per CU
    const int64_t cap = NTH == 256 ? 2048 : NTH == 512 ? 512 : 256;
    hipLaunchKernelGGL((fused_gemv_kernel<FORM, P, T, NTH>), dim3((unsigned)std::min<int64_t>(nblk, cap)),
                       dim3(NTH), (size_t)lds, s, a);
    return hipGetLastError();
}

template <int FORM, int P, int T>
hipError_t launch_gemv_t(const FusedArgs &a, int64_t lds, hipStream_t s) {
    constexpr int BIG = gemv_rows_per_lane<FORM, T>() == 2 ? 512 : 1024;
    return gemv_threads<FORM, T>(lds) == 256 ? launch_gemv_tn<FORM, P, T, 256>(a, lds, s)
                                             : launch_gemv_tn<FORM, P, T, BIG>(a, lds, s);
}

template <int FORM, int P>
hipError_t launch_gemv_t(const FusedArgs &a, hipStream_t s) {
    if (a.mi <= 0 || a.tb <= 0) return hipSuccess;
    const int64_t lds = gemv_lds<FORM>(P, a.tb, a.n_pad);
    if (a.tb > kSmallT || a.n_pad % 64 || lds > kGemvLdsMax) return hipErrorInvalidValue;
    static_assert(kSmallT == 3, "one instantiation per trait count");
    switch (a.tb) {
    case 1: return launch_gemv_t<FORM, P, 1>(a, lds, s);
    case 2: return launch_gemv_t<FORM, P, 2>(a, lds, s);
    default: return launch_gemv_t<FORM, P, 3>(a, lds, s);
    }
}

template <int FORM>
hipError_t dispatch_gemv(const FusedArgs &a, hipStream_t s) {
    switch (a.p) {
#define GW_CASE(PP) case PP: return launch_gemv_t<FORM, PP>(a, s);
        GW_CASE(2) GW_CASE(3) GW_CASE(4) GW_CASE(5) GW_CASE(6) GW_CASE(7) GW_CASE(8) GW_CASE(9)
        GW_CASE(10) GW_CASE(11) GW_CASE(12) GW_CASE(13) GW_CASE(14) GW_CASE(15) GW_CASE(16)
        GW_CASE(17) GW_CASE(18) GW_CASE(19) GW_CASE(20)
#undef GW_CASE
    default: return hipErrorInvalidValue;
    }
}

}  // namespace gw

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
// Arithmetic: FP64 form in FP64. FP32 and split-BF16 forms multiply and add in
// FP32 within each window (8 products per lane) and add the window sums in
// FP64; the split-BF16 operands are used as hi + lo (exact in FP32), which
// keeps the lo*lo product the three-product MFMA form drops.
#pragma once

#include <algorithm>

#include "fused.h"

namespace gw {

template <int FORM>
struct GemvType { using type = float; };
template <>
struct GemvType<GWAS_FORM_F64> { using type = double; };

// 4 consecutive values of a row (element e0) of a form's store, as the compute type.
template <int FORM>
__device__ __forceinline__ void gemv_load4(const void *base, int64_t plane, int64_t e0,
                                           typename GemvType<FORM>::type *v) {
    if constexpr (FORM == GWAS_FORM_F64) {
        const double2 a = *(const double2 *)((const double *)base + e0);
        const double2 b = *(const double2 *)((const double *)base + e0 + 2);
        v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    } else if constexpr (FORM == GWAS_FORM_F32) {
        const float4 a = *(const float4 *)((const float *)base + e0);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    } else {
        const uint16_t *p = (const uint16_t *)base + e0;
        const uint2 h = *(const uint2 *)p, l = *(const uint2 *)(p + plane);
        const uint32_t hw[2] = {h.x, h.y}, lw[2] = {l.x, l.y};
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            v[2 * k] = __uint_as_float(hw[k] << 16) + __uint_as_float(lw[k] << 16);
            v[2 * k + 1] = __uint_as_float(hw[k] & 0xffff0000u) + __uint_as_float(lw[k] & 0xffff0000u);
        }
    }
}

// LDS bytes of a workgroup's panels (p+1 contractions x T traits x n_pad samples).
template <int FORM>
constexpr int64_t gemv_lds(int p, int t, int n_pad) {
    return (int64_t)(p + 1) * t * n_pad * (FORM == GWAS_FORM_F64 ? 8 : 4);
}

template <int FORM, int P, int T>
__global__ __launch_bounds__(256) void fused_gemv_kernel(FusedArgs a) {
    using ct = typename GemvType<FORM>::type;
    constexpr int NQ = P + 1;
    extern __shared__ __attribute__((aligned(16))) uint8_t gemv_lds_raw[];
    ct *pan = (ct *)gemv_lds_raw;   // [q][j][n_pad], in the compute type
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // L consecutive lanes per row, R rows per wave: 16 x 4 for FP64 (whole
    // cache lines per row and load), 4 x 16 for FP32 (measured best at n = 1000)
    constexpr int L = FORM == GWAS_FORM_F64 ? 16 : 4, R = 64 / L;
    const int k = lane % L, rr = lane / L;   // lane k of row rr
    const int n_pad = a.n_pad;
    const int esz = FORM == GWAS_FORM_F64 ? 8 : (FORM == GWAS_FORM_F32 ? 4 : 2);
    const int64_t x_plane = a.a_plane_rows * n_pad;   // BF16 lo plane offset (elements)
    const int64_t b_plane = (int64_t)a.tcap * n_pad;  // panel plane stride (elements)

    // the workgroup's copy of the T traits' panels (BF16: hi + lo, exact in FP32)
    for (int e = threadIdx.x * 4; e < NQ * T * n_pad; e += 256 * 4) {
        const int q = e / (T * n_pad), j = (e / n_pad) % T, s = e % n_pad;
        const int pl = FORM == GWAS_FORM_BF16X3 ? 2 * q : q;
        ct v[4];
        gemv_load4<FORM>((const uint8_t *)a.panels + ((int64_t)pl * b_plane + (int64_t)j * n_pad) * esz, b_plane,
                         s, v);
#pragma unroll
        for (int k = 0; k < 4; ++k) pan[e + k] = v[k];
    }
    __syncthreads();

    const int64_t nblk = (a.mi + 4 * R - 1) / (4 * R);
    for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const int64_t i = (blk * 4 + wave) * R + rr;
        const int64_t ic = i < a.mi ? i : a.mi - 1;   // rows past the range load a valid row, store nothing
        const uint8_t *xrow = (const uint8_t *)a.a + (a.i0 + ic) * n_pad * esz;

        double acc[T][NQ];
#pragma unroll
        for (int j = 0; j < T; ++j)
#pragma unroll
            for (int q = 0; q < NQ; ++q) acc[j][q] = 0.0;

        // lane k takes samples s0 .. s0 + 3 and s0 + 4L .. s0 + 4L + 3 of each
        // 8L-sample window (s0 = 8L w + 4k): the L lanes of a row read 16L
        // contiguous elements per load. n_pad is a multiple of 64, so the second
        // half of the last window is absent for the whole wave or for none.
#pragma unroll 2
        for (int s0 = 4 * k; s0 < n_pad; s0 += 8 * L) {
            // windows of 8L <= 64 samples always fit n_pad (a multiple of 64)
            const bool two = 64 % (8 * L) == 0 || s0 + 4 * L < n_pad;
            ct x[8];
            gemv_load4<FORM>(xrow, x_plane, s0, x);
            if (two) {
                gemv_load4<FORM>(xrow, x_plane, s0 + 4 * L, x + 4);
            } else {
#pragma unroll
                for (int e = 4; e < 8; ++e) x[e] = 0;
            }
            ct xx[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) xx[e] = x[e] * x[e];
#pragma unroll
            for (int j = 0; j < T; ++j)
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    const ct *pp = pan + (q * T + j) * n_pad + s0;
                    ct pv[8];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        pv[e] = pp[e];
                        pv[4 + e] = two ? pp[4 * L + e] : ct(0);
                    }
                    ct w = 0;
#pragma unroll
                    for (int e = 0; e < 8; ++e) w += (q == 0 ? xx[e] : x[e]) * pv[e];
                    acc[j][q] += (double)w;
                }
        }
        // sum the L lanes of each row
#pragma unroll
        for (int j = 0; j < T; ++j)
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                double v = acc[j][q];
#pragma unroll
                for (int o = 1; o < L; o <<= 1) v += __shfl_xor(v, o);
                acc[j][q] = v;
            }
        // lane k solves trait k of row i
        const int j = k;
        if (i < a.mi && j < T) {
            double cq[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                double v = acc[0][q];
#pragma unroll
                for (int jj = 1; jj < T; ++jj)
                    if (j == jj) v = acc[jj][q];
                cq[q] = v;
            }
            constexpr int Q = P - 1, NTL = Q * (Q + 1) / 2;
            const double *F = a.fac + (int64_t)j * a.fac_stride;
            double z[Q];
#pragma unroll
            for (int u = 0; u < Q; ++u) z[u] = F[NTL + u];
            auto Lf = [&](int u) -> double { return F[u]; };
            if (!gls_solve_store<FORM, P>(a, cq, Lf, z, i, j)) atomicAdd(a.non_spd, 1ull);
        }
    }
}

template <int FORM, int P>
hipError_t launch_gemv_t(const FusedArgs &a, hipStream_t s) {
    if (a.mi <= 0 || a.tb <= 0) return hipSuccess;
    const int64_t lds = gemv_lds<FORM>(P, a.tb, a.n_pad);
    if (a.tb > kSmallT || a.n_pad % 64 || lds > kGemvLdsMax) return hipErrorInvalidValue;
    constexpr int RPW = 64 / (FORM == GWAS_FORM_F64 ? 16 : 4);   // rows per wave, as in the kernel
    const int64_t nblk = (a.mi + 4 * RPW - 1) / (4 * RPW);
    const dim3 grid((unsigned)std::min<int64_t>(nblk, 2048)), block(256);
    static_assert(kSmallT == 3, "one instantiation per trait count");
    switch (a.tb) {
    case 1: hipLaunchKernelGGL((fused_gemv_kernel<FORM, P, 1>), grid, block, lds, s, a); break;
    case 2: hipLaunchKernelGGL((fused_gemv_kernel<FORM, P, 2>), grid, block, lds, s, a); break;
    default: hipLaunchKernelGGL((fused_gemv_kernel<FORM, P, 3>), grid, block, lds, s, a); break;
    }
    return hipGetLastError();
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

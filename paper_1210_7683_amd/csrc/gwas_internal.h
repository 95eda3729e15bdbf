// Internal declarations shared by the HIP sources of libgwas (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gwas.h"

namespace gw {

// Sample axis padding: rotated rows are stored with n_pad = round_up(n, 64)
// values (zeros beyond n), so every K loop runs over whole chunks of up to
// 128 bytes (FP16/BF16), 256 bytes (FP32) or 512 bytes (FP64) per row.
constexpr int kPadN = 64;

// Relative floor of the Schur pivot of the SNP column, per form: a problem
// whose S_BR - |L^{-1} S_BL|^2 does not exceed this fraction of S_BR is
// treated as rank-deficient (b = NaN). It scales with the contraction
// precision: the pivot's computed value is noise below it.
constexpr double kRankRtol[4] = {1e-10, 1e-4, 1e-3, 1e-4};

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Row of a 16x16 MFMA result held in register r of a lane in lane group g
// (= lane / 16); the column is lane % 16. The FP64 16x16x4 variant interleaves
// its four rows (g, g+4, g+8, g+12); the FP32 and BF16 variants hold four
// consecutive rows (4g .. 4g+3).
template <bool F64>
__device__ __forceinline__ int mfma16_row(int g, int r) { return F64 ? g + 4 * r : 4 * g + r; }

// Workgroup -> tile order over ntn column tiles (see fused_dma.h): XCD-aware when
// ntn is a multiple of 8, identity otherwise; a bijection of [0, tiles).
__host__ __device__ constexpr int64_t xcd_order(int64_t b, int ntn) {
    if (ntn % 8) return b;
    const int64_t x = b % 8, local = b / 8;
    const int g = ntn / 8;
    return (local / g) * ntn + x * g + local % g;
}

// Workgroup -> tile (tm * ntn + tn) over ntm x ntn tiles, a bijection for any
// ntn (checked at compile time in api.hip); workgroup b runs on XCD b mod 8.
// The first 8 floor(ntn / 8) column tiles of every row come first, in
// XCD-aware order (each XCD a contiguous eighth of them, over all rows). The
// remaining r = ntn mod 8 column tiles follow by groups of 8 rows, XCD x taking
// the r tiles of row 8 G + x, so that a row's tail tiles share one XCD's L2;
// rows past the last whole group of 8, and grids with fewer than 8 column
// tiles, run in plain order.
__host__ __device__ constexpr int64_t tile_order(int64_t b, int64_t ntm, int ntn) {
    const int g = ntn / 8;
    if (g == 0) return b;
    const int n8 = 8 * g;
    const int64_t na = ntm * n8;
    if (b < na) {
        const int64_t t = xcd_order(b, n8);
        return (t / n8) * ntn + t % n8;
    }
    const int r = ntn - n8;                      // > 0 here: b < ntm ntn
    b -= na;                                     // na is a multiple of 8: b keeps its XCD
    const int64_t nfull = (ntm / 8) * 8 * r;     // tail tiles of the whole groups of 8 rows
    if (b < nfull) {
        const int64_t k = b / 8, x = b % 8;
        return ((k / r) * 8 + x) * ntn + n8 + k % r;
    }
    b -= nfull;
    return ((ntm / 8) * 8 + b / r) * ntn + n8 + b % r;
}

// True if tile_order maps [0, NTM NTN) onto itself one to one.
template <int64_t NTM, int NTN>
constexpr bool tile_order_is_bijection() {
    bool seen[NTM * NTN] = {};
    for (int64_t b = 0; b < NTM * NTN; ++b) {
        const int64_t t = tile_order(b, NTM, NTN);
        if (t < 0 || t >= NTM * NTN || seen[t]) return false;
        seen[t] = true;
    }
    return true;
}

// Round-to-nearest-even of an FP32 value to BF16 (finite inputs), as raw bits.
__device__ __forceinline__ uint16_t bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// x = hi + lo with hi = bf16(x) and lo = bf16(x - hi); x - hi is exact in FP32.
__device__ __forceinline__ void bf16_split(float x, uint16_t &hi, uint16_t &lo) {
    hi = bf16_rne(x);
    lo = bf16_rne(x - bf16_to_f32(hi));
}

// x = hi + mid + lo exactly (24 bits in three BF16 pieces); each residual is
// exact in FP32.
__device__ __forceinline__ void bf16_split3(float x, uint16_t &hi, uint16_t &mid, uint16_t &lo) {
    hi = bf16_rne(x);
    const float r = x - bf16_to_f32(hi);
    mid = bf16_rne(r);
    lo = bf16_rne(r - bf16_to_f32(mid));
}

// Split-BF16 planes (rotated SNPs and trait panels) are stored in MFMA
// fragment order rather than row-major: the 1 KB block (row / 16, sample / 32),
// at block index (row / 16) (n_pad / 32) + sample / 32, holds 16 rows x 32
// samples in the operand lane order of the 16x16x32 BF16 MFMA: lane
// L = ((sample mod 32) / 8) 16 + row mod 16 owns bytes 16 L .. 16 L + 15,
// samples 8 (L / 16) .. + 7 of row L mod 16. A wave then stages a fragment with
// one contiguous 1 KB copy (whole cache lines), where a row-major plane needs 16
// half cache lines from 16 rows. A plane of R rows (R a multiple of 16) spans
// R n_pad elements, as row-major.
__host__ __device__ constexpr int64_t bf_frag_index(int64_t row, int k, int n_pad) {
    return (((row >> 4) * (n_pad >> 5) + (k >> 5)) << 9) + ((int64_t)(((k & 31) >> 3) * 16 + (row & 15)) << 3) +
           (k & 7);
}
static_assert(bf_frag_index(0, 0, 64) == 0 && bf_frag_index(1, 0, 64) == 8 && bf_frag_index(0, 8, 64) == 128 &&
                  bf_frag_index(0, 32, 64) == 512 && bf_frag_index(16, 0, 64) == 1024 &&
                  bf_frag_index(17, 41, 64) == 1024 + 512 + (16 + 1) * 8 + 1,
              "fragment order");

// Rows of a trait-panel plane holding t traits: a multiple of 16, so that the
// fragment-ordered BF16 planes of consecutive contractions do not overlap.
inline int panel_rows(int t) { return (t + 15) / 16 * 16; }

// Output planes of a rotation (any pointer may be null).
struct RotOut {
    double *f64;      // [rows][ld]
    float *f32;       // [rows][ld]
    uint16_t *bf;     // 2 planes, each [plane_rows][ld]: x hi, x lo
    uint16_t *bf3;    // 3 planes, each [plane_rows][ld]: x hi, mid, lo
    int64_t plane_rows;
    int64_t row0;     // first output row
    int ld;           // n_pad
};

// Z in fixed point, sliced into int8 digits, for the genotype rotation on the
// int8 MFMAs: row k of Z is scaled by 2^E_k and rounded to an integer q_k[r]
// with |q_k| <= 2^(8 kZSlices - 2); q_k = sum_d 256^(kZSlices-1-d) s_d with
// balanced digits s_d in [-128, 127]. For genotype bytes v (offset to
// a = v - 128, exact in int8) every digit's contraction sum_r a_r s_d[k][r] is
// exact in int32 (|.| <= 2^14 n_pad), and
//   x'[k] = 2^-E_k (sum_d 256^(kZSlices-1-d) acc_d + 128 sum_r q_k[r]).
// The only error is the rounding of Z to 8 kZSlices - 1 bits (relative to the
// row's largest entry): with 6 digits below 1e-14 of x' for unit-norm rows.
// Rotations that fill no FP64 store use only the leading kZSlicesShort digits
// (Z to about 2^-30 of its row maximum, far below FP32 rounding): the
// truncated integer q'_k = sum_{d < kZSlicesShort} 256^(kZSlicesShort-1-d) s_d
// stands for 2^-(E_k - 8 (kZSlices - kZSlicesShort)) q'_k.
constexpr int kZSlices = 6;
constexpr int kZSlicesShort = 4;
constexpr int kZSliceMaxNpad = 1 << 17;   // int32 headroom of the digit sums
// The digits are stored in MFMA fragment order: 1 KB block (d, kb, s) =
// ((d n_pad/16 + kb) n_pad/64 + s) holds at bytes 16 l .. 16 l + 15 digit d of
// row 16 kb + l % 16, samples 64 s + 16 (l / 16) .. + 15, so a wave copies one
// contiguous block per instruction.
struct ZSlices {
    const int8_t *q;       // kZSlices n_pad^2 bytes in fragment order
    const double *off;     // [2][n_pad]: 128 sum_r q_k[r], then 128 sum_r q'_k[r]
    const double *scale;   // [n_pad]: 2^-E_k (0 for an all-zero row)
    uint8_t *pack;         // device scratch: pack_rows genotype rows of n_pad bytes in fragment
    int64_t pack_rows;     // blocks (a multiple of 256); the rotation runs in chunks of this many rows
};
// Default bytes of the genotype repack chunk (rows of n_pad bytes).
constexpr int64_t kGenoPackBytes = 256ll << 20;
// Host: slices of the padded row-major Z (row k = eigenvector k, zeros past n).
void slice_z_int8(const double *zh, int n_pad, int8_t *q, double *off, double *scale);

// out[row0 + i][k] = sum_r X[i][r] Z[k][r]  for i < rows, k < n_pad. Genotype
// bytes (GWAS_DT_U8) use the int8 digit kernels and need zs with its pack
// buffer (n_pad <= kZSliceMaxNpad; hipErrorInvalidValue otherwise); calls that
// share a zs must be ordered (one stream, or events), as they share its pack
// buffer. FP64 and FP32 inputs FP64 MFMA.
hipError_t launch_rotate(const void *X, int dtype, int64_t rows, int n, int64_t ldx,
                         const double *Zrows, int n_pad, const RotOut &out, hipStream_t s,
                         const ZSlices *zs = nullptr);

// Per-trait prologue (FP64): weights, contraction panels, and the factor of S_TL.
struct PrepArgs {
    const double *yt;    // [tb][n_pad] rotated traits
    const double *h2;    // [tb]
    const double *w;     // [n_pad]
    const double *xlt;   // [p-1][n_pad] rotated covariates
    void *panels;        // form layout, plane stride tcap rows
    double *fac;         // [tb][fac_stride]: packed L^{-1} (lower), then z = L^{-1} b_T
    int tb, n, n_pad, p, tcap, fac_stride, form;
};
hipError_t launch_prep(const PrepArgs &a, hipStream_t s);

inline int fac_stride(int p) {
    int q = p - 1;
    int v = q * (q + 1) / 2 + q;
    return (v + 1) & ~1;
}

// Fused contraction + solve.
struct FusedArgs {
    const void *a;          // resident rotated SNP planes (form layout), rows of n_pad
    int64_t a_plane_rows;   // rows per plane (the bf16 form has 2 planes)
    int64_t i0, mi;         // SNP range
    const void *panels;     // trait panels, plane stride tcap rows
    int tcap;
    const double *fac;      // [tb][fac_stride]
    int fac_stride;
    int tb;                 // traits in this sub-block
    int n_pad, p;
    int n;                  // samples: both operands are zero from n to n_pad, so a
                            // K loop may stop at the stage that holds sample n - 1
    void *b;                // output: b[(i - i0) * ldt + j] * p ...
    int64_t ldt;            // trait stride of b (in problems)
    double rank_rtol;
    unsigned long long *non_spd;
    int f32_flush;
    int small_t;            // nonzero: the call has at most kSmallT traits (dot-product kernel)
    unsigned *tile_counters;  // 8 device words for persistent launches (zeroed by the launcher)
    // Rows [i0, i0 + row_lo) are computed but not stored: the split-BF16 forms
    // stage whole 16-row groups of their fragment-ordered store, so a range
    // starting inside a group starts at the group (b row i lands at i - row_lo).
    int64_t row_lo;
};
hipError_t launch_fused(int form, const FusedArgs &a, hipStream_t s);

// FP64 and FP32 solve calls with at most kSmallT traits in total, whose panels
// fit the dot-product kernel's LDS copy (a CU's 160 KB), use that kernel
// (HBM-bound, fused_gemv.h) instead of the MFMA tiles; measured on MI355X at
// n = 1000, p = 4, it is faster there (the split-BF16 MFMA tiles are not
// slower at any t, and both split-BF16 forms keep them). The choice is per
// call, so every problem of a call is computed the same way whatever the
// sub-blocking.
constexpr int kSmallT = 3;
constexpr int64_t kGemvLdsMax = 160 * 1024;
inline bool use_dot_kernel(int form, int p, int tb_call, int n_pad) {
    const int64_t lds = (int64_t)(p + 1) * tb_call * n_pad * (form == GWAS_FORM_F64 ? 8 : 4);
    return (form == GWAS_FORM_F64 || form == GWAS_FORM_F32) && tb_call <= kSmallT && lds <= kGemvLdsMax;
}

// Copy `bytes` (a multiple of 4; 16-byte aligned pointers) from device memory
// to pinned host memory, given the host buffer's device-side address.
hipError_t launch_copy_to_host(void *dst_dev_view, const void *src, int64_t bytes, int grid, hipStream_t s);
hipError_t launch_fused_f64(const FusedArgs &a, hipStream_t s);
hipError_t launch_fused_f32(const FusedArgs &a, hipStream_t s);
hipError_t launch_fused_bf16(const FusedArgs &a, hipStream_t s);
hipError_t launch_fused_bf16x6(const FusedArgs &a, hipStream_t s);

}  // namespace gw

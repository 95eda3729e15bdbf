// Rotation by Z^T (the preloop GEMMs of Algorithm 5): out = X Z, i.e. every
// input column x (n samples) becomes x' = Z^T x, computed as an FP64 MFMA GEMM
// (v_mfma_f64_16x16x4) with both operands contiguous along the samples.
//
// The rotated rows are written in every resident form at once: FP64, rounded
// to FP32, and split to BF16 hi/lo together with the split of the square x'^2
// (the square is taken in FP64 and rounded to FP32 before the split).
#include "gwas_internal.h"

namespace gw {
namespace {

constexpr int RT_M = 64;      // input columns (SNPs / traits) per workgroup
constexpr int RT_N = 64;      // rotated sample indices per workgroup
constexpr int RT_K = 16;      // samples per K chunk
constexpr int RT_LD = RT_K + 2;  // LDS row stride in doubles (16 bytes of padding)

template <typename T>
__device__ __forceinline__ double to_f64(T v) { return (double)v; }

template <typename Tin>
__global__ __launch_bounds__(256) void rotate_kernel(const Tin *__restrict__ X, int64_t rows, int n,
                                                     int64_t ldx, const double *__restrict__ Zr,
                                                     int n_pad, RotOut out) {
    __shared__ double la[RT_M * RT_LD];
    __shared__ double lb[RT_N * RT_LD];
    const int ntn = n_pad / RT_N;
    const int64_t tile = blockIdx.x;
    const int tn = (int)(tile % ntn);
    const int64_t tm = tile / ntn;
    const int64_t i_base = tm * RT_M;
    const int k_base = tn * RT_N;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int l16 = lane & 15, g = lane >> 4;

    // loader coordinates: 64 rows x 16 values, 4 consecutive values per thread
    const int lrow = tid >> 2, lcol = (tid & 3) * 4;
    const int64_t gi = i_base + lrow;
    const Tin *xrow = X + gi * ldx;
    const double *zrow = Zr + (int64_t)(k_base + lrow) * n_pad;

    d4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

    const int kend = (n + RT_K - 1) / RT_K * RT_K;   // <= n_pad
    for (int k0 = 0; k0 < kend; k0 += RT_K) {
        double va[4], vb[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int r = k0 + lcol + e;
            va[e] = (gi < rows && r < n) ? to_f64(xrow[r]) : 0.0;
            vb[e] = zrow[r];   // Z rows are n_pad long and zero beyond n
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            la[lrow * RT_LD + lcol + e] = va[e];
            lb[lrow * RT_LD + lcol + e] = vb[e];
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < RT_K / 4; ++s) {
            double fa[2], fb[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) fa[a] = la[(wm * 32 + a * 16 + l16) * RT_LD + s * 4 + g];
#pragma unroll
            for (int b = 0; b < 2; ++b) fb[b] = lb[(wn * 32 + b * 16 + l16) * RT_LD + s * 4 + g];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fb[b], acc[a][b], 0, 0, 0);
        }
    }

    // FP64 16x16 MFMA result: register r of lane group g is row g + 4r, column lane % 16.
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = i_base + wm * 32 + a * 16 + mfma16_row<true>(g, r);
                const int k = k_base + wn * 32 + b * 16 + l16;
                if (i >= rows) continue;
                const double v = acc[a][b][r];
                const int64_t o = (out.row0 + i) * out.ld + k;
                if (out.f64) out.f64[o] = v;
                if (out.f32) out.f32[o] = (float)v;
                if (out.bf) {
                    uint16_t h, l;
                    bf16_split((float)v, h, l);
                    const int64_t ps = out.plane_rows * out.ld;
                    out.bf[o] = h;
                    out.bf[ps + o] = l;
                    bf16_split((float)(v * v), h, l);
                    out.bf[2 * ps + o] = h;
                    out.bf[3 * ps + o] = l;
                }
            }
}

}  // namespace

hipError_t launch_rotate(const void *X, int dtype, int64_t rows, int n, int64_t ldx,
                         const double *Zrows, int n_pad, const RotOut &out, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    const int64_t tiles = ((rows + RT_M - 1) / RT_M) * (n_pad / RT_N);
    dim3 grid((unsigned)tiles), block(256);
    switch (dtype) {
    case GWAS_DT_F64:
        hipLaunchKernelGGL(rotate_kernel<double>, grid, block, 0, s, (const double *)X, rows, n, ldx,
                           Zrows, n_pad, out);
        break;
    case GWAS_DT_F32:
        hipLaunchKernelGGL(rotate_kernel<float>, grid, block, 0, s, (const float *)X, rows, n, ldx,
                           Zrows, n_pad, out);
        break;
    case GWAS_DT_U8:
        hipLaunchKernelGGL(rotate_kernel<uint8_t>, grid, block, 0, s, (const uint8_t *)X, rows, n,
                           ldx, Zrows, n_pad, out);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace gw

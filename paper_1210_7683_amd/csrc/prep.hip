// Per-trait prologue of the loops of Algorithm 5, in FP64. One workgroup per
// trait j of the block:
//   d_jk = 1 / (h2_j w_k + 1 - h2_j)           (D_j^{-1} with sigma2 dropped)
//   panels of the fused contraction, each n_pad long (zero beyond n):
//     plane 0      d_j                        -> S_BR = sum_k d_jk x'_ki^2
//     plane 1+c    d_j o x'_L[:, c]           -> S_BL[c] = sum_k x'_ki d_jk x'_L,kc
//     plane p      d_j o y'_j                 -> b_B = sum_k x'_ki d_jk y'_kj
//   S_TL_j = X'_L^T diag(d_j) X'_L, b_T_j = X'_L^T (d_j o y'_j)  (the syrk and
//   gemv of the trait loop), L_j = chol(S_TL_j), and the fused kernel's
//   per-trait data: L_j^{-1} (packed lower) and z_j = L_j^{-1} b_T_j.
// The paper scales by K_j = D_j^{-1/2} before forming the products; folding
// d_j = K_j^2 into the trait side gives the same sums without square roots.
#include <math.h>

#include "gwas_internal.h"

namespace gw {
namespace {

constexpr int PT = 256;

__device__ double block_sum(double v, double *red) {
    // wave reduction, then across the 4 waves (fixed order: deterministic)
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
}

template <int FORM>
__device__ __forceinline__ void put(void *panels, int plane, int tcap, int j, int n_pad, int k,
                                    double v) {
    const int64_t o = ((int64_t)plane * tcap + j) * n_pad + k;
    if constexpr (FORM == GWAS_FORM_F64) {
        ((double *)panels)[o] = v;
    } else if constexpr (FORM == GWAS_FORM_F32) {
        ((float *)panels)[o] = (float)v;
    } else {   // split BF16: fragment-ordered planes (tcap a multiple of 16)
        const int64_t ps = (int64_t)tcap * n_pad;
        const int64_t f = bf_frag_index(j, k, n_pad);
        if constexpr (FORM == GWAS_FORM_BF16X3) {
            uint16_t h, l;
            bf16_split((float)v, h, l);
            ((uint16_t *)panels)[2 * plane * ps + f] = h;
            ((uint16_t *)panels)[(2 * plane + 1) * ps + f] = l;
        } else {
            uint16_t h, md, l;
            bf16_split3((float)v, h, md, l);
            ((uint16_t *)panels)[3 * plane * ps + f] = h;
            ((uint16_t *)panels)[(3 * plane + 1) * ps + f] = md;
            ((uint16_t *)panels)[(3 * plane + 2) * ps + f] = l;
        }
    }
}

template <int FORM>
__global__ __launch_bounds__(PT) void prep_kernel(PrepArgs a) {
    __shared__ double red[4];
    __shared__ double sums[20 * 21 / 2 + 20];
    const int j = blockIdx.x;
    const int q = a.p - 1;
    const double h = a.h2[j];
    const double *y = a.yt + (int64_t)j * a.n_pad;

    for (int k = threadIdx.x; k < a.n_pad; k += PT) {
        const double d = k < a.n ? 1.0 / (h * a.w[k] + (1.0 - h)) : 0.0;
        put<FORM>(a.panels, 0, a.tcap, j, a.n_pad, k, d);
        for (int c = 0; c < q; ++c)
            put<FORM>(a.panels, 1 + c, a.tcap, j, a.n_pad, k, d * a.xlt[(int64_t)c * a.n_pad + k]);
        put<FORM>(a.panels, a.p, a.tcap, j, a.n_pad, k, d * y[k]);
    }

    // S_TL (packed lower, row-major) then b_T
    const int ntl = q * (q + 1) / 2;
    for (int s = 0; s < ntl + q; ++s) {
        int r, c;
        if (s < ntl) {
            r = 0;
            while ((r + 1) * (r + 2) / 2 <= s) ++r;
            c = s - r * (r + 1) / 2;
        } else {
            r = s - ntl;
            c = -1;
        }
        double v = 0.0;
        for (int k = threadIdx.x; k < a.n; k += PT) {
            const double d = 1.0 / (h * a.w[k] + (1.0 - h));
            const double xr = a.xlt[(int64_t)r * a.n_pad + k];
            const double o = c >= 0 ? a.xlt[(int64_t)c * a.n_pad + k] : y[k];
            v += d * xr * o;
        }
        v = block_sum(v, red);
        if (threadIdx.x == 0) sums[s] = v;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;

    // Cholesky of S_TL in place (lower, packed), with a relative pivot floor
    double *L = sums;
    bool ok = true;
    for (int jj = 0; jj < q && ok; ++jj) {
        double s = L[jj * (jj + 1) / 2 + jj];
        const double diag = s;
        for (int k = 0; k < jj; ++k) s -= L[jj * (jj + 1) / 2 + k] * L[jj * (jj + 1) / 2 + k];
        if (!(s > 1e-10 * diag) || !isfinite(s)) { ok = false; break; }
        const double dd = sqrt(s);
        L[jj * (jj + 1) / 2 + jj] = dd;
        for (int i = jj + 1; i < q; ++i) {
            double v = L[i * (i + 1) / 2 + jj];
            for (int k = 0; k < jj; ++k) v -= L[i * (i + 1) / 2 + k] * L[jj * (jj + 1) / 2 + k];
            L[i * (i + 1) / 2 + jj] = v / dd;
        }
    }
    double *F = a.fac + (int64_t)j * a.fac_stride;
    if (!ok) {
        for (int i = 0; i < a.fac_stride; ++i) F[i] = __builtin_nan("");
        return;
    }
    // L^{-1}, column by column (forward substitution on unit vectors)
    for (int c = 0; c < q; ++c) {
        for (int i = 0; i < q; ++i) {
            if (i < c) continue;
            double v = (i == c) ? 1.0 : 0.0;
            for (int k = c; k < i; ++k) v -= L[i * (i + 1) / 2 + k] * F[k * (k + 1) / 2 + c];
            F[i * (i + 1) / 2 + c] = v / L[i * (i + 1) / 2 + i];
        }
    }
    // z = L^{-1} b_T
    for (int i = 0; i < q; ++i) {
        double v = 0.0;
        for (int k = 0; k <= i; ++k) v += F[i * (i + 1) / 2 + k] * sums[ntl + k];
        F[ntl + i] = v;
    }
}

}  // namespace

hipError_t launch_prep(const PrepArgs &a, hipStream_t s) {
    if (a.tb <= 0) return hipSuccess;
    dim3 grid(a.tb), block(PT);
    switch (a.form) {
    case GWAS_FORM_F64: hipLaunchKernelGGL(prep_kernel<GWAS_FORM_F64>, grid, block, 0, s, a); break;
    case GWAS_FORM_F32: hipLaunchKernelGGL(prep_kernel<GWAS_FORM_F32>, grid, block, 0, s, a); break;
    case GWAS_FORM_BF16X3: hipLaunchKernelGGL(prep_kernel<GWAS_FORM_BF16X3>, grid, block, 0, s, a); break;
    case GWAS_FORM_BF16X6: hipLaunchKernelGGL(prep_kernel<GWAS_FORM_BF16X6>, grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace gw

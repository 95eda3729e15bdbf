// Rotation by Z^T (the preloop GEMMs of Algorithm 5, bundled over columns as
// Section 3.2 describes): every input column x (n samples) becomes x' = Z^T x.
// As a GEMM, out[i][k] = sum_r X[i][r] Z[k][r] (rows of Z are eigenvectors):
// both operands are contiguous along the samples r. FP64 and FP32 inputs are
// computed in FP64 MFMA (v_mfma_f64_16x16x4f64) over LDS-staged K chunks;
// genotype bytes only on the int8 MFMAs against Z sliced into int8 digits, whose
// sums are exact integers (the slicing of a floating-point operand into
// integer digits with exact integer products and sums follows Ozaki's scheme
// for emulating high-precision GEMM on integer matrix units).
//
// The rotated rows are written in every resident form at once: FP64, rounded
// to FP32, split to BF16 hi/lo, and split to BF16 hi/mid/lo (the splits of
// x'^2 are formed by the fused kernels from these).
#include <math.h>

#include <algorithm>
#include <type_traits>

#include "gwas_internal.h"
#include "lds_dma.h"

namespace gw {
namespace {

// TM input columns x TN rotated indices per workgroup of WM x WN waves; KC
// samples (doubles) staged per K chunk.
template <int TM_, int TN_, int KC_, int WM_, int WN_>
struct RotTile {
    static constexpr int TM = TM_, TN = TN_, KC = KC_, WM = WM_, WN = WN_;
    static constexpr int NT = 64 * WM * WN;
    static constexpr int FM = TM / WM / 16, FN = TN / WN / 16;
    static constexpr int LD = KC + 2;   // LDS row stride in doubles (16 bytes of padding)
    static constexpr int EA = TM * KC / NT;   // A elements loaded per thread per chunk
    static constexpr int EB = TN * KC / NT;   // B elements loaded per thread per chunk
    static_assert(FM >= 1 && FN >= 1 && EA >= 1 && EB >= 2 && KC % 8 == 0, "bad rotation tile");
    static constexpr int LDS = (TM + TN) * LD * 8;
};

// fastest of a tile sweep on MI355X (n = 1000)
using DefaultRot = RotTile<128, 64, 32, 4, 1>;
// few rows (a trait block): 4x the workgroups; 1000 x 1000 on MI355X 0.059 ms
// against 0.14 ms with the default tile
using SmallRot = RotTile<64, 32, 32, 4, 1>;

// One rotated value into every requested resident form.
__device__ __forceinline__ void rot_store(const RotOut &out, int64_t i, int k, double v) {
    const int64_t o = (out.row0 + i) * out.ld + k;
    if (out.f64) out.f64[o] = v;
    if (out.f32) out.f32[o] = (float)v;
    if (out.bf || out.bf3) {   // fragment-ordered planes (bf_frag_index)
        const int64_t f = bf_frag_index(out.row0 + i, k, out.ld);
        const int64_t ps = out.plane_rows * out.ld;
        if (out.bf) {
            uint16_t h, l;
            bf16_split((float)v, h, l);
            out.bf[f] = h;
            out.bf[ps + f] = l;
        }
        if (out.bf3) {
            uint16_t h, md, l;
            bf16_split3((float)v, h, md, l);
            out.bf3[f] = h;
            out.bf3[ps + f] = md;
            out.bf3[2 * ps + f] = l;
        }
    }
}

template <typename Tin, class R>
__global__ __launch_bounds__(R::NT) void rotate_kernel(const Tin *__restrict__ X, int64_t rows, int n,
                                                       int64_t ldx, const double *__restrict__ Zr,
                                                       int n_pad, RotOut out) {
    constexpr int TM = R::TM, TN = R::TN, KC = R::KC, LD = R::LD, FM = R::FM, FN = R::FN;
    extern __shared__ __attribute__((aligned(16))) double rot_lds[];
    double *la = rot_lds;
    double *lb = rot_lds + TM * LD;
    const int ntn = n_pad / TN;
    // XCD-aware order: each XCD keeps an eighth of Z's rows in its L2 and
    // streams the input columns (a bijection of the tiles; results unchanged)
    const int64_t tile = xcd_order(blockIdx.x, ntn);
    const int tn = (int)(tile % ntn);
    const int64_t tm = tile / ntn;
    const int64_t i_base = tm * TM;
    const int k_base = tn * TN;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave % R::WM, wn = wave / R::WM;
    const int l16 = lane & 15, g = lane >> 4;

    // loaders: thread covers EA consecutive samples of one input row and EB of one Z row
    constexpr int APR = KC / R::EA;   // threads per A row
    constexpr int BPR = KC / R::EB;
    const int arow = tid / APR, acol = (tid % APR) * R::EA;
    const int brow = tid / BPR, bcol = (tid % BPR) * R::EB;
    const int64_t gi = i_base + arow;
    const Tin *xrow = X + gi * ldx;
    const double *zrow = Zr + (int64_t)(k_base + brow) * n_pad;

    d4 acc[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

    double va[R::EA], vb[R::EB];
    auto gload = [&](int k0) {
#pragma unroll
        for (int e = 0; e < R::EA; ++e) {
            const int r = k0 + acol + e;
            va[e] = (gi < rows && r < n) ? (double)xrow[r] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < R::EB; e += 2) {
            const double2 z2 = *(const double2 *)(zrow + k0 + bcol + e);   // Z rows are n_pad long, zero beyond n
            vb[e] = z2.x;
            vb[e + 1] = z2.y;
        }
    };

    const int kend = (n + KC - 1) / KC * KC;   // <= n_pad (n_pad is a multiple of 64)
    gload(0);
    for (int k0 = 0; k0 < kend; k0 += KC) {
        __syncthreads();
#pragma unroll
        for (int e = 0; e < R::EA; ++e) la[arow * LD + acol + e] = va[e];
#pragma unroll
        for (int e = 0; e < R::EB; e += 2) *(double2 *)(lb + brow * LD + bcol + e) = double2{vb[e], vb[e + 1]};
        __syncthreads();
        if (k0 + KC < kend) gload(k0 + KC);
#pragma unroll
        for (int h = 0; h < KC / 8; ++h) {
            // lane group g reads samples 8h + 2g, 8h + 2g + 1 of its rows (same for A and B)
            double2 fa[FM], fb[FN];
#pragma unroll
            for (int a = 0; a < FM; ++a)
                fa[a] = *(const double2 *)(la + (wm * FM * 16 + a * 16 + l16) * LD + 8 * h + 2 * g);
#pragma unroll
            for (int b = 0; b < FN; ++b)
                fb[b] = *(const double2 *)(lb + (wn * FN * 16 + b * 16 + l16) * LD + 8 * h + 2 * g);
#pragma unroll
            for (int a = 0; a < FM; ++a)
#pragma unroll
                for (int b = 0; b < FN; ++b) {
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a].x, fb[b].x, acc[a][b], 0, 0, 0);
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a].y, fb[b].y, acc[a][b], 0, 0, 0);
                }
        }
    }

    // FP64 16x16 MFMA result: register r of lane group g is row g + 4r, column lane % 16.
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = i_base + wm * FM * 16 + a * 16 + mfma16_row<true>(g, r);
                const int k = k_base + wn * FN * 16 + b * 16 + l16;
                if (i < rows) rot_store(out, i, k, acc[a][b][r]);
            }
}


// Genotype rotation on the int8 MFMAs (v_mfma_i32_16x16x64_i8) with Z sliced
// into int8 digits (ZSlices). The genotype rows are first repacked on the
// device (pack_u8_kernel) into 1 KB fragment blocks, 16 rows x 64 samples, as
// signed bytes v - 128: lane l of a block owns bytes 16 l .. 16 l + 15, samples
// 16 (l / 16) .. + 15 of row l % 16 (-128 past n and past the rows: they meet
// zero Z columns or feed outputs that are not stored). Z block (d, cb) holds for
// lane l the same 16 samples of digit d of rotated index k0 + 16 cb + l % 16,
// so both operands put sample s in the same MFMA slot; one MFMA per (digit,
// SNP block, Z block) and 64-sample stage, exact int32 digit sums recombined
// in FP64 by the epilogue. Both operands are loaded by direct global->LDS
// copies, each block one contiguous 1 KB copy, into a ring of three stage
// buffers two stages ahead of the MFMAs; each wave waits only for the stage it
// is about to read (every wave issues the same number of copies per stage).
// Copying genotype blocks of 16 row segments straight from the caller's rows
// (4 bytes per lane, 16 rows x 16 bytes per instruction) measured slower on
// MI355X at n = 1000, m = 1e6 (six digits 8.57 against 7.14 ms, four digits
// 5.20 against 4.77, the repack included), and a row-major genotype block at
// an 80-byte pitch slower still (its 16-byte reads conflict on LDS banks).
template <int WM_, int WN_, int FM_, int FN_, int ND_ = kZSlices>
struct RotI8L {
    static constexpr int WM = WM_, WN = WN_, FM = FM_, FN = FN_, ND = ND_;   // ND leading digits
    static constexpr int NW = WM * WN, NT = 64 * NW;
    static constexpr int TM = WM * FM * 16, TN = WN * FN * 16;
    static constexpr int AB = TM / 16, CB = TN / 16;
    static constexpr int SBYTES = (AB + ND * CB) * 1024;   // genotype blocks, then Z (digit-major)
    static constexpr int NBUF = 3;
    static constexpr int LDS = NBUF * SBYTES;
    static constexpr int AI = AB / NW;                   // genotype block copies per wave and stage
    static constexpr int ZI = ND * CB / NW;              // Z block copies per wave and stage
    static constexpr int PER = AI + ZI;                  // copies per wave and stage
    static constexpr int NF = FM + ND * FN;              // fragments per wave and stage: genotype x, then (digit, y)
    static constexpr bool frag_is_b(int i) { return i >= FM; }
    static constexpr int frag_off(int i) {
        return i < FM ? i * 1024 : (((i - FM) / FN) * CB + (i - FM) % FN) * 1024;
    }
    static_assert(AB % NW == 0 && ND * CB % NW == 0, "every wave issues the same copies");
    static_assert(PER < 64 && SBYTES <= 65536 && LDS <= 160 * 1024, "rotation stage too large");
};

// fastest of sweeps on MI355X at n = 1000: 2 x 2 waves with six digits,
// 2 x 4 waves (twice the rotated indices per genotype block) with four; with
// the repacked genotypes also against 2 x 4 waves of 4 x 1 and 4 x 2 waves of
// 2 x 2 blocks (six digits: 9.0-9.2 against 7.1 ms at m = 1e6) and 2 x 2
// waves of 8 x 1 blocks (10.0 ms); four digits 4 x 2 waves of 4 x 2 and 2 x 2,
// 2 x 4 waves of 8 x 1 (5.0-5.4 against 4.8 ms)
template <int ND>
using DefaultRotI8L =
    typename std::conditional<ND == kZSlices, RotI8L<2, 2, 4, 1, ND>, RotI8L<2, 4, 4, 1, ND>>::type;

// P: the packed genotype blocks of `rows` rows (pack_u8_kernel), at least
// the tiles' rows (a multiple of TM) of them.
template <class R>
__global__ __launch_bounds__(R::NT) void rotate_u8_i8_lds_kernel(const uint8_t *__restrict__ P, int64_t rows, int n,
                                                                 ZSlices zs, int n_pad, RotOut out) {
    constexpr int TN = R::TN, FM = R::FM, FN = R::FN, ND = R::ND, CB = R::CB, AB = R::AB;
    extern __shared__ __attribute__((aligned(1024))) uint8_t lds[];
    const int ntn = n_pad / TN;
    const int64_t tile = tile_order(blockIdx.x, (rows + R::TM - 1) / R::TM, ntn);
    const int tn = (int)(tile % ntn);
    const int64_t tm = tile / ntn;
    const int64_t i_base = tm * R::TM;
    const int k_base = tn * TN;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave % R::WM, wn = wave / R::WM;
    const int g = lane >> 4;
    const int nst = (n + 63) / 64;   // stages of 64 samples; 64 nst <= n_pad

    // genotype copy u of this wave: block rb = wave + u NW of the tile, one
    // contiguous 1 KB block per stage
    const uint8_t *asrc[R::AI];
#pragma unroll
    for (int u = 0; u < R::AI; ++u)
        asrc[u] = P + ((i_base / 16 + wave + u * R::NW) * (int64_t)(n_pad / 64)) * 1024 + 16 * lane;
    // Z copy u: block b = d CB + cb holds for lane l the 16 bytes of digit d,
    // row k0 + 16 cb + l % 16, samples 16 (l / 16) .. + 15 (one stored block)
    const int8_t *zsrc[R::ZI];
    int zdst[R::ZI];
#pragma unroll
    for (int u = 0; u < R::ZI; ++u) {
        const int b = wave + u * R::NW, d = b / CB, cb = b % CB;
        zsrc[u] = zs.q + ((int64_t)d * (n_pad / 16) + k_base / 16 + cb) * (n_pad / 64) * 1024 + 16 * lane;
        zdst[u] = AB * 1024 + b * 1024;
    }
    auto issue = [&](int c) {
        uint8_t *buf = lds + (c % R::NBUF) * R::SBYTES;
#pragma unroll
        for (int u = 0; u < R::AI; ++u) lds_dma16(asrc[u] + (int64_t)c * 1024, buf + (wave + u * R::NW) * 1024);
#pragma unroll
        for (int u = 0; u < R::ZI; ++u) lds_dma16((const uint8_t *)(zsrc[u] + (int64_t)c * 1024), buf + zdst[u]);
    };

    i4v acc[ND][FM][FN];
#pragma unroll
    for (int d = 0; d < ND; ++d)
#pragma unroll
        for (int x = 0; x < FM; ++x)
#pragma unroll
            for (int y = 0; y < FN; ++y) acc[d][x][y] = i4v{0, 0, 0, 0};

    issue(0);
    if (nst > 1) issue(1);
    const uint32_t sa = lds_addr(lds) + lane * 16 + wm * FM * 1024;
    const uint32_t sz = lds_addr(lds) + lane * 16 + AB * 1024 + wn * FN * 1024;
    for (int c = 0; c < nst; ++c) {
        // this wave's copies of stage c landed; those of stage c + 1 may be in flight
        if (c + 1 < nst) __builtin_amdgcn_s_waitcnt(vmcnt_imm(R::PER));
        else __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
        // every wave's copies too; every wave has read stage c - 1 (its reads
        // waited for their data). A plain barrier: the fence of __syncthreads
        // would wait for the copies of stage c + 1 as well.
        __builtin_amdgcn_s_barrier();
        if (c + 2 < nst) issue(c + 2);   // into the buffer of stage c - 1
        const uint32_t so = (c % R::NBUF) * R::SBYTES;
        i4v f[R::NF];
        lds_read_frags<R, 0, R::NF>(f, sa + so, sz + so);
#pragma unroll
        for (int d = 0; d < ND; ++d)
#pragma unroll
            for (int y = 0; y < FN; ++y)
#pragma unroll
                for (int x = 0; x < FM; ++x)
                    acc[d][x][y] =
                        __builtin_amdgcn_mfma_i32_16x16x64_i8(f[x], f[FM + d * FN + y], acc[d][x][y], 0, 0, 0);
    }

    const int l16 = lane & 15;
#pragma unroll
    for (int y = 0; y < FN; ++y) {
        const int k = k_base + wn * FN * 16 + y * 16 + l16;
        // ND leading digits: the offset of their sum, and 2^-E_k times 256^(kZSlices - ND)
        const double off = zs.off[(ND == kZSlices ? 0 : n_pad) + k];
        const double sc = zs.scale[k] * (double)(1ull << (8 * (kZSlices - ND)));
#pragma unroll
        for (int x = 0; x < FM; ++x)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = i_base + wm * FM * 16 + x * 16 + mfma16_row<false>(g, r);
                double v = (double)acc[0][x][y][r];
#pragma unroll
                for (int d = 1; d < ND; ++d) v = fma(v, 256.0, (double)acc[d][x][y][r]);
                if (i < rows) rot_store(out, i, k, (v + off) * sc);
            }
    }
}

}  // namespace

void slice_z_int8(const double *zh, int n_pad, int8_t *q, double *off, double *scale) {
    static_assert(kZSlicesShort >= 1 && kZSlicesShort <= kZSlices, "digit counts");
    // byte of digit d, row k, sample r in fragment order (see ZSlices)
    auto at = [&](int d, int k, int r) -> int8_t & {
        const int64_t blk = ((int64_t)d * (n_pad / 16) + k / 16) * (n_pad / 64) + r / 64;
        return q[blk * 1024 + 16 * ((k % 16) + 16 * ((r % 64) / 16)) + r % 16];
    };
    for (int k = 0; k < n_pad; ++k) {
        const double *z = zh + (int64_t)k * n_pad;
        double mx = 0.0;
        for (int r = 0; r < n_pad; ++r) mx = std::max(mx, fabs(z[r]));
        int e = 0;
        frexp(mx, &e);                            // mx < 2^e
        const int E = 8 * kZSlices - 2 - e;       // |z| 2^E < 2^(8 kZSlices - 2)
        scale[k] = mx > 0.0 ? ldexp(1.0, -E) : 0.0;
        __int128 sum = 0, sum_short = 0;
        for (int r = 0; r < n_pad; ++r) {
            int64_t v = mx > 0.0 ? llround(ldexp(z[r], E)) : 0;
            sum += v;
            int64_t dig[kZSlices];
            for (int d = kZSlices - 1; d >= 1; --d) {   // balanced base-256 digits, low first
                int64_t t = v & 255;
                if (t >= 128) t -= 256;
                dig[d] = t;
                v = (v - t) / 256;
            }
            dig[0] = v;                                 // |v| <= 65
            int64_t q_short = 0;                        // the leading kZSlicesShort digits
            for (int d = 0; d < kZSlices; ++d) {
                at(d, k, r) = (int8_t)dig[d];
                if (d < kZSlicesShort) q_short = q_short * 256 + dig[d];
            }
            sum_short += q_short;
        }
        off[k] = 128.0 * (double)sum;
        off[n_pad + k] = 128.0 * (double)sum_short;
    }
}

template <class R>
hipError_t launch_rotate_t(const void *X, int dtype, int64_t rows, int n, int64_t ldx, const double *Zrows,
                           int n_pad, const RotOut &out, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    if (n_pad % R::TN) return hipErrorInvalidValue;
    const int64_t tiles = ((rows + R::TM - 1) / R::TM) * (n_pad / R::TN);
    dim3 grid((unsigned)tiles), block(R::NT);
    if (R::LDS > 65536) {
        static bool attr_set = false;   // per instantiation
        if (!attr_set) {
            hipError_t e = hipFuncSetAttribute((const void *)rotate_kernel<double, R>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, R::LDS);
            if (e == hipSuccess)
                e = hipFuncSetAttribute((const void *)rotate_kernel<float, R>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, R::LDS);
            if (e != hipSuccess) return e;
            attr_set = true;
        }
    }
    switch (dtype) {
    case GWAS_DT_F64:
        hipLaunchKernelGGL((rotate_kernel<double, R>), grid, block, R::LDS, s, (const double *)X, rows, n, ldx,
                           Zrows, n_pad, out);
        break;
    case GWAS_DT_F32:
        hipLaunchKernelGGL((rotate_kernel<float, R>), grid, block, R::LDS, s, (const float *)X, rows, n, ldx,
                           Zrows, n_pad, out);
        break;
    default:   // genotype bytes go to the int8 digit kernels only
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Genotype rows -> fragment blocks for rotate_u8_i8_lds_kernel: block
// (rg, c) = rows 16 rg .. + 15, samples 64 c .. + 63, at P + (rg (n_pad / 64)
// + c) KB; thread t writes the 16 bytes of lane t % 64 of block t / 64 as
// signed bytes v - 128 (byte v XOR 0x80; -128 past n and past `rows`). Rows,
// stride and base aligned to 4 bytes (aligned4) are read a word at a time,
// any others byte by byte.
__global__ void pack_u8_kernel(const uint8_t *__restrict__ X, int64_t rows, int n, int64_t ldx, int n_pad,
                               int64_t units, uint8_t *__restrict__ P, int aligned4) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= units) return;
    const int l = (int)(t & 63);
    const int64_t blk = t >> 6;
    const int nkb = n_pad / 64;
    const int c = (int)(blk % nkb);
    const int64_t row = (blk / nkb) * 16 + (l & 15);
    const int s0 = c * 64 + 16 * (l >> 4);
    uint32_t w[4] = {0u, 0u, 0u, 0u};
    if (row < rows) {
        const uint8_t *src = X + row * ldx;
        if (aligned4) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (s0 + 4 * q < n) w[q] = *(const uint32_t *)(src + s0 + 4 * q);   // n % 4 == 0
        } else {
            for (int e = 0; e < 16; ++e)
                if (s0 + e < n) w[e >> 2] |= (uint32_t)src[s0 + e] << (8 * (e & 3));
        }
    }
    *(uint4 *)(P + t * 16) = make_uint4(w[0] ^ 0x80808080u, w[1] ^ 0x80808080u, w[2] ^ 0x80808080u, w[3] ^ 0x80808080u);
}

// Rows in chunks of zs.pack_rows: pack the chunk into zs.pack, rotate it.
template <class R>
hipError_t launch_rotate_u8_i8_t(const uint8_t *X, int64_t rows, int n, int64_t ldx, const ZSlices &zs, int n_pad,
                                 const RotOut &out, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    if (n_pad % R::TN || n_pad % 64 || n > n_pad || n_pad > kZSliceMaxNpad || !zs.pack || zs.pack_rows <= 0 ||
        zs.pack_rows % 256)
        return hipErrorInvalidValue;
    static_assert(256 % R::TM == 0, "a chunk of whole tiles");
    if (R::LDS > 65536) {
        static bool attr_set = false;   // per instantiation
        if (!attr_set) {
            hipError_t e = hipFuncSetAttribute((const void *)rotate_u8_i8_lds_kernel<R>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, R::LDS);
            if (e != hipSuccess) return e;
            attr_set = true;
        }
    }
    const int aligned4 = (n % 4 == 0 && ldx % 4 == 0 && ((uintptr_t)X) % 4 == 0) ? 1 : 0;
    for (int64_t r0 = 0; r0 < rows; r0 += zs.pack_rows) {
        const int64_t cnt = std::min(zs.pack_rows, rows - r0);
        const int64_t units = (cnt + R::TM - 1) / R::TM * R::TM / 16 * (n_pad / 64) * 64;   // <= pack_rows n_pad / 16
        hipLaunchKernelGGL(pack_u8_kernel, dim3((unsigned)((units + 255) / 256)), dim3(256), 0, s, X + r0 * ldx, cnt,
                           n, ldx, n_pad, units, zs.pack, aligned4);
        RotOut o = out;
        o.row0 += r0;
        const int64_t tiles = ((cnt + R::TM - 1) / R::TM) * (n_pad / R::TN);
        hipLaunchKernelGGL((rotate_u8_i8_lds_kernel<R>), dim3((unsigned)tiles), dim3(R::NT), R::LDS, s,
                           (const uint8_t *)zs.pack, cnt, n, zs, n_pad, o);
    }
    return hipGetLastError();
}

hipError_t launch_rotate(const void *X, int dtype, int64_t rows, int n, int64_t ldx, const double *Zrows,
                         int n_pad, const RotOut &out, hipStream_t s, const ZSlices *zs) {
    // all digits when an FP64 store is written, the leading ones otherwise
    const bool full = out.f64 != nullptr;
    if (dtype == GWAS_DT_U8 && zs && zs->q && zs->pack && n_pad <= kZSliceMaxNpad &&
        n_pad % DefaultRotI8L<kZSlices>::TN == 0 && n_pad % DefaultRotI8L<kZSlicesShort>::TN == 0)
        return full ? launch_rotate_u8_i8_t<DefaultRotI8L<kZSlices>>((const uint8_t *)X, rows, n, ldx, *zs, n_pad,
                                                                     out, s)
                    : launch_rotate_u8_i8_t<DefaultRotI8L<kZSlicesShort>>((const uint8_t *)X, rows, n, ldx, *zs,
                                                                          n_pad, out, s);
    if (dtype == GWAS_DT_U8) return hipErrorInvalidValue;   // needs the digits of Z and the pack buffer
    const int64_t wgs = ((rows + DefaultRot::TM - 1) / DefaultRot::TM) * (n_pad / DefaultRot::TN);
    if (wgs < 1024 && n_pad % SmallRot::TN == 0)   // fewer than 4 workgroups per CU
        return launch_rotate_t<SmallRot>(X, dtype, rows, n, ldx, Zrows, n_pad, out, s);
    return launch_rotate_t<DefaultRot>(X, dtype, rows, n, ldx, Zrows, n_pad, out, s);
}

}  // namespace gw

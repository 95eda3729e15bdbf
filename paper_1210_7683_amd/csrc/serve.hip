// Grouped launch of the serving loop: the tiles of every work item of a
// scheduling round (one SNP slab of each admitted request, each with its own
// trait count, covariate count and panels) run in one launch. Workgroups take
// tile indices from a counter in device memory until the round's list is
// exhausted, so uneven items balance across the chip and every workgroup
// reaches the exit; a switch on the item's p selects the tile code
// specialised for that design width (the same code for a request alone or in
// any mix, so its results are the same).
#include "serve.h"

#include "fused_dma.h"

namespace gw {
namespace {

// Tile code of the direct solve (fused_dma.h) with one workgroup shape for all
// p of a launch: the direct solve's tiles for p = 5..9 (8 waves; FP64 and FP32
// 128 SNPs x 16 traits, split BF16 256 x 16, three-piece 128 x 16).
// Requests have few traits, so narrow trait tiles waste little; a problem's
// sums take the same MFMAs in the same order as in every direct-solve kernel.
// The three-piece split BF16 form always folds its FP32 sums into FP64 per stage.
template <int FORM, bool FLUSH>
struct ServeTile {
    using type = typename std::conditional<FORM == GWAS_FORM_F64, DmaTile<8, 1, 1, 1, 1>,
                 typename std::conditional<FORM == GWAS_FORM_F32, DmaTile<8, 1, 1, 1, 2, true>,
                 typename std::conditional<FORM == GWAS_FORM_BF16X3, DmaTile<8, 1, 2, 1, 1, true>,
                                           DmaTile<8, 1, 1, 1, 1, true>>::type>::type>::type;
    static_assert(FORM != GWAS_FORM_BF16X6 || FLUSH, "the three-piece form folds every stage");
};

template <int FORM, bool FLUSH>
struct ServeCfg {
    using T = typename ServeTile<FORM, FLUSH>::type;
    using C8 = DmaCfg<FORM, kServeMaxP, T>;   // the largest p needs the most LDS
    static constexpr int NT = C8::NT;
    static constexpr int LDS = C8::LDS;
};

template <int FORM, bool FLUSH>
__global__ __launch_bounds__((ServeCfg<FORM, FLUSH>::NT)) void serve_kernel(ServeBatch bt) {
    using T = typename ServeTile<FORM, FLUSH>::type;
    extern __shared__ __attribute__((aligned(1024))) uint8_t lds[];
    __shared__ unsigned long long next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(bt.counter, 1ull);
        __syncthreads();
        const int64_t tile = (int64_t)(next - bt.counter_base);
        __syncthreads();   // every thread has read `next` before it is overwritten
        if (tile >= bt.total_tiles) return;
        int it = 0;
        while (it + 1 < bt.n_items && bt.items[it + 1].tile0 <= tile) ++it;
        const ServeItem &s = bt.items[it];
        FusedArgs fa{};
        fa.a = bt.a;
        fa.a_plane_rows = bt.a_plane_rows;
        fa.i0 = s.i0;
        fa.mi = s.mi;
        fa.row_lo = s.row_lo;
        fa.panels = s.panels;
        fa.tcap = s.tcap;
        fa.fac = s.fac;
        fa.fac_stride = s.fac_stride;
        fa.tb = s.tb;
        fa.n_pad = bt.n_pad;
        fa.n = bt.n;
        fa.p = s.p;
        fa.b = s.b;
        fa.ldt = s.tb;
        fa.rank_rtol = bt.rank_rtol;
        fa.non_spd = bt.non_spd;
        fa.f32_flush = bt.f32_flush;
        const int64_t local = tile - s.tile0;
        switch (s.p) {
        case 2: dma_tile<FORM, 2, FLUSH, T>(fa, local, lds); break;
        case 3: dma_tile<FORM, 3, FLUSH, T>(fa, local, lds); break;
        case 4: dma_tile<FORM, 4, FLUSH, T>(fa, local, lds); break;
        case 5: dma_tile<FORM, 5, FLUSH, T>(fa, local, lds); break;
        case 6: dma_tile<FORM, 6, FLUSH, T>(fa, local, lds); break;
        case 7: dma_tile<FORM, 7, FLUSH, T>(fa, local, lds); break;
        default: dma_tile<FORM, 8, FLUSH, T>(fa, local, lds); break;
        }
    }
}

template <int FORM, bool FLUSH>
hipError_t launch_serve_t(const ServeBatch &bt, int grid, hipStream_t s) {
    using SC = ServeCfg<FORM, FLUSH>;
    static bool attr_set = false;
    if (SC::LDS > 65536 && !attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)serve_kernel<FORM, FLUSH>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, SC::LDS);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL((serve_kernel<FORM, FLUSH>), dim3(grid), dim3(SC::NT), SC::LDS, s, bt);
    return hipGetLastError();
}

template <int FORM, bool FLUSH>
int occupancy_t() {
    using SC = ServeCfg<FORM, FLUSH>;
    if (SC::LDS > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)serve_kernel<FORM, FLUSH>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, SC::LDS);
        if (e != hipSuccess) return 1;
    }
    int n = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, serve_kernel<FORM, FLUSH>, SC::NT, SC::LDS) != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

template <int FORM, bool FLUSH>
void tile_shape_t(int p, int &tm, int &tn) {
    using T = typename ServeTile<FORM, FLUSH>::type;
    switch (p) {
#define GW_SHAPE(PP) case PP: tm = DmaCfg<FORM, PP, T>::TM; tn = DmaCfg<FORM, PP, T>::TN; return;
        GW_SHAPE(2) GW_SHAPE(3) GW_SHAPE(4) GW_SHAPE(5) GW_SHAPE(6) GW_SHAPE(7)
#undef GW_SHAPE
    default: tm = DmaCfg<FORM, 8, T>::TM; tn = DmaCfg<FORM, 8, T>::TN; return;
    }
}

}  // namespace

void serve_tile_shape(int form, bool flush, int p, int &tm, int &tn) {
    if (form == GWAS_FORM_F64) tile_shape_t<GWAS_FORM_F64, false>(p, tm, tn);
    else if (form == GWAS_FORM_BF16X6) tile_shape_t<GWAS_FORM_BF16X6, true>(p, tm, tn);
    else if (form == GWAS_FORM_F32 && flush) tile_shape_t<GWAS_FORM_F32, true>(p, tm, tn);
    else if (form == GWAS_FORM_F32) tile_shape_t<GWAS_FORM_F32, false>(p, tm, tn);
    else tile_shape_t<GWAS_FORM_BF16X3, false>(p, tm, tn);
}

int serve_occupancy(int form, bool flush) {
    if (form == GWAS_FORM_F64) return occupancy_t<GWAS_FORM_F64, false>();
    if (form == GWAS_FORM_BF16X6) return occupancy_t<GWAS_FORM_BF16X6, true>();
    if (form == GWAS_FORM_F32 && flush) return occupancy_t<GWAS_FORM_F32, true>();
    if (form == GWAS_FORM_F32) return occupancy_t<GWAS_FORM_F32, false>();
    return occupancy_t<GWAS_FORM_BF16X3, false>();
}

hipError_t launch_serve(int form, bool flush, const ServeBatch &bt, int grid, hipStream_t s) {
    if (grid <= 0 || bt.total_tiles <= 0) return hipSuccess;
    if (form == GWAS_FORM_F64) return launch_serve_t<GWAS_FORM_F64, false>(bt, grid, s);
    if (form == GWAS_FORM_BF16X6) return launch_serve_t<GWAS_FORM_BF16X6, true>(bt, grid, s);
    if (form == GWAS_FORM_F32 && flush) return launch_serve_t<GWAS_FORM_F32, true>(bt, grid, s);
    if (form == GWAS_FORM_F32) return launch_serve_t<GWAS_FORM_F32, false>(bt, grid, s);
    return launch_serve_t<GWAS_FORM_BF16X3, false>(bt, grid, s);
}

}  // namespace gw

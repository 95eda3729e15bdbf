// Grouped launch of the serving loop (work items of several requests in one launch).
#pragma once

#include "gwas_internal.h"

namespace gw {

constexpr int kServeMaxP = 8;       // largest design width a request may use
constexpr int kServeMaxItems = 32;  // work items per launch (one per admitted request)

// One work item: a slab of SNPs of one request against all its traits.
struct ServeItem {
    const void *panels;   // the request's trait panels (plane stride tcap = tb rounded up to 16 rows)
    const double *fac;    // its per-trait factors
    void *b;              // device staging for the slab's b: mi x tb x p
    int64_t i0, mi;       // SNP range
    int64_t row_lo;       // rows [i0, i0 + row_lo) computed but not stored (FusedArgs::row_lo)
    int64_t tile0;        // first tile index of this item within the launch
    int32_t tb, p, tcap, fac_stride;
};

struct ServeBatch {
    const void *a;               // resident rotated SNPs of the form
    int64_t a_plane_rows;
    // Tile counter, never reset: every workgroup takes tiles with an atomic add
    // until it draws one past the round's list, so one round advances it by
    // exactly total_tiles + grid, and the next round's tiles start there.
    unsigned long long *counter;
    unsigned long long counter_base;   // the counter's value when this round starts
    unsigned long long *non_spd;
    int64_t total_tiles;
    double rank_rtol;
    int32_t n_pad, f32_flush, n_items, n;   // n: samples (zeros from n to n_pad)
    ServeItem items[kServeMaxItems];
};

// Tile shape (SNPs x traits per tile) of the serving kernel for a form and p.
void serve_tile_shape(int form, bool flush, int p, int &tm, int &tn);

// Workgroups of the serving kernel that fit one CU at once (LDS, registers).
int serve_occupancy(int form, bool flush);

// Launch `grid` persistent workgroups over the batch's tiles.
hipError_t launch_serve(int form, bool flush, const ServeBatch &bt, int grid, hipStream_t s);

}  // namespace gw

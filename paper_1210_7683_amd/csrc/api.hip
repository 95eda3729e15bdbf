// C ABI of libgwas: context, resident cohort, rotation, solve, streaming of b.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "ctx.h"

using namespace gw;


// the tile orders of the fused and rotation kernels cover every tile once, on
// shapes that take each branch (whole and partial groups of 8 rows, tails of
// 1 to 7 column tiles, multiples of 8, fewer than 8)
static_assert(gw::tile_order_is_bijection<13, 63>() && gw::tile_order_is_bijection<16, 9>() &&
                  gw::tile_order_is_bijection<7, 20>() && gw::tile_order_is_bijection<9, 8>() &&
                  gw::tile_order_is_bijection<3, 5>() && gw::tile_order_is_bijection<24, 15>() &&
                  gw::tile_order_is_bijection<98, 63>() && gw::tile_order_is_bijection<1, 17>(),
              "tile_order must be a bijection");
namespace gw {
std::string &last_error() {
    thread_local std::string e;
    return e;
}
}  // namespace gw

namespace {

template <typename T>
gwas_status dalloc(gwas_ctx *c, T **p, size_t bytes) {
    void *v = nullptr;
    hipError_t e = hipMalloc(&v, bytes ? bytes : 16);
    if (e != hipSuccess)
        return fail(e == hipErrorOutOfMemory ? GWAS_ENOMEM : GWAS_EHIP, "hipMalloc(%zu): %s", bytes,
                    hipGetErrorString(e));
    e = hipMemset(v, 0, bytes ? bytes : 16);
    if (e != hipSuccess) return fail(GWAS_EHIP, "hipMemset: %s", hipGetErrorString(e));
    *p = (T *)v;
    c->resident += (int64_t)bytes;
    return GWAS_OK;
}

hipError_t timed_begin(gwas_ctx *c, hipStream_t s, std::pair<hipEvent_t, hipEvent_t> &ev) {
    if (!c->timing) return hipSuccess;
    if (!c->t_pool.empty()) {
        ev = c->t_pool.back();
        c->t_pool.pop_back();
    } else {
        hipError_t e = hipEventCreate(&ev.first);
        if (e == hipSuccess) e = hipEventCreate(&ev.second);
        if (e != hipSuccess) return e;
    }
    return hipEventRecord(ev.first, s);
}

hipError_t timed_end(gwas_ctx *c, hipStream_t s, std::pair<hipEvent_t, hipEvent_t> &ev,
                     std::vector<std::pair<hipEvent_t, hipEvent_t>> &list) {
    if (!c->timing) return hipSuccess;
    hipError_t e = hipEventRecord(ev.second, s);
    list.push_back(ev);
    return e;
}

double drain(gwas_ctx *c, std::vector<std::pair<hipEvent_t, hipEvent_t>> &list, int64_t &count) {
    double tot = 0.0;
    for (auto &ev : list) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev.first, ev.second) == hipSuccess) tot += ms;
        c->t_pool.push_back(ev);
    }
    count = (int64_t)list.size();
    list.clear();
    return tot;
}

void release(gwas_ctx *c) {
    if (!c) return;
    hipSetDevice(c->dev);
    hipDeviceSynchronize();
    for (auto *lst : {&c->t_fused, &c->t_rot, &c->t_pool})
        for (auto &ev : *lst) {
            hipEventDestroy(ev.first);
            hipEventDestroy(ev.second);
        }
    void *ptrs[] = {c->Z, c->w, c->xlt, c->xr64, c->xr32, c->xrbf, c->y_in, c->yt, c->h2,
                    c->panels[0], c->panels[1], c->panels[2], c->panels[3], c->xrbf3, c->fac, c->counters, c->stage,
                    c->bstage[0], c->bstage[1], c->xin[0], c->xin[1], c->zq, c->zoff, c->zscale, c->zpack};
    for (void *p : ptrs)
        if (p) hipFree(p);
    for (int i = 0; i < 2; ++i) {
        if (c->ev_done[i]) hipEventDestroy(c->ev_done[i]);
        if (c->ev_free[i]) hipEventDestroy(c->ev_free[i]);
        if (c->ev_rot[i]) hipEventDestroy(c->ev_rot[i]);
        if (c->ev_half[i]) hipEventDestroy(c->ev_half[i]);
    }
    if (c->aux) hipStreamDestroy(c->aux);
    if (c->ev_side) hipEventDestroy(c->ev_side);
    for (void *p : c->ring)
        if (p) hipHostFree(p);
    for (hipEvent_t e : c->ring_ev)
        if (e) hipEventDestroy(e);
    if (c->side) hipStreamDestroy(c->side);
    delete c;
}

bool all_finite(const double *v, size_t count) {
    for (size_t i = 0; i < count; ++i)
        if (!isfinite(v[i])) return false;
    return true;
}

size_t elt_size(int form) { return form == GWAS_FORM_F64 ? 8 : (form == GWAS_FORM_F32 ? 4 : 2); }

// planes per trait panel (and per SNP row) of a form: the BF16 pieces
int panel_planes(int form) { return form == GWAS_FORM_BF16X3 ? 2 : (form == GWAS_FORM_BF16X6 ? 3 : 1); }

}  // namespace

// Scratch of gwas_solve_noalloc: one fixed array per device (each GPU the
// library runs on holds its own copy until the process ends). It holds one
// trait sub-block at a time (staged and rotated traits, h2, panels, factors,
// tile counters); calls on one device share it.
constexpr size_t kNoAllocScratchBytes = (size_t)32 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

namespace {

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on device dev, which must be current. The
// array's name in host code is a host-side stand-in, not a device address:
// host code uses only the pointer obtained here.
gwas_status noalloc_scratch(int dev, void **ptr) {
    if (dev < 0 || dev >= kMaxDevices) return fail(GWAS_EINVAL, "device %d outside [0, %d)", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(GWAS_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return GWAS_OK;
}

}  // namespace

namespace gw {
hipError_t launch_fused(int form, const FusedArgs &a0, hipStream_t s) {
    FusedArgs a = a0;
    if ((form == GWAS_FORM_BF16X3 || form == GWAS_FORM_BF16X6) && (a.i0 & 15)) {
        // the fragment-ordered store is staged by whole 16-row groups: start the
        // range at the group and leave its first rows unstored
        a.row_lo = a.i0 & 15;
        a.i0 -= a.row_lo;
        a.mi += a.row_lo;
    }
    switch (form) {
    case GWAS_FORM_F64: return launch_fused_f64(a, s);
    case GWAS_FORM_F32: return launch_fused_f32(a, s);
    case GWAS_FORM_BF16X3: return launch_fused_bf16(a, s);
    case GWAS_FORM_BF16X6: return launch_fused_bf16x6(a, s);
    default: return hipErrorInvalidValue;
    }
}
}  // namespace gw

extern "C" {

const char *gwas_last_error(void) { return last_error().c_str(); }

const char *gwas_version(void) { return "libgwas 0.1 (gfx950)"; }

void gwas_default_options(gwas_options *opt) {
    if (!opt) return;
    memset(opt, 0, sizeof *opt);
    opt->forms = 0;
    opt->device = -1;
    opt->max_traits = 1024;
    opt->slab_snps = 0;
    opt->f32_flush = 2;
}

gwas_status gwas_setup(gwas_ctx **out, int32_t n, int32_t p, const double *Z, const double *w,
                       const double *X_L, const gwas_options *opt) {
    last_error().clear();
    if (!out) return fail(GWAS_EINVAL, "ctx pointer is NULL");
    *out = nullptr;
    if (n < 1 || n > 16384) return fail(GWAS_EINVAL, "n = %d outside [1, 16384]", n);
    if (p < 2 || p > 20) return fail(GWAS_EINVAL, "p = %d outside [2, 20]", p);
    if (!Z || !w || !X_L || !opt) return fail(GWAS_EINVAL, "NULL input pointer");
    if (opt->m_capacity <= 0) return fail(GWAS_EINVAL, "m_capacity must be positive");
    if (opt->max_traits < 0 || opt->slab_snps < 0 || opt->f32_flush < 0 || opt->ring_slots < 0 ||
        opt->host_threads < 0 || opt->ring_slots > 64 || opt->host_threads > 256)
        return fail(GWAS_EINVAL, "negative option");
    if (opt->geno_chunk_snps < 0 || opt->geno_chunk_snps % 256)
        return fail(GWAS_EINVAL, "geno_chunk_snps = %d: a non-negative multiple of 256", opt->geno_chunk_snps);
    if (opt->f32_flush != 0 && opt->f32_flush != 2)
        return fail(GWAS_EINVAL, "f32_flush = %d: 0 (no fold) or 2 (FP64 folds, the default)", opt->f32_flush);
    const uint32_t forms = opt->forms ? opt->forms : 7u;
    if (forms & ~15u) return fail(GWAS_EINVAL, "unknown form bits 0x%x", forms);
    if (!all_finite(Z, (size_t)n * n) || !all_finite(w, n) || !all_finite(X_L, (size_t)n * (p - 1)))
        return fail(GWAS_EINVAL, "non-finite value in Z, w or X_L");

    gwas_ctx *c = new gwas_ctx();
    int dev = opt->device;
    if (dev < 0) {
        if (hipGetDevice(&dev) != hipSuccess) { delete c; return fail(GWAS_EHIP, "hipGetDevice failed"); }
    }
    c->dev = dev;
    if (hipSetDevice(dev) != hipSuccess) { delete c; return fail(GWAS_EINVAL, "bad device %d", dev); }
    {   // the device's address of the no-allocation scratch, taken once per device
        void *sp = nullptr;
        gwas_status sst = noalloc_scratch(dev, &sp);
        if (sst != GWAS_OK) { delete c; return sst; }
    }
    c->n = n;
    c->n_pad = (int)round_up(n, kPadN);
    c->p = p;
    c->m_cap = opt->m_capacity;
    c->m_rows = round_up(opt->m_capacity, 256);
    c->forms = forms;
    c->tcap = opt->max_traits ? opt->max_traits : 1024;
    c->f32_flush = opt->f32_flush;
    c->timing = opt->timing != 0;
    c->ring_slots = opt->ring_slots > 0 ? opt->ring_slots : 4;
    c->host_threads = opt->host_threads > 0 ? opt->host_threads : 8;
    c->w_min = *std::min_element(w, w + n);

    gwas_status st;
    const int np = c->n_pad;
#define TRY(x) do { if ((st = (x)) != GWAS_OK) { release(c); return st; } } while (0)
    TRY(dalloc(c, &c->Z, sizeof(double) * np * np));
    if (np <= kZSliceMaxNpad) {
        TRY(dalloc(c, &c->zq, (size_t)kZSlices * np * np));
        TRY(dalloc(c, &c->zoff, sizeof(double) * 2 * np));
        TRY(dalloc(c, &c->zscale, sizeof(double) * np));
        c->zpack_rows = opt->geno_chunk_snps ? opt->geno_chunk_snps
                                             : std::max<int64_t>(256, kGenoPackBytes / np / 256 * 256);
        TRY(dalloc(c, &c->zpack, (size_t)c->zpack_rows * np));
    }
    TRY(dalloc(c, &c->w, sizeof(double) * np));
    TRY(dalloc(c, &c->xlt, sizeof(double) * (size_t)(p - 1) * np));
    const size_t plane = (size_t)c->m_rows * np;
    if (forms & GWAS_FORM_BIT(GWAS_FORM_F64)) TRY(dalloc(c, &c->xr64, sizeof(double) * plane));
    if (forms & GWAS_FORM_BIT(GWAS_FORM_F32)) TRY(dalloc(c, &c->xr32, sizeof(float) * plane));
    if (forms & GWAS_FORM_BIT(GWAS_FORM_BF16X3)) TRY(dalloc(c, &c->xrbf, sizeof(uint16_t) * 2 * plane));
    if (forms & GWAS_FORM_BIT(GWAS_FORM_BF16X6)) TRY(dalloc(c, &c->xrbf3, sizeof(uint16_t) * 3 * plane));
    TRY(dalloc(c, &c->y_in, sizeof(double) * (size_t)c->tcap * n));
    TRY(dalloc(c, &c->yt, sizeof(double) * (size_t)c->tcap * np));
    TRY(dalloc(c, &c->h2, sizeof(double) * (size_t)c->tcap));
    for (int f = 0; f < 4; ++f)
        if (forms & GWAS_FORM_BIT(f)) {
            const size_t planes = (size_t)panel_planes(f) * (p + 1);
            TRY(dalloc(c, &c->panels[f], elt_size(f) * planes * panel_rows(c->tcap) * np));
        }
    TRY(dalloc(c, &c->fac, sizeof(double) * (size_t)c->tcap * fac_stride(p)));
    // [0..3] statistics, [4..7] the 8 tile counters of persistent launches
    TRY(dalloc(c, &c->counters, sizeof(unsigned long long) * 8));
    c->stage_bytes = (size_t)64 << 20;
    TRY(dalloc(c, &c->stage, c->stage_bytes));

    // upload Z (row k = eigenvector k, padded), w, X_L; rotate X_L in FP64
    {
        double *zh = (double *)calloc((size_t)np * np, sizeof(double));
        if (!zh) { release(c); return fail(GWAS_ENOMEM, "host allocation"); }
        for (int k = 0; k < n; ++k) memcpy(zh + (size_t)k * np, Z + (size_t)k * n, sizeof(double) * n);
        hipError_t e = hipMemcpy(c->Z, zh, sizeof(double) * np * np, hipMemcpyHostToDevice);
        if (e == hipSuccess && c->zq) {   // int8 digits of Z for the genotype rotation
            std::vector<int8_t> q((size_t)kZSlices * np * np);
            std::vector<double> off(2 * (size_t)np), sc(np);
            slice_z_int8(zh, np, q.data(), off.data(), sc.data());
            e = hipMemcpy(c->zq, q.data(), q.size(), hipMemcpyHostToDevice);
            if (e == hipSuccess) e = hipMemcpy(c->zoff, off.data(), sizeof(double) * 2 * np, hipMemcpyHostToDevice);
            if (e == hipSuccess) e = hipMemcpy(c->zscale, sc.data(), sizeof(double) * np, hipMemcpyHostToDevice);
        }
        free(zh);
        if (e != hipSuccess) { release(c); return fail(GWAS_EHIP, "upload Z: %s", hipGetErrorString(e)); }
        double *wh = (double *)malloc(sizeof(double) * np);
        for (int k = 0; k < np; ++k) wh[k] = k < n ? w[k] : 1.0;
        e = hipMemcpy(c->w, wh, sizeof(double) * np, hipMemcpyHostToDevice);
        free(wh);
        if (e != hipSuccess) { release(c); return fail(GWAS_EHIP, "upload w: %s", hipGetErrorString(e)); }
        e = hipMemcpy(c->stage, X_L, sizeof(double) * (size_t)n * (p - 1), hipMemcpyHostToDevice);
        if (e != hipSuccess) { release(c); return fail(GWAS_EHIP, "upload X_L: %s", hipGetErrorString(e)); }
        RotOut ro{c->xlt, nullptr, nullptr, nullptr, 0, 0, np};
        e = launch_rotate(c->stage, GWAS_DT_F64, p - 1, n, n, c->Z, np, ro, nullptr);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) { release(c); return fail(GWAS_EHIP, "rotate X_L: %s", hipGetErrorString(e)); }
        c->bytes_h2d += (int64_t)sizeof(double) * ((int64_t)n * n + n + (int64_t)n * (p - 1));
    }

    // D2H streaming: two staging buffers for b slabs, a side stream, events
    c->slab = opt->slab_snps ? opt->slab_snps : (int)std::min<int64_t>(c->m_rows, 16384);
    c->bstage_bytes = (size_t)c->slab * c->tcap * p * sizeof(double);
    if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess) {
        release(c); return fail(GWAS_EHIP, "stream creation failed");
    }
    for (int i = 0; i < 2; ++i) {
        if (hipEventCreateWithFlags(&c->ev_done[i], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&c->ev_free[i], hipEventDisableTiming) != hipSuccess) {
            release(c); return fail(GWAS_EHIP, "event creation failed");
        }
    }
    if (hipEventCreateWithFlags(&c->ev_side, hipEventDisableTiming) != hipSuccess) {
        release(c); return fail(GWAS_EHIP, "event creation failed");
    }
#undef TRY
    *out = c;
    return GWAS_OK;
}

gwas_status gwas_rotate(gwas_ctx *c, int64_t m0, int64_t mb, const void *X, int32_t dtype,
                        int32_t on_device, void *stream) {
    last_error().clear();
    if (!c) return fail(GWAS_EINVAL, "ctx is NULL");
    if (m0 < 0 || mb < 0 || m0 + mb > c->m_cap)
        return fail(GWAS_EINVAL, "SNP range [%lld, %lld) outside capacity %lld", (long long)m0,
                    (long long)(m0 + mb), (long long)c->m_cap);
    if (dtype != GWAS_DT_F64 && dtype != GWAS_DT_F32 && dtype != GWAS_DT_U8)
        return fail(GWAS_EINVAL, "unknown dtype %d", dtype);
    if (mb == 0) return GWAS_OK;
    if (!X) return fail(GWAS_EINVAL, "X_R is NULL");
    HIP_TRY(hipSetDevice(c->dev));
    hipStream_t s = (hipStream_t)stream;
    const size_t esz = dtype == GWAS_DT_F64 ? 8 : (dtype == GWAS_DT_F32 ? 4 : 1);
    RotOut ro{c->xr64, c->xr32, c->xrbf, c->xrbf3, c->m_rows, 0, c->n_pad};
    const ZSlices zs = c->zs();
    std::pair<hipEvent_t, hipEvent_t> ev{};
    if (on_device) {
        ro.row0 = m0;
        HIP_TRY(timed_begin(c, s, ev));
        HIP_TRY(launch_rotate(X, dtype, mb, c->n, c->n, c->Z, c->n_pad, ro, s, &zs));
        HIP_TRY(timed_end(c, s, ev, c->t_rot));
    } else {
        const int64_t per = std::max<int64_t>(1, (int64_t)(c->stage_bytes / (esz * c->n)));
        for (int64_t done = 0; done < mb; done += per) {
            const int64_t cnt = std::min(per, mb - done);
            const size_t bytes = (size_t)cnt * c->n * esz;
            HIP_TRY(hipMemcpyAsync(c->stage, (const uint8_t *)X + (size_t)done * c->n * esz, bytes,
                                   hipMemcpyHostToDevice, s));
            ro.row0 = m0 + done;
            HIP_TRY(timed_begin(c, s, ev));
            HIP_TRY(launch_rotate(c->stage, dtype, cnt, c->n, c->n, c->Z, c->n_pad, ro, s, &zs));
            HIP_TRY(timed_end(c, s, ev, c->t_rot));
            c->bytes_h2d += (int64_t)bytes;
        }
    }
    c->snps_rotated += mb;
    return GWAS_OK;
}

}  // extern "C"

namespace {

gwas_status check_solve(gwas_ctx *c, int64_t i0, int64_t mi, int32_t tb, const double *Y, int32_t y_on_device,
                        const double *h2, int32_t form) {
    if (!c) return fail(GWAS_EINVAL, "ctx is NULL");
    if (form < 0 || form > 3) return fail(GWAS_EINVAL, "unknown form %d", form);
    if (!(c->forms & GWAS_FORM_BIT(form))) return fail(GWAS_EINVAL, "form %d is not resident", form);
    if (i0 < 0 || mi < 0 || i0 + mi > c->m_cap)
        return fail(GWAS_EINVAL, "SNP range [%lld, %lld) outside capacity %lld", (long long)i0,
                    (long long)(i0 + mi), (long long)c->m_cap);
    if (tb < 1) return fail(GWAS_EINVAL, "tb = %d must be >= 1", tb);
    if (!Y || !h2) return fail(GWAS_EINVAL, "NULL pointer");
    for (int j = 0; j < tb; ++j) {
        const double h = h2[j];
        const bool in_range = (h >= 0.0 && h < 1.0) || (h == 1.0 && c->w_min > 0.0);
        if (!isfinite(h) || !in_range || !(h * c->w_min + (1.0 - h) > 0.0))
            return fail(GWAS_EINVAL, "h2[%d] = %g gives a covariance that is not SPD", j, h);
    }
    if (!y_on_device && !all_finite(Y, (size_t)tb * c->n)) return fail(GWAS_EINVAL, "non-finite value in Y");
    return GWAS_OK;
}

// Device memory of a trait sub-block: staged traits, rotated traits, h2, the
// form's panels (plane stride tcap rows, a multiple of 16), factors, persistent
// tile counters.
struct TraitScratch {
    double *y_in, *yt, *h2, *fac;
    void *panels;
    unsigned *tile_counters;
    int tcap;
};

TraitScratch ctx_scratch(gwas_ctx *c, int32_t form) {
    return TraitScratch{c->y_in, c->yt, c->h2, c->fac, c->panels[form], (unsigned *)(c->counters + 4),
                        panel_rows(c->tcap)};
}

// Trait sub-block [j0, j0 + jb): stage, rotate y' = Z^T y (FP64), and run the
// per-trait prologue into the scratch's panels and factors.
gwas_status prep_traits(gwas_ctx *c, const TraitScratch &ts, int j0, int jb, const double *Y, int32_t y_on_device,
                        const double *h2, int32_t form, hipStream_t s) {
    const double *ysrc = Y + (size_t)j0 * c->n;
    if (!y_on_device) {
        HIP_TRY(hipMemcpyAsync(ts.y_in, ysrc, sizeof(double) * (size_t)jb * c->n, hipMemcpyHostToDevice, s));
        c->bytes_h2d += (int64_t)sizeof(double) * jb * c->n;
        ysrc = ts.y_in;
    }
    HIP_TRY(hipMemcpyAsync(ts.h2, h2 + j0, sizeof(double) * jb, hipMemcpyHostToDevice, s));
    RotOut ro{ts.yt, nullptr, nullptr, nullptr, 0, 0, c->n_pad};
    HIP_TRY(launch_rotate(ysrc, GWAS_DT_F64, jb, c->n, c->n, c->Z, c->n_pad, ro, s));
    PrepArgs pa{ts.yt, ts.h2, c->w, c->xlt, ts.panels, ts.fac, jb, c->n, c->n_pad, c->p, ts.tcap,
                fac_stride(c->p), form};
    HIP_TRY(launch_prep(pa, s));
    return GWAS_OK;
}

gwas_status prep_traits(gwas_ctx *c, int j0, int jb, const double *Y, int32_t y_on_device, const double *h2,
                        int32_t form, hipStream_t s) {
    return prep_traits(c, ctx_scratch(c, form), j0, jb, Y, y_on_device, h2, form, s);
}

FusedArgs fused_args(gwas_ctx *c, const TraitScratch &ts, int jb, int32_t form, int tb_call) {
    FusedArgs fa{};
    fa.a = form == GWAS_FORM_F64 ? (const void *)c->xr64
         : form == GWAS_FORM_F32 ? (const void *)c->xr32
         : form == GWAS_FORM_BF16X3 ? (const void *)c->xrbf : (const void *)c->xrbf3;
    fa.a_plane_rows = c->m_rows;
    fa.panels = ts.panels;
    fa.tcap = ts.tcap;
    fa.fac = ts.fac;
    fa.fac_stride = fac_stride(c->p);
    fa.tb = jb;
    fa.n_pad = c->n_pad;
    fa.n = c->n;
    fa.p = c->p;
    fa.rank_rtol = kRankRtol[form];
    fa.non_spd = c->counters;
    fa.tile_counters = ts.tile_counters;
    fa.f32_flush = form == GWAS_FORM_F32 ? c->f32_flush : 0;
    fa.small_t = use_dot_kernel(form, c->p, tb_call, c->n_pad);
    return fa;
}

FusedArgs fused_args(gwas_ctx *c, int jb, int32_t form, int tb_call) {
    return fused_args(c, ctx_scratch(c, form), jb, form, tb_call);
}

gwas_status launch_fused_timed(gwas_ctx *c, int32_t form, const FusedArgs &fa, hipStream_t s) {
    std::pair<hipEvent_t, hipEvent_t> ev{};
    HIP_TRY(timed_begin(c, s, ev));
    HIP_TRY(launch_fused(form, fa, s));
    if (fa.small_t) ++c->dot_launches;
    HIP_TRY(timed_end(c, s, ev, c->t_fused));
    return GWAS_OK;
}

gwas_status ensure_bstage(gwas_ctx *c) {
    if (c->bstage[0]) return GWAS_OK;
    for (int u = 0; u < 2; ++u) {
        hipError_t e = hipMalloc(&c->bstage[u], c->bstage_bytes);
        if (e != hipSuccess)
            return fail(GWAS_ENOMEM, "b staging (%zu bytes): %s", c->bstage_bytes, hipGetErrorString(e));
        c->resident += (int64_t)c->bstage_bytes;
    }
    return GWAS_OK;
}

}  // namespace

extern "C" {

uint64_t gwas_checksum(const void *p, int64_t bytes) {
    if (!p || bytes <= 0) return 0;
    return checksum_range((const uint32_t *)p, 0, bytes / 4);
}

gwas_status gwas_solve(gwas_ctx *c, int64_t i0, int64_t mi, int32_t tb, const double *Y,
                       int32_t y_on_device, const double *h2, int32_t form, void *b,
                       int32_t b_on_device, void *stream) {
    last_error().clear();
    gwas_status st = check_solve(c, i0, mi, tb, Y, y_on_device, h2, form);
    if (st != GWAS_OK) return st;
    if (mi > 0 && !b) return fail(GWAS_EINVAL, "b is NULL");
    if (mi == 0) return GWAS_OK;
    HIP_TRY(hipSetDevice(c->dev));
    hipStream_t s = (hipStream_t)stream;
    const int p = c->p;
    const size_t besz = form == GWAS_FORM_F64 ? 8 : 4;

    for (int j0 = 0; j0 < tb; j0 += c->tcap) {
        const int jb = std::min(c->tcap, tb - j0);
        if ((st = prep_traits(c, j0, jb, Y, y_on_device, h2, form, s)) != GWAS_OK) return st;
        FusedArgs fa = fused_args(c, jb, form, tb);
        if (b_on_device) {
            fa.i0 = i0;
            fa.mi = mi;
            fa.b = (uint8_t *)b + (size_t)j0 * p * besz;
            fa.ldt = tb;
            if ((st = launch_fused_timed(c, form, fa, s)) != GWAS_OK) return st;
        } else {
            // slabs of SNPs into two device buffers; copies out on the side stream
            if ((st = ensure_bstage(c)) != GWAS_OK) return st;
            int slot = 0;
            for (int64_t s0 = 0; s0 < mi; s0 += c->slab, slot ^= 1) {
                const int64_t cnt = std::min<int64_t>(c->slab, mi - s0);
                HIP_TRY(hipStreamWaitEvent(s, c->ev_free[slot], 0));
                fa.i0 = i0 + s0;
                fa.mi = cnt;
                fa.b = c->bstage[slot];
                fa.ldt = jb;
                if ((st = launch_fused_timed(c, form, fa, s)) != GWAS_OK) return st;
                HIP_TRY(hipEventRecord(c->ev_done[slot], s));
                HIP_TRY(hipStreamWaitEvent(c->side, c->ev_done[slot], 0));
                const size_t row = (size_t)jb * p * besz;
                HIP_TRY(hipMemcpy2DAsync((uint8_t *)b + ((size_t)s0 * tb + j0) * p * besz,
                                         (size_t)tb * p * besz, c->bstage[slot], row, row, (size_t)cnt,
                                         hipMemcpyDeviceToHost, c->side));
                HIP_TRY(hipEventRecord(c->ev_free[slot], c->side));
                c->bytes_d2h += (int64_t)(row * cnt);
            }
            HIP_TRY(hipEventRecord(c->ev_side, c->side));
            HIP_TRY(hipStreamWaitEvent(s, c->ev_side, 0));
        }
    }
    c->problems += mi * (int64_t)tb;
    return GWAS_OK;
}

gwas_status gwas_solve_noalloc(gwas_ctx *c, int64_t i0, int64_t mi, int32_t tb, const double *Y,
                               int32_t y_on_device, const double *h2, int32_t form, void *b, void *stream) {
    last_error().clear();
    gwas_status st = check_solve(c, i0, mi, tb, Y, y_on_device, h2, form);
    if (st != GWAS_OK) return st;
    if (mi > 0 && !b) return fail(GWAS_EINVAL, "b is NULL");
    if (mi == 0) return GWAS_OK;
    HIP_TRY(hipSetDevice(c->dev));
    {
        hipPointerAttribute_t at{};
        hipError_t e = hipPointerGetAttributes(&at, b);
        if (e != hipSuccess || at.type != hipMemoryTypeDevice) {
            (void)hipGetLastError();   // a host pointer leaves an error code behind
            return fail(GWAS_EINVAL, "b must be device memory");
        }
    }
    void *base = nullptr;
    if ((st = noalloc_scratch(c->dev, &base)) != GWAS_OK) return st;
    // the largest trait sub-block whose regions (each rounded to 256 bytes) fit the array
    const int p = c->p, np = c->n_pad;
    auto r256 = [](size_t v) { return (size_t)round_up((int64_t)v, 256); };
    auto need = [&](int jb) {
        return r256(8 * sizeof(unsigned)) + (y_on_device ? 0 : r256(sizeof(double) * (size_t)jb * c->n)) +
               r256(sizeof(double) * (size_t)jb * np) + r256(sizeof(double) * jb) +
               r256(sizeof(double) * (size_t)jb * fac_stride(p)) +
               r256(elt_size(form) * (size_t)panel_planes(form) * (p + 1) * panel_rows(jb) * np);
    };
    if (need(1) > kNoAllocScratchBytes)
        return fail(GWAS_EINVAL, "one trait needs %zu scratch bytes at n = %d, p = %d, above the %zu of the array",
                    need(1), c->n, p, kNoAllocScratchBytes);
    int jmax = std::min(tb, c->tcap);
    while (need(jmax) > kNoAllocScratchBytes) jmax = std::max(1, (int)((int64_t)jmax * kNoAllocScratchBytes / need(jmax)) - 1);
    uint8_t *q = (uint8_t *)base;
    auto take = [&](size_t bytes) {
        uint8_t *r = q;
        q += r256(bytes);
        return (void *)r;
    };
    TraitScratch ts{};
    ts.tcap = panel_rows(jmax);
    ts.tile_counters = (unsigned *)take(8 * sizeof(unsigned));
    ts.y_in = y_on_device ? nullptr : (double *)take(sizeof(double) * (size_t)jmax * c->n);
    ts.yt = (double *)take(sizeof(double) * (size_t)jmax * np);
    ts.h2 = (double *)take(sizeof(double) * jmax);
    ts.fac = (double *)take(sizeof(double) * (size_t)jmax * fac_stride(p));
    ts.panels = take(elt_size(form) * (size_t)panel_planes(form) * (p + 1) * ts.tcap * np);
    hipStream_t s = (hipStream_t)stream;
    const size_t besz = form == GWAS_FORM_F64 ? 8 : 4;
    for (int j0 = 0; j0 < tb; j0 += jmax) {
        const int jb = std::min(jmax, tb - j0);
        if ((st = prep_traits(c, ts, j0, jb, Y, y_on_device, h2, form, s)) != GWAS_OK) return st;
        FusedArgs fa = fused_args(c, ts, jb, form, tb);
        fa.i0 = i0;
        fa.mi = mi;
        fa.b = (uint8_t *)b + (size_t)j0 * p * besz;
        fa.ldt = tb;
        HIP_TRY(launch_fused(form, fa, s));
        if (fa.small_t) ++c->dot_launches;
    }
    c->problems += mi * (int64_t)tb;
    return GWAS_OK;
}

namespace {

// The streamed sink: a pinned host ring (library-owned, allocated on first
// use) and the slabs in flight, consumed in issue order on the calling thread.
struct RingSink {
    gwas_ctx *c;
    int form;
    gwas_slab_fn fn;
    void *user;
    uint64_t *checksums;
    int64_t max_checksums;
    struct Pending {
        gwas_slab slab;
        int slot;
    };
    std::vector<Pending> inflight;   // issued, not yet consumed, in issue order
    int64_t issued = 0, consumed = 0;
    int dslot = 0;                   // device staging buffer of the next slab

    gwas_status init() {
        gwas_status st = ensure_bstage(c);
        if (st != GWAS_OK) return st;
        if (!c->ring.empty()) return GWAS_OK;
        const int R = c->ring_slots;
        c->ring_bytes = c->bstage_bytes;
        c->ring.assign(R, nullptr);
        c->ring_ev.assign(R, nullptr);
        for (int r = 0; r < R; ++r) {
            hipError_t e = hipHostMalloc(&c->ring[r], c->ring_bytes, hipHostMallocDefault);
            if (e != hipSuccess)
                return fail(GWAS_ENOMEM, "pinned ring slot (%zu bytes): %s", c->ring_bytes, hipGetErrorString(e));
            HIP_TRY(hipEventCreateWithFlags(&c->ring_ev[r], hipEventDisableTiming));
            void *pd = nullptr;
            HIP_TRY(hipHostGetDevicePointer(&pd, c->ring[r], 0));
            c->ring_dev.push_back(pd);
        }
        return GWAS_OK;
    }

    gwas_status consume_one() {
        Pending pd = inflight.front();
        inflight.erase(inflight.begin());
        HIP_TRY(hipEventSynchronize(c->ring_ev[pd.slot]));
        pd.slab.b = c->ring[pd.slot];
        pd.slab.checksum = checksum_parallel(pd.slab.b, pd.slab.bytes, c->host_threads);
        if (checksums && consumed < max_checksums) checksums[consumed] = pd.slab.checksum;
        if (fn) fn(user, &pd.slab);
        ++consumed;
        return GWAS_OK;
    }

    gwas_status drain() {
        while (!inflight.empty()) {
            gwas_status st = consume_one();
            if (st != GWAS_OK) return st;
        }
        return GWAS_OK;
    }

    // Solve store rows [row0, row0 + count) (SNPs global0 ...) against the trait
    // sub-block [j0, j0 + fa.tb) prepared in the context, slab by slab into the ring.
    gwas_status solve_rows(FusedArgs fa, int64_t row0, int64_t global0, int64_t count, int j0, hipStream_t s) {
        const int R = c->ring_slots;
        const int p = c->p;
        const size_t besz = form == GWAS_FORM_F64 ? 8 : 4;
        const int jb = fa.tb;
        for (int64_t s0 = 0; s0 < count; s0 += c->slab, dslot ^= 1) {
            const int64_t cnt = std::min<int64_t>(c->slab, count - s0);
            const int rslot = (int)(issued % R);
            if ((int64_t)inflight.size() >= R) {   // the ring slot is still held: consume the oldest slab
                gwas_status st = consume_one();
                if (st != GWAS_OK) return st;
            }
            HIP_TRY(hipStreamWaitEvent(s, c->ev_free[dslot], 0));
            fa.i0 = row0 + s0;
            fa.mi = cnt;
            fa.b = c->bstage[dslot];
            fa.ldt = jb;
            gwas_status st = launch_fused_timed(c, form, fa, s);
            if (st != GWAS_OK) return st;
            HIP_TRY(hipEventRecord(c->ev_done[dslot], s));
            HIP_TRY(hipStreamWaitEvent(c->side, c->ev_done[dslot], 0));
            const size_t bytes = (size_t)cnt * jb * p * besz;
            // the library's copy kernel moves the slab into the pinned slot (its rate does
            // not depend on which engine the runtime would pick for a copy)
            HIP_TRY(launch_copy_to_host(c->ring_dev[rslot], c->bstage[dslot], (int64_t)bytes, 64, c->side));
            HIP_TRY(hipEventRecord(c->ring_ev[rslot], c->side));
            HIP_TRY(hipEventRecord(c->ev_free[dslot], c->side));
            c->bytes_d2h += (int64_t)bytes;
            Pending pd{};
            pd.slab.index = issued;
            pd.slab.i0 = global0 + s0;
            pd.slab.count = cnt;
            pd.slab.j0 = j0;
            pd.slab.tb = jb;
            pd.slab.p = p;
            pd.slab.form = form;
            pd.slab.bytes = (int64_t)bytes;
            pd.slot = rslot;
            inflight.push_back(pd);
            ++issued;
        }
        return GWAS_OK;
    }

    // the caller's stream waits for the sink's last copy
    gwas_status join(hipStream_t s) {
        HIP_TRY(hipEventRecord(c->ev_side, c->side));
        HIP_TRY(hipStreamWaitEvent(s, c->ev_side, 0));
        return GWAS_OK;
    }
};

}  // namespace

gwas_status gwas_solve_stream(gwas_ctx *c, int64_t i0, int64_t mi, int32_t tb, const double *Y,
                              int32_t y_on_device, const double *h2, int32_t form, gwas_slab_fn fn,
                              void *user, uint64_t *checksums, int64_t max_checksums, int64_t *n_slabs,
                              void *stream) {
    last_error().clear();
    gwas_status st = check_solve(c, i0, mi, tb, Y, y_on_device, h2, form);
    if (st != GWAS_OK) return st;
    if (n_slabs) *n_slabs = 0;
    if (mi == 0) return GWAS_OK;
    HIP_TRY(hipSetDevice(c->dev));
    hipStream_t s = (hipStream_t)stream;
    RingSink sink{c, form, fn, user, checksums, max_checksums};
    if ((st = sink.init()) != GWAS_OK) return st;
    for (int j0 = 0; j0 < tb; j0 += c->tcap) {
        const int jb = std::min(c->tcap, tb - j0);
        if ((st = prep_traits(c, j0, jb, Y, y_on_device, h2, form, s)) != GWAS_OK) return st;
        if ((st = sink.solve_rows(fused_args(c, jb, form, tb), i0, i0, mi, j0, s)) != GWAS_OK) return st;
    }
    if ((st = sink.drain()) != GWAS_OK) return st;
    if ((st = sink.join(s)) != GWAS_OK) return st;
    if (n_slabs) *n_slabs = sink.issued;
    c->problems += mi * (int64_t)tb;
    return GWAS_OK;
}

gwas_status gwas_solve_snp_stream(gwas_ctx *c, const void *X_R, int32_t dtype, int64_t m, int32_t tb,
                                  const double *Y, int32_t y_on_device, const double *h2, int32_t form,
                                  gwas_slab_fn fn, void *user, uint64_t *checksums, int64_t max_checksums,
                                  int64_t *n_slabs, void *stream) {
    last_error().clear();
    if (!c) return fail(GWAS_EINVAL, "ctx is NULL");
    if (m < 0) return fail(GWAS_EINVAL, "m = %lld is negative", (long long)m);
    if (dtype != GWAS_DT_F64 && dtype != GWAS_DT_F32 && dtype != GWAS_DT_U8)
        return fail(GWAS_EINVAL, "unknown dtype %d", dtype);
    if (c->m_cap < 2) return fail(GWAS_EINVAL, "m_capacity must be at least 2 (the store holds two blocks)");
    gwas_status st = check_solve(c, 0, 0, tb, Y, y_on_device, h2, form);
    if (st != GWAS_OK) return st;
    if (n_slabs) *n_slabs = 0;
    if (m == 0) return GWAS_OK;
    if (!X_R) return fail(GWAS_EINVAL, "X_R is NULL");
    HIP_TRY(hipSetDevice(c->dev));
    hipStream_t s = (hipStream_t)stream;
    const size_t esz = dtype == GWAS_DT_F64 ? 8 : (dtype == GWAS_DT_F32 ? 4 : 1);
    const int64_t B = c->m_cap / 2;   // SNPs per block; block k uses store half k % 2
    // device staging of the raw SNP blocks (two, so the next block's copy can start
    // while this one rotates), the stream that copies and rotates, and its events
    const size_t in_bytes = (size_t)B * c->n * esz;
    if (c->xin_bytes < in_bytes) {
        for (int h = 0; h < 2; ++h) {
            if (c->xin[h]) HIP_TRY(hipFree(c->xin[h]));
            c->xin[h] = nullptr;
        }
        c->xin_bytes = 0;
        for (int h = 0; h < 2; ++h) {
            hipError_t e = hipMalloc(&c->xin[h], in_bytes);
            if (e != hipSuccess) return fail(GWAS_ENOMEM, "SNP block staging (%zu bytes): %s", in_bytes,
                                             hipGetErrorString(e));
        }
        c->xin_bytes = in_bytes;
    }
    if (!c->aux) {
        HIP_TRY(hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking));
        for (int h = 0; h < 2; ++h) {
            HIP_TRY(hipEventCreateWithFlags(&c->ev_rot[h], hipEventDisableTiming));
            HIP_TRY(hipEventCreateWithFlags(&c->ev_half[h], hipEventDisableTiming));
        }
    }
    RingSink sink{c, form, fn, user, checksums, max_checksums};
    if ((st = sink.init()) != GWAS_OK) return st;
    // the store halves start free once the caller's stream has reached this call
    for (int h = 0; h < 2; ++h) HIP_TRY(hipEventRecord(c->ev_half[h], s));
    const bool one_trait_block = tb <= c->tcap;
    if (one_trait_block && (st = prep_traits(c, 0, tb, Y, y_on_device, h2, form, s)) != GWAS_OK) return st;
    const int64_t nblk = (m + B - 1) / B;
    std::pair<hipEvent_t, hipEvent_t> ev{};
    // copy + rotate block k into store half k % 2 once the block before it in
    // that half is solved (enqueued two blocks ahead, so it runs while the
    // previous block is solved and its b leaves)
    auto load_block = [&](int64_t k) -> gwas_status {
        const int h = (int)(k % 2);
        const int64_t g0 = k * B, cnt = std::min(B, m - g0);
        HIP_TRY(hipStreamWaitEvent(c->aux, c->ev_half[h], 0));
        HIP_TRY(hipMemcpyAsync(c->xin[h], (const uint8_t *)X_R + (size_t)g0 * c->n * esz,
                               (size_t)cnt * c->n * esz, hipMemcpyDefault, c->aux));
        c->bytes_h2d += (int64_t)cnt * c->n * (int64_t)esz;
        RotOut ro{c->xr64, c->xr32, c->xrbf, c->xrbf3, c->m_rows, (int64_t)h * B, c->n_pad};
        HIP_TRY(timed_begin(c, c->aux, ev));
        const ZSlices zs = c->zs();
        HIP_TRY(launch_rotate(c->xin[h], dtype, cnt, c->n, c->n, c->Z, c->n_pad, ro, c->aux, &zs));
        HIP_TRY(timed_end(c, c->aux, ev, c->t_rot));
        HIP_TRY(hipEventRecord(c->ev_rot[h], c->aux));
        c->snps_rotated += cnt;
        return GWAS_OK;
    };
    for (int64_t k = 0; k < std::min<int64_t>(2, nblk); ++k)
        if ((st = load_block(k)) != GWAS_OK) return st;
    for (int64_t k = 0; k < nblk; ++k) {
        const int h = (int)(k % 2);
        const int64_t g0 = k * B, cnt = std::min(B, m - g0);
        // solve block k from half h on the caller's stream
        HIP_TRY(hipStreamWaitEvent(s, c->ev_rot[h], 0));
        for (int j0 = 0; j0 < tb; j0 += c->tcap) {
            const int jb = std::min(c->tcap, tb - j0);
            if (!one_trait_block && (st = prep_traits(c, j0, jb, Y, y_on_device, h2, form, s)) != GWAS_OK)
                return st;
            if ((st = sink.solve_rows(fused_args(c, jb, form, tb), (int64_t)h * B, g0, cnt, j0, s)) != GWAS_OK)
                return st;
        }
        HIP_TRY(hipEventRecord(c->ev_half[h], s));
        if (k + 2 < nblk && (st = load_block(k + 2)) != GWAS_OK) return st;
    }
    if ((st = sink.drain()) != GWAS_OK) return st;
    if ((st = sink.join(s)) != GWAS_OK) return st;
    if (n_slabs) *n_slabs = sink.issued;
    c->problems += m * (int64_t)tb;
    return GWAS_OK;
}

gwas_status gwas_copy_rotated(gwas_ctx *c, int64_t i0, int64_t mi, int32_t form, void *dst,
                              int32_t dst_on_device, void *stream) {
    last_error().clear();
    if (!c) return fail(GWAS_EINVAL, "ctx is NULL");
    if (form != GWAS_FORM_F64 && form != GWAS_FORM_F32)
        return fail(GWAS_EINVAL, "copy_rotated supports the FP64 and FP32 stores only");
    if (!(c->forms & GWAS_FORM_BIT(form))) return fail(GWAS_EINVAL, "form %d is not resident", form);
    if (i0 < 0 || mi < 0 || i0 + mi > c->m_cap) return fail(GWAS_EINVAL, "SNP range outside capacity");
    if (mi == 0) return GWAS_OK;
    if (!dst) return fail(GWAS_EINVAL, "dst is NULL");
    HIP_TRY(hipSetDevice(c->dev));
    hipStream_t s = (hipStream_t)stream;
    const size_t esz = form == GWAS_FORM_F64 ? 8 : 4;
    const uint8_t *src = (const uint8_t *)(form == GWAS_FORM_F64 ? (void *)c->xr64 : (void *)c->xr32) +
                         (size_t)i0 * c->n_pad * esz;
    HIP_TRY(hipMemcpy2DAsync(dst, c->n * esz, src, c->n_pad * esz, c->n * esz, (size_t)mi,
                             dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    if (!dst_on_device) HIP_TRY(hipStreamSynchronize(s));
    return GWAS_OK;
}

gwas_status gwas_stats(gwas_ctx *c, gwas_stats_t *out) {
    last_error().clear();
    if (!c || !out) return fail(GWAS_EINVAL, "NULL pointer");
    HIP_TRY(hipSetDevice(c->dev));
    HIP_TRY(hipDeviceSynchronize());
    unsigned long long cnt[4];
    HIP_TRY(hipMemcpy(cnt, c->counters, sizeof cnt, hipMemcpyDeviceToHost));
    memset(out, 0, sizeof *out);
    out->non_spd = (int64_t)cnt[0];
    out->snps_rotated = c->snps_rotated;
    out->problems = c->problems;
    out->dot_launches = c->dot_launches;
    out->bytes_h2d = c->bytes_h2d;
    out->bytes_d2h = c->bytes_d2h;
    out->resident_bytes = c->resident;
    // timing record: kept until reset, so repeated queries see the same totals
    double fms = 0.0, rms = 0.0;
    for (auto &ev : c->t_fused) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev.first, ev.second) == hipSuccess) fms += ms;
    }
    for (auto &ev : c->t_rot) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev.first, ev.second) == hipSuccess) rms += ms;
    }
    out->fused_launches = (int64_t)c->t_fused.size();
    out->fused_ms = fms;
    out->rotate_launches = (int64_t)c->t_rot.size();
    out->rotate_ms = rms;
    return GWAS_OK;
}

gwas_status gwas_reset_stats(gwas_ctx *c) {
    last_error().clear();
    if (!c) return fail(GWAS_EINVAL, "NULL pointer");
    HIP_TRY(hipSetDevice(c->dev));
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemset(c->counters, 0, sizeof(unsigned long long) * 4));
    int64_t cnt;
    drain(c, c->t_fused, cnt);
    drain(c, c->t_rot, cnt);
    c->snps_rotated = c->problems = c->bytes_h2d = c->bytes_d2h = c->dot_launches = 0;
    return GWAS_OK;
}

int64_t gwas_debug_size(gwas_ctx *c, int32_t what, int32_t form) {
    if (!c) return -1;
    const int64_t np = c->n_pad;
    switch (what) {
    case GWAS_DBG_XL: return (int64_t)sizeof(double) * (c->p - 1) * np;
    case GWAS_DBG_YT: return (int64_t)sizeof(double) * c->tcap * np;
    case GWAS_DBG_FAC: return (int64_t)sizeof(double) * c->tcap * fac_stride(c->p);
    case GWAS_DBG_PANELS:
        if (form < 0 || form > 3 || !(c->forms & GWAS_FORM_BIT(form))) return -1;
        return (int64_t)elt_size(form) * panel_planes(form) * (c->p + 1) * panel_rows(c->tcap) * np;
    default: return -1;
    }
}

gwas_status gwas_debug_copy(gwas_ctx *c, int32_t what, int32_t form, void *dst, int64_t bytes) {
    last_error().clear();
    const int64_t need = gwas_debug_size(c, what, form);
    if (need < 0 || !dst || bytes != need) return fail(GWAS_EINVAL, "bad debug request");
    const void *src = what == GWAS_DBG_XL ? (const void *)c->xlt
                    : what == GWAS_DBG_YT ? (const void *)c->yt
                    : what == GWAS_DBG_FAC ? (const void *)c->fac : c->panels[form];
    HIP_TRY(hipSetDevice(c->dev));
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(dst, src, (size_t)bytes, hipMemcpyDeviceToHost));
    return GWAS_OK;
}

void gwas_destroy(gwas_ctx *c) { release(c); }

}  // extern "C"

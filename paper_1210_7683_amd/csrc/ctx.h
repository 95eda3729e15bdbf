// Host-side state of a libgwas context, shared by the C-ABI translation units.
#pragma once

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <thread>
#include <utility>
#include <vector>

#include "gwas_internal.h"

namespace gw {

// Thread-local message of the last failure (gwas_last_error).
std::string &last_error();

inline gwas_status fail(gwas_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    last_error() = buf;
    return st;
}

#define HIP_TRY(expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return ::gw::fail(e_ == hipErrorOutOfMemory ? GWAS_ENOMEM : GWAS_EHIP, "%s: %s (%d)", \
                              #expr, hipGetErrorString(e_), (int)e_);                        \
    } while (0)

inline int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// Position-weighted checksum of 32-bit words (gwas_checksum), over [k0, k1).
inline uint64_t checksum_range(const uint32_t *w, int64_t k0, int64_t k1) {
    uint64_t s0 = 0, s1 = 0, s2 = 0, s3 = 0;   // four independent chains
    int64_t k = k0;
    for (; k + 3 < k1; k += 4) {
        s0 += (uint64_t)(k + 1) * (uint64_t)w[k];
        s1 += (uint64_t)(k + 2) * (uint64_t)w[k + 1];
        s2 += (uint64_t)(k + 3) * (uint64_t)w[k + 2];
        s3 += (uint64_t)(k + 4) * (uint64_t)w[k + 3];
    }
    for (; k < k1; ++k) s0 += (uint64_t)(k + 1) * (uint64_t)w[k];
    return s0 + s1 + s2 + s3;
}

inline uint64_t checksum_parallel(const void *p, int64_t bytes, int threads) {
    const uint32_t *w = (const uint32_t *)p;
    const int64_t words = bytes / 4;
    if (threads <= 1 || words < (1 << 20)) return checksum_range(w, 0, words);
    std::vector<uint64_t> part(threads, 0);
    std::vector<std::thread> pool;
    const int64_t per = (words + threads - 1) / threads;
    for (int t = 0; t < threads; ++t)
        pool.emplace_back([&, t] {
            const int64_t k0 = std::min(words, t * per), k1 = std::min(words, k0 + per);
            part[t] = checksum_range(w, k0, k1);
        });
    uint64_t s = 0;
    for (int t = 0; t < threads; ++t) {
        pool[t].join();
        s += part[t];
    }
    return s;
}

}  // namespace gw

struct gwas_ctx {
    int dev = 0;
    int n = 0, n_pad = 0, p = 0;
    int64_t m_cap = 0;       // SNPs the store holds
    int64_t m_rows = 0;      // rows allocated per plane (>= m_cap)
    uint32_t forms = 0;
    int tcap = 0;            // traits per internal sub-block
    int slab = 0;            // SNPs per D2H slab
    int f32_flush = 0;
    double w_min = 0.0;

    double *Z = nullptr;     // [n_pad][n_pad]: row k = eigenvector k (zeros beyond n)
    int8_t *zq = nullptr;    // int8 digits of Z for the genotype rotation (ZSlices)
    double *zoff = nullptr, *zscale = nullptr;   // [2][n_pad] and [n_pad]
    uint8_t *zpack = nullptr;   // genotype repack chunk: zpack_rows x n_pad bytes
    int64_t zpack_rows = 0;
    double *w = nullptr;     // [n_pad]
    double *xlt = nullptr;   // [p-1][n_pad]
    double *xr64 = nullptr;  // [m_rows][n_pad]
    float *xr32 = nullptr;   // [m_rows][n_pad]
    uint16_t *xrbf = nullptr;  // 2 planes (x' hi, lo) [m_rows][n_pad]
    uint16_t *xrbf3 = nullptr; // 3 planes (x' hi, mid, lo) [m_rows][n_pad]

    double *y_in = nullptr;  // [tcap][n] staging of host traits
    double *yt = nullptr;    // [tcap][n_pad]
    double *h2 = nullptr;    // [tcap]
    void *panels[4] = {nullptr, nullptr, nullptr, nullptr};  // per form
    double *fac = nullptr;   // [tcap][fac_stride]
    unsigned long long *counters = nullptr;  // [0] non-SPD problems; [4..7] persistent tile counters

    void *stage = nullptr;   // rotation staging for host SNP blocks
    size_t stage_bytes = 0;
    void *bstage[2] = {nullptr, nullptr};
    size_t bstage_bytes = 0;
    hipStream_t side = nullptr;
    hipEvent_t ev_done[2] = {nullptr, nullptr};   // slab computed
    hipEvent_t ev_free[2] = {nullptr, nullptr};   // slab copied out
    hipEvent_t ev_side = nullptr;

    // genotype stream (gwas_solve_snp_stream): raw SNP block staging, the stream
    // that copies and rotates blocks, block rotated / store half free events
    void *xin[2] = {nullptr, nullptr};
    size_t xin_bytes = 0;
    hipStream_t aux = nullptr;
    hipEvent_t ev_rot[2] = {nullptr, nullptr};
    hipEvent_t ev_half[2] = {nullptr, nullptr};

    // streamed sink: pinned host ring
    int ring_slots = 4, host_threads = 8;
    std::vector<void *> ring;
    std::vector<void *> ring_dev;   // device-side addresses of the ring slots
    size_t ring_bytes = 0;
    std::vector<hipEvent_t> ring_ev;

    gw::ZSlices zs() const { return gw::ZSlices{zq, zoff, zscale, zpack, zpack_rows}; }

    int64_t snps_rotated = 0, problems = 0, bytes_h2d = 0, bytes_d2h = 0, resident = 0, dot_launches = 0;

    // optional per-launch timing: event pairs recorded around launches
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> t_fused, t_rot, t_pool;
};


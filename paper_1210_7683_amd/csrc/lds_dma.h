// Direct global->LDS staging shared by the fused and rotation kernels.
//
// A wave-wide global_load_lds_dwordx4 moves 16 bytes per lane from a per-lane
// global address to LDS at (wave-uniform base + 16 * lane). The kernels lay
// their LDS out as 1 KB blocks that each hold one MFMA operand fragment in lane
// order, so one such load fills a block and one ds_read_b128 per lane reads a
// fragment back.
//
// The compiler places a wait for every outstanding global->LDS load before any
// LDS read it can see, since it cannot tell LDS buffers apart. Kernels that
// keep the next stage's loads in flight while reading the current stage read
// their fragments with lds_read_frags instead: blocks of ds_read_b128 written
// as inline assembly, each block waiting for its own results before it ends.
#pragma once

#include "gwas_internal.h"

namespace gw {

__device__ __forceinline__ void lds_dma16(const uint8_t *g, uint8_t *l) {
    __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1))) *)g,
                                     (void __attribute__((address_space(3))) *)l, 16, 0, 0);
}

// 4 bytes per lane: lane l's dword lands at LDS (wave-uniform base + 4 l).
__device__ __forceinline__ void lds_dma4(const uint8_t *g, uint8_t *l) {
    __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1))) *)g,
                                     (void __attribute__((address_space(3))) *)l, 4, 0, 0);
}

// s_waitcnt immediate that waits until at most n (< 64) vector memory
// operations of this wave are outstanding (lgkmcnt and expcnt not waited).
constexpr int vmcnt_imm(int n) { return 0x0F70 | (n & 15) | ((n >> 4) << 14); }

typedef int i4v __attribute__((ext_vector_type(4)));

// LDS byte address (offset within the workgroup's LDS) of a shared-memory pointer.
__device__ __forceinline__ uint32_t lds_addr(const void *p) {
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void *)p;
}

// Reads fragments [I0, I0 + N) of a stage into f, in blocks of 16/8/4/2/1
// ds_read_b128 that each wait for their own reads before they end. Fragment i
// is at LDS byte address (C::frag_is_b(i) ? bb : ba) + C::frag_off(i), with
// frag_off a compile-time constant below 64 KB.
#define GW_DSR(k) "ds_read_b128 %" #k ", %[b" #k "] offset:%c[o" #k "]\n"
#define GW_OUT(k) "=&v"(f[I0 + k])
#define GW_IN(k) [b##k] "v"(C::frag_is_b(I0 + k) ? bb : ba), [o##k] "i"(C::frag_off(I0 + k))
template <class C, int I0, int N>
__device__ __forceinline__ void lds_read_frags(i4v *f, uint32_t ba, uint32_t bb) {
    if constexpr (N >= 16) {
        asm volatile(GW_DSR(0) GW_DSR(1) GW_DSR(2) GW_DSR(3) GW_DSR(4) GW_DSR(5) GW_DSR(6) GW_DSR(7) GW_DSR(8)
                         GW_DSR(9) GW_DSR(10) GW_DSR(11) GW_DSR(12) GW_DSR(13) GW_DSR(14) GW_DSR(15)
                             "s_waitcnt lgkmcnt(0)"
                     : GW_OUT(0), GW_OUT(1), GW_OUT(2), GW_OUT(3), GW_OUT(4), GW_OUT(5), GW_OUT(6), GW_OUT(7),
                       GW_OUT(8), GW_OUT(9), GW_OUT(10), GW_OUT(11), GW_OUT(12), GW_OUT(13), GW_OUT(14), GW_OUT(15)
                     : GW_IN(0), GW_IN(1), GW_IN(2), GW_IN(3), GW_IN(4), GW_IN(5), GW_IN(6), GW_IN(7), GW_IN(8),
                       GW_IN(9), GW_IN(10), GW_IN(11), GW_IN(12), GW_IN(13), GW_IN(14), GW_IN(15)
                     : "memory");
        lds_read_frags<C, I0 + 16, N - 16>(f, ba, bb);
    } else if constexpr (N >= 8) {
        asm volatile(GW_DSR(0) GW_DSR(1) GW_DSR(2) GW_DSR(3) GW_DSR(4) GW_DSR(5) GW_DSR(6) GW_DSR(7)
                         "s_waitcnt lgkmcnt(0)"
                     : GW_OUT(0), GW_OUT(1), GW_OUT(2), GW_OUT(3), GW_OUT(4), GW_OUT(5), GW_OUT(6), GW_OUT(7)
                     : GW_IN(0), GW_IN(1), GW_IN(2), GW_IN(3), GW_IN(4), GW_IN(5), GW_IN(6), GW_IN(7)
                     : "memory");
        lds_read_frags<C, I0 + 8, N - 8>(f, ba, bb);
    } else if constexpr (N >= 4) {
        asm volatile(GW_DSR(0) GW_DSR(1) GW_DSR(2) GW_DSR(3) "s_waitcnt lgkmcnt(0)"
                     : GW_OUT(0), GW_OUT(1), GW_OUT(2), GW_OUT(3)
                     : GW_IN(0), GW_IN(1), GW_IN(2), GW_IN(3)
                     : "memory");
        lds_read_frags<C, I0 + 4, N - 4>(f, ba, bb);
    } else if constexpr (N >= 2) {
        asm volatile(GW_DSR(0) GW_DSR(1) "s_waitcnt lgkmcnt(0)"
                     : GW_OUT(0), GW_OUT(1)
                     : GW_IN(0), GW_IN(1)
                     : "memory");
        lds_read_frags<C, I0 + 2, N - 2>(f, ba, bb);
    } else if constexpr (N == 1) {
        asm volatile(GW_DSR(0) "s_waitcnt lgkmcnt(0)" : GW_OUT(0) : GW_IN(0) : "memory");
    }
}
#undef GW_DSR
#undef GW_OUT
#undef GW_IN

}  // namespace gw

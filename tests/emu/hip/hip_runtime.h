// Host stand-in for the parts of the HIP device API that the Sprintz kernels
// use, for the CPU test harness: kernels are compiled as ordinary host code
// and run lane by lane by emu_sched.h. Cross-lane builtins meet the other
// lanes of the wavefront; bit-field builtins are computed as the ISA
// defines them.
#pragma once

#include <stdint.h>
#include <string.h>

#include <algorithm>

#include "../emu_sched.h"

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __shared__ static
#define __launch_bounds__(...)
#define __restrict__ __restrict

typedef void *hipStream_t;
typedef int hipError_t;

#define threadIdx (emu::me().tid)
#define blockIdx (emu::current_block()->bid)
#define blockDim (emu::current_block()->bdim)

struct uint2 { uint32_t x, y; };
struct uint4 { uint32_t x, y, z, w; };
struct int4 { int32_t x, y, z, w; };
inline int4 make_int4(int a, int b, int c, int d) { return int4{a, b, c, d}; }
inline uint2 make_uint2(uint32_t a, uint32_t b) { return uint2{a, b}; }
inline uint4 make_uint4(uint32_t a, uint32_t b, uint32_t c, uint32_t d) { return uint4{a, b, c, d}; }

using std::max;
using std::min;
inline uint64_t min(uint64_t a, uint32_t b) { return a < b ? a : (uint64_t)b; }
inline uint64_t min(uint32_t a, uint64_t b) { return a < b ? (uint64_t)a : b; }

inline void __syncthreads() { emu::barrier(); }
inline int __mul24(int a, int b) {
    // the low 32 bits of the product of the sign-extended low 24 bits
    const int64_t x = (int64_t)((int32_t)((uint32_t)a << 8) >> 8), y = (int64_t)((int32_t)((uint32_t)b << 8) >> 8);
    return (int)(uint32_t)(uint64_t)(x * y);
}
inline int __clz(int v) { return v == 0 ? 32 : __builtin_clz((uint32_t)v); }

inline int __shfl_up(int v, unsigned d, int width = 64) {
    return (int)emu::wave_op(emu::OP_SHFL_UP, (uint32_t)v, (int)d, width);
}
inline unsigned long long __shfl_up(unsigned long long v, unsigned d, int width = 64) {
    const uint32_t lo = emu::wave_op(emu::OP_SHFL_UP, (uint32_t)v, (int)d, width);
    const uint32_t hi = emu::wave_op(emu::OP_SHFL_UP, (uint32_t)(v >> 32), (int)d, width);
    return ((unsigned long long)hi << 32) | lo;
}
inline int __shfl(int v, int src, int width = 64) { return (int)emu::wave_op(emu::OP_SHFL, (uint32_t)v, src, width); }

template <typename T> inline T atomicOr(T *p, T v) { const T o = *p; *p = o | v; return o; }
template <typename T> inline T atomicAnd(T *p, T v) { const T o = *p; *p = o & v; return o; }
template <typename T> inline T atomicAdd(T *p, T v) { const T o = *p; *p = o + v; return o; }

// bit-field and funnel-shift builtins (gfx9 semantics: offset and width
// taken modulo 32)
inline uint32_t emu_ubfe(uint32_t v, uint32_t off, uint32_t w) {
    off &= 31; w &= 31;
    if (w == 0) return 0;
    return (v >> off) & (w >= 32 ? ~0u : ((1u << w) - 1u));
}
inline int32_t emu_sbfe(int32_t v, uint32_t off, uint32_t w) {
    off &= 31; w &= 31;
    if (w == 0) return 0;
    const uint32_t u = ((uint32_t)v >> off) & ((1u << w) - 1u);
    return (int32_t)(u << (32 - w)) >> (32 - w);
}
inline uint32_t emu_alignbit(uint32_t hi, uint32_t lo, uint32_t s) {
    return (uint32_t)((((uint64_t)hi << 32) | lo) >> (s & 31));
}
inline uint32_t emu_bitreverse32(uint32_t v) {
    uint32_t r = 0;
    for (int i = 0; i < 32; ++i) r |= ((v >> i) & 1u) << (31 - i);
    return r;
}
inline int emu_update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl) {
    (void)old; (void)row_mask; (void)bank_mask; (void)bound_ctrl;   // the kernels use old 0, all rows, bound_ctrl
    return (int)emu::wave_op(emu::OP_DPP, (uint32_t)src, ctrl, 64);
}
inline uint32_t emu_readfirstlane(uint32_t v) { return emu::wave_op(emu::OP_FIRST, v, 0, 64); }
inline uint32_t emu_sad_u8(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t t = c;
    for (int k = 0; k < 4; ++k) {
        const int x = (int)((a >> (8 * k)) & 255u), y = (int)((b >> (8 * k)) & 255u);
        t += (uint32_t)(x > y ? x - y : y - x);
    }
    return t;
}
#define __builtin_amdgcn_sad_u8 emu_sad_u8
#define __builtin_amdgcn_ubfe emu_ubfe
#define __builtin_amdgcn_sbfe emu_sbfe
#define __builtin_amdgcn_alignbit emu_alignbit
#define __builtin_bitreverse32 emu_bitreverse32
#define __builtin_amdgcn_update_dpp emu_update_dpp
#define __builtin_amdgcn_readfirstlane emu_readfirstlane
#define __builtin_amdgcn_sched_barrier(x) ((void)0)
#define __builtin_amdgcn_s_sleep(x) ((void)0)

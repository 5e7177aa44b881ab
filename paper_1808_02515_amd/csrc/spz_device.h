// Device-side building blocks of the gfx950 Sprintz codec.
//
// Work decomposition: one lane per (segment, column) "chain". The D lanes of
// a segment form a lane group of Dp = next_pow2(D) <= 64 lanes inside one
// wavefront; lanes j >= D of a group carry a zero column. Groups exchange
// per-block bit widths with wave shuffles (group-local scans), so every lane
// knows its column's bit offset inside a packed row and the record size.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spz {

constexpr int kThreads = 256;       // threads per workgroup (4 wavefronts)
constexpr uint32_t kRleMax = 65535; // run counts are u16

// Launch geometry and container layout shared by the kernels.
struct Geom {
    uint64_t rows;
    uint64_t data_start;  // byte offset of segment data in the container
    uint64_t cap;         // encode: dst capacity; decode: container size
    uint64_t data_bytes;  // decode: bytes of segment data
    uint32_t D;
    uint32_t S;           // rows per segment (multiple of 8)
    uint32_t nseg;
    uint32_t dp_log2;     // log2 of the lane-group size
    uint32_t G;           // records per header group, 0 = whole segment
    uint32_t sh;          // FIRE: alpha = acc >> sh  (learn_shift + 2)
    int32_t acc_lo;       // FIRE accumulator range
    int32_t acc_hi;
};

template <int W> struct Elem;
template <> struct Elem<8> { using T = uint8_t; };
template <> struct Elem<16> { using T = uint16_t; };

// Low W bits of v as a signed W-bit value (v_bfe_i32).
template <int W> __device__ __forceinline__ int32_t sext(int32_t v) {
    return __builtin_amdgcn_sbfe(v, 0u, (uint32_t)W);
}

// Zigzag of a signed W-bit error: 2e for e >= 0, -2e-1 for e < 0.
__device__ __forceinline__ uint32_t zigzag(int32_t e) {
    return ((uint32_t)e << 1) ^ (uint32_t)(e >> 31);
}

__device__ __forceinline__ int32_t unzigzag(uint32_t z) {
    return (int32_t)(z >> 1) ^ -(int32_t)(z & 1u);
}

__device__ __forceinline__ int32_t sgn(int32_t e) { return min(max(e, -1), 1); }

// sign(e) in one v_med3_i32 (the compiler lowers the clamp above to two
// compare/select pairs).
__device__ __forceinline__ int32_t sgn_med3(int32_t e) {
    int32_t r;
    asm("v_med3_i32 %0, %1, -1, 1" : "=v"(r) : "v"(e));
    return r;
}

// Number of significant bits (0 for 0).
__device__ __forceinline__ uint32_t bitlen(uint32_t v) { return 32u - (uint32_t)__clz((int)v); }

// Inclusive sum over the lane group (Dp lanes, Dp a power of two).
__device__ __forceinline__ uint32_t group_incl_sum(uint32_t v, uint32_t Dp, uint32_t lane) {
    for (uint32_t k = 1; k < Dp; k <<= 1) {
        uint32_t t = (uint32_t)__shfl_up((int)v, k, (int)Dp);
        if (lane >= k) v += t;
    }
    return v;
}

__device__ __forceinline__ uint32_t group_last(uint32_t v, uint32_t Dp) {
    return (uint32_t)__shfl((int)v, (int)(Dp - 1), (int)Dp);
}

__device__ __forceinline__ uint64_t ld_u64_aligned(const uint8_t *p) {
    return *reinterpret_cast<const uint64_t *>(p);
}

// Bounded global memory: a buffer resource covers [base, base + bytes) and the
// hardware returns 0 for reads and drops writes outside it, so a wrong or
// hostile offset cannot reach other memory. Offsets are 32-bit byte offsets.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
constexpr int kBufferFlags = 0x00020000;  // raw 32-bit buffer, gfx9 family

struct Buf {
    __amdgpu_buffer_rsrc_t r;
};

__device__ __forceinline__ Buf make_buf(const void *base, uint32_t bytes) {
    Buf b;
    b.r = __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, kBufferFlags);
    return b;
}

__device__ __forceinline__ uint32_t buf_ld32(Buf b, uint32_t off) {
    return __builtin_amdgcn_raw_buffer_load_b32(b.r, off, 0, 0);
}

__device__ __forceinline__ uint32_t buf_ld8(Buf b, uint32_t off) {
    return __builtin_amdgcn_raw_buffer_load_b8(b.r, off, 0, 0);
}

__device__ __forceinline__ u32x4 buf_ld128(Buf b, uint32_t off) {
    return __builtin_amdgcn_raw_buffer_load_b128(b.r, off, 0, 0);
}

__device__ __forceinline__ void buf_st8(Buf b, uint32_t off, uint32_t v) {
    __builtin_amdgcn_raw_buffer_store_b8((uint8_t)v, b.r, off, 0, 0);
}

__device__ __forceinline__ void buf_st16(Buf b, uint32_t off, uint32_t v) {
    __builtin_amdgcn_raw_buffer_store_b16((uint16_t)v, b.r, off, 0, 0);
}

__device__ __forceinline__ void buf_st32(Buf b, uint32_t off, uint32_t v) {
    __builtin_amdgcn_raw_buffer_store_b32(v, b.r, off, 0, 0);
}

__device__ __forceinline__ void buf_st128(Buf b, uint32_t off, u32x4 v) {
    __builtin_amdgcn_raw_buffer_store_b128(v, b.r, off, 0, 0);
}

// Hand-off point between lanes of one wavefront through LDS: the lanes run
// in lockstep and a wavefront's LDS accesses complete in order, so this only
// keeps the compiler from moving memory accesses across the point.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Global-memory accessors for pointers the compiler cannot trace to a kernel
// argument (for instance pointers kept in LDS): without the address space they
// become flat accesses, which also count against the LDS wait counter.
#define SPZ_GLOBAL __attribute__((address_space(1)))
__device__ __forceinline__ u32x4 gld128(const uint8_t *p) { return *(const SPZ_GLOBAL u32x4 *)p; }
__device__ __forceinline__ void gst128(uint8_t *p, u32x4 v) { *(SPZ_GLOBAL u32x4 *)p = v; }
__device__ __forceinline__ void gst32(uint8_t *p, uint32_t v) { *(SPZ_GLOBAL uint32_t *)p = v; }
__device__ __forceinline__ uint32_t gld8(const uint8_t *p) { return *(const SPZ_GLOBAL uint8_t *)p; }
__device__ __forceinline__ uint32_t gld32(const uint8_t *p) { return *(const SPZ_GLOBAL uint32_t *)p; }
__device__ __forceinline__ uint64_t gld64(const uint8_t *p) { return *(const SPZ_GLOBAL uint64_t *)p; }
__device__ __forceinline__ void gst8(uint8_t *p, uint32_t v) { *(SPZ_GLOBAL uint8_t *)p = (uint8_t)v; }

// Make a value the compiler cannot prove uniform usable as a scalar operand.
__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    return ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32)) << 32) |
           __builtin_amdgcn_readfirstlane((uint32_t)v);
}

}  // namespace spz

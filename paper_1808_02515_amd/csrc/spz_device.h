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

// Memory accessors, cross-lane hand-off and the one inline-asm operation live
// in their own header, found on the include path (the HIP build's csrc/
// directory), so that a host build of the kernels can put bounds-checked
// versions in their place.
#include <spz_device_ops.h>

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

}  // namespace spz

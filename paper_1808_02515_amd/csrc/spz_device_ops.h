// Hardware-specific operations of the gfx950 Sprintz kernels: bounded
// buffer resources, plain global accessors, the wavefront hand-off point, the
// sign in one v_med3_i32 and a 24-bit product with a sign-extended byte. Included by spz_device.h through the include
// path, so that a host build of the kernel source can supply checked
// versions of exactly these operations.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spz {

// sign(e) in one v_med3_i32 (the compiler lowers min(max(e, -1), 1) to two
// compare/select pairs).
__device__ __forceinline__ int32_t sgn_med3(int32_t e) {
    int32_t r;
    asm("v_med3_i32 %0, %1, -1, 1" : "=v"(r) : "v"(e));
    return r;
}

// a * (low byte of d, sign-extended) in one v_mul_i32_i24 with an SDWA
// operand (a within 24 bits). Written out because the compiler widens the
// 8-bit form into a 32-bit multiply.
__device__ __forceinline__ int32_t mul24_sext8(int32_t a, int32_t d) {
    int32_t p;
    asm("v_mul_i32_i24_sdwa %0, %1, sext(%2) dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_0"
        : "=v"(p)
        : "v"(a), "v"(d));
    return p;
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

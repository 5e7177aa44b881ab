// Bounds-checked host versions of the hardware-specific operations of the
// Sprintz kernels (the HIP build's own versions are in
// paper_1808_02515_amd/csrc/spz_device_ops.h). Every plain global access
// must lie inside a buffer the harness registered, every buffer resource
// must be made inside one; violations are counted (and the access skipped),
// and AddressSanitizer watches the host memory under all of it.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace emu {

struct Region { const uint8_t *p; size_t n; bool writable; };
inline std::vector<Region> &regions() { static std::vector<Region> r; return r; }
inline size_t &violations() { static size_t v = 0; return v; }
inline void add_region(const void *p, size_t n, bool writable) { regions().push_back({(const uint8_t *)p, n, writable}); }

inline bool inside(const void *p, size_t n, bool write) {
    const uint8_t *q = (const uint8_t *)p;
    for (const Region &r : regions())
        if (q >= r.p && q + n <= r.p + r.n && (!write || r.writable)) return true;
    if (violations()++ < 20)
        fprintf(stderr, "emulation: %s of %zu bytes at %p outside every registered buffer (thread %u)\n",
                write ? "write" : "read", n, p, me().tid.x);
    return false;
}

}  // namespace emu

namespace spz {

__device__ __forceinline__ int32_t sgn_med3(int32_t e) { return e < -1 ? -1 : e > 1 ? 1 : e; }
// v_mul_i32_i24 of a (low 24 bits, signed) and the sign-extended low byte of
// d; the low 32 bits of the product
__device__ __forceinline__ int32_t mul24_sext8(int32_t a, int32_t d) {
    const int64_t a24 = (int64_t)(int32_t)((uint32_t)a << 8) >> 8;
    return (int32_t)(uint32_t)(uint64_t)(a24 * (int64_t)(int8_t)d);
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// A buffer resource: reads outside [base, base + bytes) give 0 and writes
// there are dropped, as the hardware does.
struct Buf {
    const uint8_t *base;
    uint32_t bytes;
};

__device__ __forceinline__ Buf make_buf(const void *base, uint32_t bytes) {
    if (bytes) (void)emu::inside(base, bytes, false);   // the resource itself must cover real memory
    return Buf{(const uint8_t *)base, bytes};
}

template <typename T> inline T buf_load(Buf b, uint32_t off) {
    T v;
    if ((uint64_t)off + sizeof(T) > b.bytes) { memset(&v, 0, sizeof(T)); return v; }
    if (!emu::inside(b.base + off, sizeof(T), false)) { memset(&v, 0, sizeof(T)); return v; }
    memcpy(&v, b.base + off, sizeof(T));
    return v;
}
template <typename T> inline void buf_store(Buf b, uint32_t off, T v) {
    if ((uint64_t)off + sizeof(T) > b.bytes) return;
    if (!emu::inside(b.base + off, sizeof(T), true)) return;
    memcpy(const_cast<uint8_t *>(b.base) + off, &v, sizeof(T));
}

__device__ __forceinline__ uint32_t buf_ld32(Buf b, uint32_t off) { return buf_load<uint32_t>(b, off); }
__device__ __forceinline__ uint32_t buf_ld8(Buf b, uint32_t off) { return buf_load<uint8_t>(b, off); }
__device__ __forceinline__ u32x4 buf_ld128(Buf b, uint32_t off) { return buf_load<u32x4>(b, off); }
__device__ __forceinline__ void buf_st8(Buf b, uint32_t off, uint32_t v) { buf_store<uint8_t>(b, off, (uint8_t)v); }
__device__ __forceinline__ void buf_st16(Buf b, uint32_t off, uint32_t v) { buf_store<uint16_t>(b, off, (uint16_t)v); }
__device__ __forceinline__ void buf_st32(Buf b, uint32_t off, uint32_t v) { buf_store<uint32_t>(b, off, v); }
__device__ __forceinline__ void buf_st128(Buf b, uint32_t off, u32x4 v) { buf_store<u32x4>(b, off, v); }

__device__ __forceinline__ void wave_sync() { emu::wave_sync(); }

template <typename T> inline T gload(const uint8_t *p) {
    T v;
    memset(&v, 0, sizeof(T));
    if (emu::inside(p, sizeof(T), false)) memcpy(&v, p, sizeof(T));
    return v;
}
template <typename T> inline void gstore(uint8_t *p, T v) {
    if (emu::inside(p, sizeof(T), true)) memcpy(p, &v, sizeof(T));
}
__device__ __forceinline__ u32x4 gld128(const uint8_t *p) { return gload<u32x4>(p); }
__device__ __forceinline__ void gst128(uint8_t *p, u32x4 v) { gstore<u32x4>(p, v); }
__device__ __forceinline__ void gst32(uint8_t *p, uint32_t v) { gstore<uint32_t>(p, v); }
__device__ __forceinline__ uint32_t gld8(const uint8_t *p) { return gload<uint8_t>(p); }
__device__ __forceinline__ uint32_t gld32(const uint8_t *p) { return gload<uint32_t>(p); }
__device__ __forceinline__ uint64_t gld64(const uint8_t *p) { return gload<uint64_t>(p); }
__device__ __forceinline__ void gst8(uint8_t *p, uint32_t v) { gstore<uint8_t>(p, (uint8_t)v); }

__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    return ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32)) << 32) |
           __builtin_amdgcn_readfirstlane((uint32_t)v);
}

}  // namespace spz

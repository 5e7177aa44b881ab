// Host runtime and C ABI of the gfx950 Sprintz codec (see include/sprintz.h).
//
// Compression: pass-1 sizing kernel -> offset-table scan -> pass-2 writing
// kernel, all on the caller's stream. Decompression: one kernel. The host
// only validates arguments, derives the launch geometry and enqueues.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "sprintz.h"
#include "spz_decode.h"
#include "spz_decode_pc.h"
#include "spz_encode.h"
#include "spz_encode_chunked.h"
#include "spz_encode_sp.h"
#include "spz_entropy.h"

namespace {

constexpr uint32_t kMaxD = 128;
constexpr uint32_t kMaxSegRows = 1u << 20;
constexpr size_t kHeader = 64;

uint32_t bits_of(spz_dtype d) {
    switch (d) {
        case SPZ_INT8: case SPZ_UINT8: return 8;
        case SPZ_INT16: case SPZ_UINT16: return 16;
        default: return 0;
    }
}

uint32_t log2_pow2_ceil(uint32_t v) {
    uint32_t k = 0;
    while ((1u << k) < v) ++k;
    return k;
}

size_t align16(size_t v) { return (v + 15) & ~size_t(15); }
size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// seg_rows 0 (autotuned) is accepted where allow_tuned is set: by the
// compression calls, not in a container
spz_status check_params(const spz_params *p, bool allow_tuned = false) {
    if (!p || p->struct_size < sizeof(spz_params)) return SPZ_EINVAL;
    if (p->forecaster != SPZ_DELTA && p->forecaster != SPZ_FIRE) return SPZ_EINVAL;
    if (!(allow_tuned && p->seg_rows == 0) && (p->seg_rows < 8 || p->seg_rows % 8 != 0 || p->seg_rows > kMaxSegRows))
        return SPZ_EINVAL;
    if (p->hdr_group > 255 || p->learn_shift > 8 || p->entropy > 1) return SPZ_EINVAL;
    return SPZ_OK;
}

uint64_t num_segments(uint64_t rows, uint32_t S) { return rows == 0 ? 0 : (rows + S - 1) / S; }

// Segment sizes the autotuner chooses from for a series of `rows` rows: the
// reference size (one segment over the first 2^20 rows, the paper's
// unsegmented stream) and the fixed candidates below it.
constexpr uint32_t kTuneCands[] = {256, 512, 1024, 2048, 4096};
std::vector<uint32_t> tune_candidates(uint64_t rows) {
    const uint64_t r = std::max<uint64_t>(8, std::min<uint64_t>(rows, kMaxSegRows));
    const uint32_t ref = (uint32_t)((r + 7) & ~7ull);
    std::vector<uint32_t> c{ref};
    for (uint32_t S : kTuneCands)
        if (S < ref) c.push_back(S);
    return c;
}

spz::Geom make_geom(uint64_t rows, uint32_t D, uint32_t w, uint32_t S, uint32_t G, uint32_t learn_shift) {
    spz::Geom g;
    memset(&g, 0, sizeof(g));
    g.rows = rows;
    g.D = D;
    g.S = S;
    g.nseg = (uint32_t)num_segments(rows, S);
    g.dp_log2 = log2_pow2_ceil(D);
    g.G = G;
    g.sh = learn_shift + 2;
    g.acc_lo = -(int32_t)((1u << (w - 1)) << g.sh);
    g.acc_hi = (int32_t)((1u << w) << g.sh);
    g.data_start = align16(kHeader + 8ull * (g.nseg + 1));
    return g;
}

// Walker kernels: one lane group of min(Dp, 64) lanes per segment.
uint32_t grid_for(const spz::Geom &g) {
    uint64_t lanes = (uint64_t)g.nseg << std::min<uint32_t>(g.dp_log2, 6);
    return (uint32_t)((lanes + spz::kThreads - 1) / spz::kThreads);
}

// The chunked encoder needs one header group per segment, 16-byte aligned
// segment rows in a 16-byte aligned input, and the workgroup's whole-segment
// header arrays and chunk payloads inside its LDS staging buffers; anything
// else goes through the per-lane walker.
bool enc_chunked_ok(const spz::Geom &g, uint32_t w, const void *src) {
    if (g.G != 0 || g.D > 64 || ((uintptr_t)src & 15) || ((uint64_t)g.S * g.D * (w / 8)) % 16 != 0) return false;
    const uint32_t spw = 64u >> g.dp_log2;
    const uint32_t cb = spz::enc_chunk_blocks(g.dp_log2);
    const uint64_t hdr_seg = (spz::enc_hdr_cap(g.S >> 3, g.D, w) + 15) & ~15ull;
    const uint64_t out_seg = ((uint64_t)cb * 8 * g.D * (w / 8) + 6 * cb + 15) & ~15ull;
    return spw * hdr_seg <= (uint64_t)spz::kEncHdrBytes && spw * out_seg <= 4ull * spz::kEncOutWords;
}

// The single-pass encoder takes whole-segment header groups, D <= 16,
// 16-byte aligned input rows of every segment and a 16-byte aligned
// workspace of sp_workspace_bytes; the two-pass encoders below need only
// 8 bytes per segment.
bool enc_sp_ok(const spz::Geom &g, uint32_t w, const void *src, const void *ws) {
    return g.G == 0 && g.D >= 1 && g.D <= 16 && !((uintptr_t)src & 15) && !((uintptr_t)ws & 15) &&
           ((uint64_t)g.S * g.D * (w / 8)) % 16 == 0;
}

uint64_t sp_slot_stride(uint32_t S, uint32_t D, uint32_t w) { return spz::es_slot_bytes(S >> 3, D, w); }

size_t sp_workspace_bytes(uint64_t nseg, uint32_t S, uint32_t D, uint32_t w) {
    return align256(16 * (size_t)nseg) + (size_t)(nseg * sp_slot_stride(S, D, w));
}

template <int W, bool FIRE, int D>
void launch_enc_sp_kernel(const void *src, const spz::Geom &g, uint8_t *slots, uint64_t stride, spz::u32x4 *info,
                          hipStream_t stream) {
    using G = spz::EsGeom<W, D>;
    const uint32_t grid = (g.nseg + G::SPW - 1) / G::SPW;
    hipLaunchKernelGGL((spz::k_encode_sp<W, FIRE, D>), dim3(grid), dim3(G::NT), 0, stream, (const uint8_t *)src, g,
                       slots, stride, info);
}

template <int W, bool FIRE>
hipError_t launch_encode_sp(const void *src, const spz::Geom &g, uint8_t *ws, uint8_t *dst, int32_t *status,
                            uint32_t dtype, uint32_t forecaster, uint32_t learn_shift, uint64_t *out_size,
                            hipStream_t stream) {
    const uint64_t stride = sp_slot_stride(g.S, g.D, W);
    spz::u32x4 *info = reinterpret_cast<spz::u32x4 *>(ws);
    uint8_t *slots = ws + align256(16 * (size_t)g.nseg);
    if (g.nseg > 0) {
        switch (g.D) {
#define SPZ_ESP(D_) case D_: launch_enc_sp_kernel<W, FIRE, D_>(src, g, slots, stride, info, stream); break;
            SPZ_ESP(1) SPZ_ESP(2) SPZ_ESP(3) SPZ_ESP(4) SPZ_ESP(5) SPZ_ESP(6) SPZ_ESP(7) SPZ_ESP(8)
            SPZ_ESP(9) SPZ_ESP(10) SPZ_ESP(11) SPZ_ESP(12) SPZ_ESP(13) SPZ_ESP(14) SPZ_ESP(15) SPZ_ESP(16)
#undef SPZ_ESP
            default: return hipErrorInvalidValue;
        }
    }
    hipLaunchKernelGGL(spz::k_enc_scan, dim3(1), dim3(1024), 0, stream, info, g, (uint32_t)W, dtype, forecaster,
                       learn_shift, dst, out_size, status);
    if (g.nseg > 0) {
        const uint64_t units = stride / 16;
        const uint32_t K = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(256, 2048 / units));
        hipLaunchKernelGGL(spz::k_enc_compact, dim3((g.nseg + K - 1) / K), dim3(256), 0, stream, slots, stride, info,
                           g, (uint32_t)W, K, dst, status);
    }
    return hipGetLastError();
}

template <int W, bool FIRE, bool COL>
hipError_t launch_encode(const void *src, const spz::Geom &g, uint32_t *ws, uint8_t *dst, int32_t *status,
                         uint32_t dtype, uint32_t forecaster, uint32_t learn_shift, uint64_t *out_size,
                         hipStream_t stream) {
    using T = typename spz::Elem<W>::T;
    if (g.nseg > 0 && enc_chunked_ok(g, W, src)) {
        const uint32_t spw = 64u >> g.dp_log2;
        const uint32_t grid = (g.nseg + spw - 1) / spw;
        hipLaunchKernelGGL((spz::k_encode_chunked<W, FIRE, COL, false>), dim3(grid), dim3(spz::kThreads), 0,
                           stream, (const uint8_t *)src, g, ws, dst, status);
        hipLaunchKernelGGL(spz::k_scan_sizes, dim3(1), dim3(1024), 0, stream, ws, g, (uint32_t)W, dtype,
                           forecaster, learn_shift, dst, out_size, status);
        hipLaunchKernelGGL((spz::k_encode_chunked<W, FIRE, COL, true>), dim3(grid), dim3(spz::kThreads), 0,
                           stream, (const uint8_t *)src, g, ws, dst, status);
        return hipGetLastError();
    }
    const uint32_t grid = grid_for(g);
    if (grid > 0)
        hipLaunchKernelGGL((spz::k_encode<W, FIRE, COL, false>), dim3(grid), dim3(spz::kThreads), 0, stream,
                           (const T *)src, g, ws, dst, status);
    hipLaunchKernelGGL(spz::k_scan_sizes, dim3(1), dim3(1024), 0, stream, ws, g, (uint32_t)W, dtype, forecaster,
                       learn_shift, dst, out_size, status);
    if (grid > 0)
        hipLaunchKernelGGL((spz::k_encode<W, FIRE, COL, true>), dim3(grid), dim3(spz::kThreads), 0, stream,
                           (const T *)src, g, ws, dst, status);
    return hipGetLastError();
}

// The producer/consumer decoder takes whole-segment header groups, D <= 16
// and 16-byte aligned output rows; everything else (D > 16 too, where it
// measured faster than a chunked workgroup decoder) takes the walker.
bool chunked_ok(const spz::Geom &g, uint32_t w, const void *dst) {
    return g.G == 0 && ((uintptr_t)dst & 15) == 0 && ((uint64_t)g.S * g.D * (w / 8)) % 16 == 0;
}

template <int W, bool FIRE, bool COL>
hipError_t launch_decode(const void *src, const spz::Geom &g, void *dst, int32_t *status, hipStream_t stream) {
    using T = typename spz::Elem<W>::T;
    if (g.nseg == 0) return hipGetLastError();
    if (chunked_ok(g, W, dst) && g.D <= 16) {
        const uint32_t spw = spz::pc_spw(g.D, spz::kPcProducers, spz::kPcConsumers);
        const uint32_t grid = (g.nseg + spw - 1) / spw;
        switch (g.D) {
#define SPZ_PC(D_)                                                                                        \
    case D_:                                                                                              \
        hipLaunchKernelGGL((spz::k_decode_pc<W, FIRE, D_, spz::kPcProducers, spz::kPcConsumers>), dim3(grid), \
                           dim3(spz::pc_single_threads(D_, spz::kPcProducers, spz::kPcConsumers)), 0, stream,  \
                           (const uint8_t *)src, g, (T *)dst, status);                                    \
        break;
            SPZ_PC(1) SPZ_PC(2) SPZ_PC(3) SPZ_PC(4) SPZ_PC(5) SPZ_PC(6) SPZ_PC(7) SPZ_PC(8)
            SPZ_PC(9) SPZ_PC(10) SPZ_PC(11) SPZ_PC(12) SPZ_PC(13) SPZ_PC(14) SPZ_PC(15) SPZ_PC(16)
#undef SPZ_PC
        }
    } else {
        hipLaunchKernelGGL((spz::k_decode<W, FIRE, COL>), dim3(grid_for(g)), dim3(spz::kThreads), 0, stream,
                           (const uint8_t *)src, g, (T *)dst, status);
    }
    return hipGetLastError();
}

uint64_t get_le(const uint8_t *p, int n) {
    uint64_t v = 0;
    for (int k = 0; k < n; ++k) v |= (uint64_t)p[k] << (8 * k);
    return v;
}

// Compression workspace of sprintz_compress_noalloc: a device array of fixed
// size that every GPU the library runs on holds until the process ends. In
// host code its name is only a stand-in; kernels get the device address that
// hipGetSymbolAddress returns, looked up once per device.
constexpr size_t kScratchBytes = 4u << 20;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;   // device -> address of its scratch array

spz_status scratch_address(void **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SPZ_EHIP;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) { *out = it->second; return SPZ_OK; }
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return SPZ_EHIP;
    g_scratch_ptr[dev] = p;
    *out = p;
    return SPZ_OK;
}

}  // namespace

extern "C" {

void spz_params_default(spz_params *p) {
    if (!p) return;
    memset(p, 0, sizeof(*p));
    p->struct_size = sizeof(spz_params);
    p->forecaster = SPZ_FIRE;
    p->seg_rows = 1024;
    p->hdr_group = 0;
    p->learn_shift = 1;
    p->entropy = 0;
}

// Largest plain segment of a container shape (16-byte multiple): the
// decoder's stride for entropy-coded containers.
static uint64_t plain_segment_max(uint64_t rows, uint32_t D, uint32_t w, const spz_params *p) {
    const uint32_t hb = w == 8 ? 3 : 4;
    const uint64_t r = std::min<uint64_t>(rows, p->seg_rows);
    const uint64_t nblk = r / 8, tail = r % 8;
    const uint64_t ngroups = p->hdr_group == 0 ? 1 : (nblk + p->hdr_group - 1) / p->hdr_group;
    const uint64_t one = 4 + (nblk * D * hb + 7) / 8 + ngroups + nblk * D * w + tail * D * (w / 8) + 15;
    return (one + 15) & ~15ull;
}

static constexpr uint64_t kHufLdsMax = 60 * 1024;   // coded segment image of the entropy write pass

static size_t bound_fixed(uint64_t rows, uint32_t D, spz_dtype dtype, const spz_params *p) {
    const uint32_t w = bits_of(dtype);
    if (w == 0 || D == 0 || check_params(p) != SPZ_OK) return 0;
    if (p->entropy == 1) {
        const uint64_t nseg = num_segments(rows, p->seg_rows);
        return align16(kHeader + 8 * (size_t)(nseg + 1)) +
               (size_t)(nseg * spz::huff_segment_bound(plain_segment_max(rows, D, w, p)));
    }
    const uint32_t hb = w == 8 ? 3 : 4;
    const uint32_t S = p->seg_rows;
    const uint64_t nseg = num_segments(rows, S);
    size_t total = align16(kHeader + 8 * (size_t)(nseg + 1));
    // all full segments are alike; the last one may be short
    for (int last = 0; last < 2; ++last) {
        if (nseg == 0) break;
        const uint64_t count = last ? 1 : nseg - 1;
        const uint64_t r = last ? rows - (uint64_t)S * (nseg - 1) : S;
        const uint64_t nblk = r / 8, tail = r % 8;
        const uint64_t ngroups = p->hdr_group == 0 ? 1 : (nblk + p->hdr_group - 1) / p->hdr_group;
        const uint64_t one = 4 + (nblk * D * hb + 7) / 8 + ngroups + nblk * D * w + tail * D * (w / 8) + 15;
        total += (size_t)(count * one);
    }
    return total;
}

static size_t ws_fixed(uint64_t rows, uint32_t D, spz_dtype dtype, const spz_params *p);

static size_t ws_min_fixed(uint64_t rows, uint32_t D, spz_dtype dtype, const spz_params *p) {
    if (bits_of(dtype) == 0 || D == 0 || check_params(p) != SPZ_OK) return 0;
    if (p->entropy == 1) return ws_fixed(rows, D, dtype, p);
    return 8 * (size_t)num_segments(rows, p->seg_rows) + 8;
}

static size_t ws_fixed(uint64_t rows, uint32_t D, spz_dtype dtype, const spz_params *p) {
    if (bits_of(dtype) == 0 || D == 0 || check_params(p) != SPZ_OK) return 0;
    const uint64_t nseg = num_segments(rows, p->seg_rows);
    const uint32_t w = bits_of(dtype);
    if (p->entropy == 0 && p->hdr_group == 0 && D <= 16)
        return std::max(sp_workspace_bytes(nseg, p->seg_rows, D, w), 8 * (size_t)nseg + 8);
    if (p->entropy == 1) {
        // plain container | its workspace | per-segment code records | plain size
        spz_params pp = *p;
        pp.entropy = 0;
        return align256(bound_fixed(rows, D, dtype, &pp)) +
               align256(ws_fixed(rows, D, dtype, &pp)) + align256(nseg * spz::kHufInfo) + 256;
    }
    return 8 * (size_t)nseg + 8;
}

}  // extern "C"

// With seg_rows 0 (autotuned) the sizes hold for every candidate the
// autotuner can choose.
template <typename F> static size_t over_candidates(uint64_t rows, const spz_params *p, F f) {
    if (!p || p->struct_size < sizeof(spz_params)) return 0;
    if (p->seg_rows != 0) return f(p);
    size_t m = 0;
    for (uint32_t S : tune_candidates(rows)) {
        spz_params q = *p;
        q.seg_rows = S;
        const size_t v = f(&q);
        if (v == 0) return 0;
        m = std::max(m, v);
    }
    return m;
}

extern "C" {

size_t sprintz_compress_bound(uint64_t rows, uint32_t D, spz_dtype dtype, const spz_params *p) {
    return over_candidates(rows, p, [&](const spz_params *q) { return bound_fixed(rows, D, dtype, q); });
}

size_t sprintz_workspace_size(uint64_t rows, uint32_t D, spz_dtype dtype, const spz_params *p) {
    return over_candidates(rows, p, [&](const spz_params *q) { return ws_fixed(rows, D, dtype, q); });
}

size_t sprintz_workspace_size_min(uint64_t rows, uint32_t D, spz_dtype dtype, const spz_params *p) {
    return over_candidates(rows, p, [&](const spz_params *q) { return ws_min_fixed(rows, D, dtype, q); });
}

// Entropy-coded compression: the plain container into the workspace, then
// the Huffman size pass, offsets and write pass (Section 4.4).
static spz_status compress_entropy(const void *d_src, uint64_t rows, uint32_t D, spz_dtype dtype, const spz_params *p,
                            void *d_dst, size_t dst_cap, uint64_t *d_out_size, void *d_ws, int32_t *d_status,
                            hipStream_t stream) {
    const uint32_t w = bits_of(dtype);
    spz_params pp = *p;
    pp.entropy = 0;
    const uint64_t nseg = num_segments(rows, p->seg_rows);
    // LDS image of the write pass: the largest coded segment, at most
    // kHufLdsMax (larger segments are written in place in the container)
    const uint64_t ldsb = std::min<uint64_t>(spz::huff_segment_bound(plain_segment_max(rows, D, w, p)), kHufLdsMax);
    const size_t plain_cap = sprintz_compress_bound(rows, D, dtype, &pp);
    const size_t plain_ws = sprintz_workspace_size(rows, D, dtype, &pp);
    uint8_t *P = (uint8_t *)d_ws;
    uint8_t *W1 = P + align256(plain_cap);
    uint8_t *info = W1 + align256(plain_ws);
    uint64_t *psize = (uint64_t *)(info + align256(nseg * spz::kHufInfo));
    const spz_status st = sprintz_compress(d_src, rows, D, dtype, &pp, P, plain_cap, psize, W1, plain_ws, d_status,
                                           stream);
    if (st != SPZ_OK) return st;
    const uint64_t data_start = align16(kHeader + 8 * (nseg + 1));
    if (nseg > 0)
        hipLaunchKernelGGL(spz::k_huff_size, dim3((uint32_t)nseg), dim3(64), 0, stream, P, data_start, (uint32_t)nseg,
                           info, d_status);
    hipLaunchKernelGGL(spz::k_huff_scan, dim3(1), dim3(1024), 0, stream, P, (uint32_t)nseg, data_start, info,
                       (uint8_t *)d_dst, (uint64_t)dst_cap, d_out_size, d_status);
    if (nseg > 0)
        hipLaunchKernelGGL(spz::k_huff_write, dim3((uint32_t)nseg), dim3(256), (uint32_t)ldsb, stream, P, data_start,
                           (uint32_t)nseg, info, (uint8_t *)d_dst, (uint32_t)ldsb, d_status);
    return hipGetLastError() == hipSuccess ? SPZ_OK : SPZ_EHIP;
}

}  // extern "C"

namespace {

// The autotuner's cache: one segment size per shape class (the first series
// of a class is measured, later ones reuse its choice).
struct TuneKey {
    uint32_t D, w, forecaster, learn_shift, hdr_group, entropy, ref;
    bool operator<(const TuneKey &o) const {
        const uint32_t a[7] = {D, w, forecaster, learn_shift, hdr_group, entropy, ref};
        const uint32_t b[7] = {o.D, o.w, o.forecaster, o.learn_shift, o.hdr_group, o.entropy, o.ref};
        return std::lexicographical_compare(a, a + 7, b, b + 7);
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, uint32_t> g_tune;

// series of one power-of-two size class of their sample share a key
TuneKey tune_key(uint64_t rows, uint32_t D, uint32_t w, const spz_params *p) {
    const uint32_t ref = tune_candidates(rows)[0];
    return TuneKey{D, w, p->forecaster, p->learn_shift, p->hdr_group, p->entropy, 32u - (uint32_t)__builtin_clz(ref)};
}

// The choice rule: the reference (cands[0], one segment) only sets the bar.
// Among the other candidates, those whose container is at most 1 % above the
// reference's, the fastest decode; if none qualifies, the smallest container
// (its loss is then above 1 %). Ties go to the candidate listed first. With
// no other candidate, the reference.
uint32_t tune_pick(const std::vector<uint32_t> &cands, const std::vector<uint64_t> &bytes,
                   const std::vector<float> &ms) {
    if (cands.size() == 1) return cands[0];
    int best = -1;
    for (size_t k = 1; k < cands.size(); ++k)
        if (bytes[k] * 100 <= bytes[0] * 101 && (best < 0 || ms[k] < ms[best])) best = (int)k;
    if (best >= 0) return cands[best];
    size_t small = 1;
    for (size_t k = 2; k < cands.size(); ++k)
        if (bytes[k] < bytes[small]) small = k;
    return cands[small];
}

}  // namespace

extern "C" {

spz_status sprintz_autotune(const void *d_src, uint64_t rows, uint32_t D, spz_dtype dtype, const spz_params *p,
                            uint32_t *seg_rows_out, hipStream_t stream) {
    const uint32_t w = bits_of(dtype);
    if (!seg_rows_out || w == 0 || D == 0 || check_params(p, true) != SPZ_OK) return SPZ_EINVAL;
    if (D > kMaxD) return SPZ_EUNSUPPORTED;
    if (rows > 0 && !d_src) return SPZ_EINVAL;
    const std::vector<uint32_t> cands = tune_candidates(rows);
    const uint64_t n = std::min<uint64_t>(rows, kMaxSegRows);   // the sample: the first 2^20 rows
    if (cands.size() == 1) {                                    // one segment is the only choice
        *seg_rows_out = cands[0];
        return SPZ_OK;
    }
    spz_params q = *p;
    q.seg_rows = 0;
    const size_t cap = sprintz_compress_bound(n, D, dtype, &q), wsz = sprintz_workspace_size(n, D, dtype, &q);
    const size_t ybytes = (size_t)(n * D * (w / 8));
    uint8_t *dst = nullptr, *ws = nullptr, *y = nullptr;
    uint64_t *small = nullptr;   // [0] container bytes, [1] status words
    hipEvent_t ev[2] = {nullptr, nullptr};
    spz_status st = SPZ_OK;
    std::vector<uint64_t> bytes;
    std::vector<float> ms;
    if (hipMalloc(&dst, cap) != hipSuccess || hipMalloc(&ws, wsz) != hipSuccess || hipMalloc(&y, ybytes) != hipSuccess ||
        hipMalloc(&small, 16) != hipSuccess || hipEventCreate(&ev[0]) != hipSuccess ||
        hipEventCreate(&ev[1]) != hipSuccess)
        st = SPZ_ENOMEM;
    for (size_t k = 0; st == SPZ_OK && k < cands.size(); ++k) {
        q.seg_rows = cands[k];
        hipLaunchKernelGGL(spz::k_zero_u32, dim3(1), dim3(64), 0, stream, (uint32_t *)small, 4u);
        st = sprintz_compress(d_src, n, D, dtype, &q, dst, cap, small, ws, wsz, (int32_t *)(small + 1), stream);
        uint64_t h[2] = {0, 0};
        uint8_t head[64];
        if (st == SPZ_OK && (hipMemcpyAsync(h, small, 16, hipMemcpyDeviceToHost, stream) != hipSuccess ||
                             hipMemcpyAsync(head, dst, 64, hipMemcpyDeviceToHost, stream) != hipSuccess ||
                             hipStreamSynchronize(stream) != hipSuccess))
            st = SPZ_EHIP;
        if (st == SPZ_OK && h[1] != 0) st = SPZ_EHIP;
        spz_info info;
        if (st == SPZ_OK) st = sprintz_get_info(head, 64, &info);
        float best = 0;
        for (int rep = 0; st == SPZ_OK && rep < 4; ++rep) {   // one warm-up, best of three
            if (hipEventRecord(ev[0], stream) != hipSuccess) st = SPZ_EHIP;
            if (st == SPZ_OK) st = sprintz_decompress(dst, cap, &info, y, ybytes, nullptr, stream);
            float t = 0;
            if (st == SPZ_OK && (hipEventRecord(ev[1], stream) != hipSuccess || hipEventSynchronize(ev[1]) != hipSuccess ||
                                 hipEventElapsedTime(&t, ev[0], ev[1]) != hipSuccess))
                st = SPZ_EHIP;
            if (rep == 1 || (rep > 1 && t < best)) best = t;
        }
        bytes.push_back(h[0]);
        ms.push_back(best);
    }
    if (ev[0]) (void)hipEventDestroy(ev[0]);
    if (ev[1]) (void)hipEventDestroy(ev[1]);
    (void)hipFree(dst);
    (void)hipFree(ws);
    (void)hipFree(y);
    (void)hipFree(small);
    if (st != SPZ_OK) return st;
    const uint32_t S = tune_pick(cands, bytes, ms);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[tune_key(rows, D, w, p)] = S;
    }
    *seg_rows_out = S;
    return SPZ_OK;
}

spz_status sprintz_compress(const void *d_src, uint64_t rows, uint32_t D, spz_dtype dtype, const spz_params *p,
                            void *d_dst, size_t dst_cap, uint64_t *d_out_size, void *d_ws, size_t ws_size,
                            int32_t *d_status, hipStream_t stream) {
    const uint32_t w = bits_of(dtype);
    if (w == 0 || D == 0) return SPZ_EINVAL;
    spz_status st = check_params(p, true);
    if (st != SPZ_OK) return st;
    if (p->seg_rows == 0) {
        // autotuned: the cached choice of this shape class, else measure now
        if (D > kMaxD) return SPZ_EUNSUPPORTED;
        if (!d_dst || !d_out_size || (rows > 0 && !d_src) || !d_ws) return SPZ_EINVAL;
        if (dst_cap < sprintz_compress_bound(rows, D, dtype, p)) return SPZ_ENOSPC;
        if (ws_size < sprintz_workspace_size_min(rows, D, dtype, p)) return SPZ_ENOSPC;
        uint32_t S = 0;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tune.find(tune_key(rows, D, w, p));
            if (it != g_tune.end()) S = it->second;
        }
        if (S == 0) {
            st = sprintz_autotune(d_src, rows, D, dtype, p, &S, stream);
            if (st != SPZ_OK) return st;
        }
        spz_params q = *p;
        q.seg_rows = S;
        return sprintz_compress(d_src, rows, D, dtype, &q, d_dst, dst_cap, d_out_size, d_ws, ws_size, d_status, stream);
    }
    if (D > kMaxD) return SPZ_EUNSUPPORTED;
    if (num_segments(rows, p->seg_rows) > 0xFFFFFFFFull) return SPZ_EUNSUPPORTED;
    if (!d_dst || !d_out_size || (rows > 0 && !d_src) || !d_ws) return SPZ_EINVAL;
    if (((uintptr_t)d_dst & 15) || ((uintptr_t)d_src & (w / 8 - 1)) || ((uintptr_t)d_ws & 7) ||
        ((uintptr_t)d_out_size & 7))
        return SPZ_EINVAL;
    if (dst_cap < sprintz_compress_bound(rows, D, dtype, p)) return SPZ_ENOSPC;
    if (ws_size < sprintz_workspace_size_min(rows, D, dtype, p)) return SPZ_ENOSPC;
    if (p->entropy == 1) return compress_entropy(d_src, rows, D, dtype, p, d_dst, dst_cap, d_out_size, d_ws, d_status,
                                                 stream);
    spz::Geom g = make_geom(rows, D, w, p->seg_rows, p->hdr_group, p->learn_shift);
    g.cap = dst_cap;
    const bool col = (uint64_t)D * w <= 32;
    const bool fire = p->forecaster == SPZ_FIRE;
    uint32_t *ws = (uint32_t *)d_ws;
    uint8_t *dst = (uint8_t *)d_dst;
    hipError_t e;
    if (enc_sp_ok(g, w, d_src, d_ws) && ws_size >= sp_workspace_bytes(g.nseg, g.S, D, w)) {
        uint8_t *wsb = (uint8_t *)d_ws;
        if (w == 8) e = fire ? launch_encode_sp<8, true>(d_src, g, wsb, dst, d_status, (uint32_t)dtype, p->forecaster,
                                                         p->learn_shift, d_out_size, stream)
                             : launch_encode_sp<8, false>(d_src, g, wsb, dst, d_status, (uint32_t)dtype,
                                                          p->forecaster, p->learn_shift, d_out_size, stream);
        else e = fire ? launch_encode_sp<16, true>(d_src, g, wsb, dst, d_status, (uint32_t)dtype, p->forecaster,
                                                   p->learn_shift, d_out_size, stream)
                      : launch_encode_sp<16, false>(d_src, g, wsb, dst, d_status, (uint32_t)dtype, p->forecaster,
                                                    p->learn_shift, d_out_size, stream);
        return e == hipSuccess ? SPZ_OK : SPZ_EHIP;
    }
#define SPZ_ENC(W_, F_, C_) \
    launch_encode<W_, F_, C_>(d_src, g, ws, dst, d_status, (uint32_t)dtype, p->forecaster, p->learn_shift, d_out_size, stream)
    if (w == 8) {
        if (fire) e = col ? SPZ_ENC(8, true, true) : SPZ_ENC(8, true, false);
        else e = col ? SPZ_ENC(8, false, true) : SPZ_ENC(8, false, false);
    } else {
        if (fire) e = col ? SPZ_ENC(16, true, true) : SPZ_ENC(16, true, false);
        else e = col ? SPZ_ENC(16, false, true) : SPZ_ENC(16, false, false);
    }
#undef SPZ_ENC
    return e == hipSuccess ? SPZ_OK : SPZ_EHIP;
}

spz_status sprintz_compress_noalloc(const void *d_src, uint64_t rows, uint32_t D, spz_dtype dtype,
                                    const spz_params *p, void *d_dst, size_t dst_cap, uint64_t *d_out_size,
                                    int32_t *d_status, hipStream_t stream) {
    // the same kernels as sprintz_compress, with the library's scratch array
    // as the workspace; every value the kernels read from it is written by
    // the same call first, so nothing needs clearing between calls
    if (!p || p->seg_rows == 0) return SPZ_EINVAL;   // the autotuner allocates: pass a segment size
    const size_t need = sprintz_workspace_size_min(rows, D, dtype, p);
    if (need > kScratchBytes) return SPZ_ENOSPC;
    void *ws = nullptr;
    const spz_status st = scratch_address(&ws);
    if (st != SPZ_OK) return st;
    return sprintz_compress(d_src, rows, D, dtype, p, d_dst, dst_cap, d_out_size, ws, kScratchBytes, d_status,
                            stream);
}

spz_status sprintz_get_info(const void *h_src, size_t n, spz_info *out) {
    if (!h_src || !out) return SPZ_EINVAL;
    const uint8_t *s = (const uint8_t *)h_src;
    if (n < kHeader || memcmp(s, "SPZ1", 4) != 0 || get_le(s + 4, 2) != 1) return SPZ_ECORRUPT;
    spz_info info;
    memset(&info, 0, sizeof(info));
    info.w = s[6];
    info.dtype = s[7];
    spz_params_default(&info.params);
    info.params.forecaster = s[8];
    info.params.learn_shift = s[9];
    info.params.hdr_group = s[10];
    info.params.entropy = s[11];
    info.D = (uint32_t)get_le(s + 12, 4);
    info.rows = get_le(s + 16, 8);
    info.params.seg_rows = (uint32_t)get_le(s + 24, 4);
    info.nseg = (uint32_t)get_le(s + 28, 4);
    const uint64_t data_bytes = get_le(s + 32, 8);
    if (bits_of((spz_dtype)info.dtype) != info.w || info.D == 0) return SPZ_ECORRUPT;
    if (info.params.forecaster > 1 || info.params.learn_shift > 8 || info.params.entropy > 1) return SPZ_ECORRUPT;
    if (info.params.seg_rows < 8 || info.params.seg_rows % 8 != 0) return SPZ_ECORRUPT;
    if (num_segments(info.rows, info.params.seg_rows) != info.nseg) return SPZ_ECORRUPT;
    // every size must be representable: a data_bytes or a row count near 2^64
    // would otherwise wrap the container or output size and pass the checks
    // of check_decompress with an out-of-range extent
    const uint64_t data_start = align16(kHeader + 8ull * (info.nseg + 1));
    if (data_bytes > UINT64_MAX - data_start || data_bytes % 16 != 0) return SPZ_ECORRUPT;
    if (info.rows > UINT64_MAX / ((uint64_t)info.D * (info.w / 8))) return SPZ_ECORRUPT;
    info.compressed_size = data_start + data_bytes;
    info.decompressed_size = info.rows * info.D * (info.w / 8);
    *out = info;
    return SPZ_OK;
}

}  // extern "C"

namespace {

// Checks one decompression request; on success fills the launch geometry.
spz_status check_decompress(const void *d_src, size_t src_size, const spz_info *info, const void *d_dst,
                            size_t dst_cap, spz::Geom *g) {
    if (!info || !d_src) return SPZ_EINVAL;
    const uint32_t w = info->w;
    if (w != 8 && w != 16) return SPZ_EINVAL;
    if (check_params(&info->params) != SPZ_OK) return SPZ_EINVAL;
    if (info->D == 0) return SPZ_EINVAL;
    if (info->D > kMaxD) return SPZ_EUNSUPPORTED;
    if (info->nseg != num_segments(info->rows, info->params.seg_rows)) return SPZ_EINVAL;
    // the container's data must start inside it and the output size must not
    // wrap (a hand-made info could hold either)
    const uint64_t data_start = align16(kHeader + 8ull * ((uint64_t)info->nseg + 1));
    if (info->compressed_size < data_start) return SPZ_EINVAL;
    if (info->rows > UINT64_MAX / ((uint64_t)info->D * (w / 8))) return SPZ_EINVAL;
    if (info->compressed_size > src_size) return SPZ_ENOSPC;
    if (dst_cap < info->rows * info->D * (w / 8)) return SPZ_ENOSPC;
    if (info->rows > 0 && !d_dst) return SPZ_EINVAL;
    if (((uintptr_t)d_src & 15) || ((uintptr_t)d_dst & (w / 8 - 1))) return SPZ_EINVAL;
    *g = make_geom(info->rows, info->D, w, info->params.seg_rows, info->params.hdr_group, info->params.learn_shift);
    g->cap = src_size;
    g->data_bytes = info->compressed_size - g->data_start;
    return SPZ_OK;
}

hipError_t launch_decode_any(const void *d_src, const spz_info *info, const spz::Geom &g, void *d_dst,
                             int32_t *d_status, hipStream_t stream) {
    const uint32_t w = info->w;
    const bool col = (uint64_t)info->D * w <= 32;
    const bool fire = info->params.forecaster == SPZ_FIRE;
#define SPZ_DEC(W_, F_, C_) launch_decode<W_, F_, C_>(d_src, g, d_dst, d_status, stream)
    if (w == 8) {
        if (fire) return col ? SPZ_DEC(8, true, true) : SPZ_DEC(8, true, false);
        return col ? SPZ_DEC(8, false, true) : SPZ_DEC(8, false, false);
    }
    if (fire) return col ? SPZ_DEC(16, true, true) : SPZ_DEC(16, true, false);
    return col ? SPZ_DEC(16, false, true) : SPZ_DEC(16, false, false);
#undef SPZ_DEC
}

// Batched decoding: the workgroup kernels of one class (w, forecaster, D)
// share one compiled form; a plan holds one work list per class.
constexpr int kClasses = 2 * 2 * 16;   // w in {8, 16} x forecaster x D in 1..16
int class_of(uint32_t w, bool fire, uint32_t D) { return ((w == 16) * 2 + fire) * 16 + (int)(D - 1); }

// Concurrent class launches. A batch's class kernels are independent; run
// one after another, a class whose few long workgroups leave most of the GPU
// idle (small D: many segments per workgroup, few workgroups) keeps the
// others waiting. They go instead to up to kLanes streams: the caller's and
// kLanes - 1 side streams of the device (default priority, created once per
// device and kept), forked from and joined back into the caller's stream
// with events, so the call stays stream-ordered and can be captured in a
// HIP graph. Calls on different caller streams that share the side streams
// are ordered on them but stay correct.
constexpr int kLanes = 4;
hipError_t side_streams(hipStream_t *out) {
    static std::mutex mu;
    static std::map<int, std::vector<hipStream_t>> pool;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(mu);
    std::vector<hipStream_t> &v = pool[dev];
    while (v.size() < kLanes - 1) {
        hipStream_t s = nullptr;
        e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e != hipSuccess) return e;
        v.push_back(s);
    }
    for (int k = 0; k < kLanes - 1; ++k) out[k] = v[k];
    return hipSuccess;
}

// Fork/join events of one plan (created with the plan).
struct Lanes {
    hipEvent_t fork = nullptr, join[kLanes - 1] = {};
    bool ok = false;
    hipError_t create() {
        hipError_t e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
        for (int k = 0; k < kLanes - 1 && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&join[k], hipEventDisableTiming);
        ok = e == hipSuccess;
        return e;
    }
    void destroy() {
        if (fork) (void)hipEventDestroy(fork);
        for (int k = 0; k < kLanes - 1; ++k)
            if (join[k]) (void)hipEventDestroy(join[k]);
        fork = nullptr;
        ok = false;
    }
    // streams[0] = the caller's; launches go to streams[i % used]
    hipError_t begin(hipStream_t stream, int used, hipStream_t *streams) const {
        streams[0] = stream;
        if (used <= 1) return hipSuccess;
        hipError_t e = side_streams(streams + 1);
        if (e == hipSuccess) e = hipEventRecord(fork, stream);
        for (int k = 1; k < used && e == hipSuccess; ++k) e = hipStreamWaitEvent(streams[k], fork, 0);
        return e;
    }
    hipError_t end(int used, hipStream_t *streams) const {
        hipError_t e = hipSuccess;
        for (int k = 1; k < used && e == hipSuccess; ++k) {
            e = hipEventRecord(join[k - 1], streams[k]);
            if (e == hipSuccess) e = hipStreamWaitEvent(streams[0], join[k - 1], 0);
        }
        return e;
    }
};

// Classes with work, longest first (samples, with a per-record share that
// weighs small D): the longest runs on the caller's stream, the rest spread
// over the side streams.
template <typename Cost> int lane_order(const uint32_t *ngroups, Cost cost, int *order) {
    int n = 0;
    for (int c = 0; c < kClasses; ++c)
        if (ngroups[c]) order[n++] = c;
    std::stable_sort(order, order + n, [&](int x, int y) { return cost(x) > cost(y); });
    return n;
}
uint32_t class_D(int c) { return (uint32_t)(c % 16) + 1; }
uint32_t class_w(int c) { return (c / 32) ? 16 : 8; }
bool class_fire(int c) { return (c / 16) % 2; }

template <int W, bool FIRE, int D>
hipError_t launch_batch_class(const spz::PcStream *streams, const uint64_t *entries, const uint32_t *group_s,
                              uint32_t ngroups, uint32_t *queue, int32_t *status, uint32_t grid, hipStream_t stream) {
    hipLaunchKernelGGL((spz::k_decode_pc_batch<W, FIRE, D, spz::kPcProducers, spz::kPcConsumers>), dim3(grid),
                       dim3(spz::pc_threads(spz::kPcProducers, spz::kPcConsumers)), 0, stream, streams, entries, group_s,
                       ngroups, queue, status);
    return hipGetLastError();
}

template <int W, bool FIRE, int D>
uint32_t batch_grid_cap() {
    // resident workgroups of this kernel on the current device (1 if the query
    // fails), cached per device
    static std::mutex mu;
    static std::map<int, uint32_t> cache;
    int per_cu = 0, dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(dev);
        if (it != cache.end()) return it->second;
    }
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, (const void *)spz::k_decode_pc_batch<W, FIRE, D, spz::kPcProducers, spz::kPcConsumers>,
            spz::pc_threads(spz::kPcProducers, spz::kPcConsumers), 0) != hipSuccess)
        return 1;
    const uint32_t cap = (uint32_t)(per_cu > 0 ? per_cu : 1) * (uint32_t)(cus > 0 ? cus : 1);
    std::lock_guard<std::mutex> lk(mu);
    cache[dev] = cap;
    return cap;
}

}  // namespace

struct spz_batch {
    uint32_t n;
    void *dmem;                                    // device tables: own allocation, or the caller's workspace
    bool owns;                                     // dmem allocated by the library
    std::vector<uint8_t> host;                     // host image of the tables (kept for asynchronous uploads)
    spz::PcStream *streams;
    uint64_t *entries[kClasses];
    uint32_t *group_s[kClasses];
    uint32_t ngroups[kClasses];
    uint32_t grid[kClasses];
    uint32_t *queues;                              // one work counter per class
    double work[kClasses];                         // launch order weight per class
    Lanes lanes;
    // entropy-coded items: one Huffman decode job each, decoded by one batched
    // launch into plain containers in the plan's workspace (past the tables)
    spz::HufJob *hjobs;
    uint64_t *hentries;                            // job << 32 | segment
    uint32_t nhent;
    size_t img_off, total;                         // workspace: plain containers, then the tables at img_off
    // streams that take the single-container path
    struct Fallback { const void *src; void *dst; spz_info info; spz::Geom g; uint32_t index; };
    Fallback *fallback;
    uint32_t nfallback;
};

extern "C" {

size_t sprintz_decompress_workspace_size(const spz_info *info) {
    if (!info || info->params.entropy != 1 || (info->w != 8 && info->w != 16)) return 0;
    return align16(kHeader + 8 * (size_t)(info->nseg + 1)) +
           (size_t)(info->nseg * plain_segment_max(info->rows, info->D, info->w, &info->params));
}

spz_status sprintz_decompress_ws(const void *d_src, size_t src_size, const spz_info *info, void *d_dst,
                                 size_t dst_cap, int32_t *d_status, void *d_ws, size_t ws_size, hipStream_t stream) {
    spz::Geom g;
    const spz_status st = check_decompress(d_src, src_size, info, d_dst, dst_cap, &g);
    if (st != SPZ_OK) return st;
    if (info->params.entropy == 0) return launch_decode_any(d_src, info, g, d_dst, d_status, stream) == hipSuccess ? SPZ_OK : SPZ_EHIP;
    if (!d_ws || ((uintptr_t)d_ws & 15) || ws_size < sprintz_decompress_workspace_size(info)) return SPZ_ENOSPC;
    if (info->nseg == 0) return SPZ_OK;
    // Huffman-decode every segment into a plain container at a fixed
    // segment stride, then decode that container
    const uint64_t stride = plain_segment_max(info->rows, info->D, info->w, &info->params);
    uint8_t *ws = (uint8_t *)d_ws;
    hipLaunchKernelGGL(spz::k_huff_plain_table, dim3((info->nseg + 1 + 255) / 256), dim3(256), 0, stream,
                       (const uint8_t *)d_src, info->nseg, stride, ws);
    hipLaunchKernelGGL(spz::k_huff_decode, dim3((info->nseg + spz::kHufSegsPerWave - 1) / spz::kHufSegsPerWave),
                       dim3(64), 0, stream, (const uint8_t *)d_src, (uint64_t)src_size, g.data_start, g.data_bytes,
                       info->nseg, ws, stride, d_status);
    spz_info pi = *info;
    pi.params.entropy = 0;
    pi.compressed_size = g.data_start + stride * info->nseg;
    spz::Geom pg = g;
    pg.cap = ws_size;
    pg.data_bytes = stride * info->nseg;
    return launch_decode_any(ws, &pi, pg, d_dst, d_status, stream) == hipSuccess ? SPZ_OK : SPZ_EHIP;
}

spz_status sprintz_decompress(const void *d_src, size_t src_size, const spz_info *info, void *d_dst,
                              size_t dst_cap, int32_t *d_status, hipStream_t stream) {
    spz::Geom g;
    const spz_status st = check_decompress(d_src, src_size, info, d_dst, dst_cap, &g);
    if (st != SPZ_OK) return st;
    if (info->params.entropy == 0)
        return launch_decode_any(d_src, info, g, d_dst, d_status, stream) == hipSuccess ? SPZ_OK : SPZ_EHIP;
    // entropy-coded: a stream-ordered workspace for the plain container
    const size_t wsz = sprintz_decompress_workspace_size(info);
    void *ws = nullptr;
    if (hipMallocAsync(&ws, wsz, stream) != hipSuccess) return SPZ_ENOMEM;
    const spz_status r = sprintz_decompress_ws(d_src, src_size, info, d_dst, dst_cap, d_status, ws, wsz, stream);
    if (hipFreeAsync(ws, stream) != hipSuccess) return SPZ_EHIP;
    return r;
}

}  // extern "C"

namespace {

// Builds the plan's tables on the host (b->host) and the pointers into them
// relative to device address `base` (nullptr: offsets only, for sizing).
spz_status build_plan(const spz_batch_item *items, const spz_info *infos, uint32_t n, spz_batch *b, uint8_t *base) {
    b->n = n;
    std::vector<spz::Geom> geoms(n);
    std::vector<int> cls(n, -1);
    // entropy-coded items decode from a plain container in the workspace:
    // their plain geometry and stride, and the coded container's geometry
    std::vector<spz::Geom> cgeoms(n);
    std::vector<uint64_t> pstride(n, 0);
    std::vector<spz_info> pinfo(infos, infos + n);
    for (uint32_t i = 0; i < n; ++i) {
        const spz_status st =
            check_decompress(items[i].d_src, items[i].src_size, &infos[i], items[i].d_dst, items[i].dst_cap, &geoms[i]);
        if (st != SPZ_OK) return st;
        const spz_info &in = infos[i];
        if (in.params.entropy > 1) return SPZ_EUNSUPPORTED;
        if (in.params.entropy == 1 && in.nseg > 0) {
            cgeoms[i] = geoms[i];
            pstride[i] = plain_segment_max(in.rows, in.D, in.w, &in.params);
            pinfo[i].params.entropy = 0;
            pinfo[i].compressed_size = geoms[i].data_start + pstride[i] * in.nseg;
            geoms[i].data_bytes = pstride[i] * in.nseg;
            geoms[i].cap = pinfo[i].compressed_size;
        }
        const uint32_t D = in.D;
        if (D >= 1 && D <= 16 && in.params.hdr_group == 0 && !((uintptr_t)items[i].d_dst & 15) &&
            ((uint64_t)in.params.seg_rows * D * (in.w / 8)) % 16 == 0 && in.nseg > 0)
            cls[i] = class_of(in.w, in.params.forecaster == SPZ_FIRE, D);
    }
    // work lists: per class, streams ordered by seg_rows so that a group of
    // segments never mixes two seg_rows; a group holds one workgroup's segments
    std::vector<std::vector<uint64_t>> ent(kClasses);
    std::vector<std::vector<uint32_t>> gs(kClasses);
    std::vector<uint32_t> order(n);
    for (uint32_t i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) {
        return infos[x].params.seg_rows < infos[y].params.seg_rows;
    });
    // the plain containers of entropy-coded items come first in the
    // workspace, the tables after them
    std::vector<size_t> poff(n, 0);
    size_t P = 0;
    uint32_t njobs = 0;
    uint64_t nhent = 0;
    for (uint32_t i = 0; i < n; ++i) {
        if (!pstride[i]) continue;
        poff[i] = P;
        P += align256(pinfo[i].compressed_size);
        ++njobs;
        nhent += infos[i].nseg;
    }
    if (nhent > 0xFFFFFFFFull) return SPZ_EUNSUPPORTED;
    auto srcof = [&](uint32_t i) -> const void * { return pstride[i] ? (const void *)(base + poff[i]) : items[i].d_src; };
    std::vector<spz_batch::Fallback> fb;
    for (uint32_t oi = 0; oi < n; ++oi) {
        const uint32_t i = order[oi];
        if (cls[i] < 0) {
            if (infos[i].rows > 0) fb.push_back({srcof(i), items[i].d_dst, pinfo[i], geoms[i], i});
            continue;
        }
        const int c = cls[i];
        const uint32_t spw = spz::pc_spw(class_D(c), spz::kPcProducers, spz::kPcConsumers);
        const uint32_t S = infos[i].params.seg_rows;
        for (uint32_t sg = 0; sg < infos[i].nseg; ++sg) {
            if (ent[c].size() % spw == 0 || gs[c].back() != S) {
                while (ent[c].size() % spw) ent[c].push_back(~0ull);
                gs[c].push_back(S);
            }
            ent[c].push_back(((uint64_t)i << 32) | sg);
        }
    }
    size_t bytes = sizeof(spz::PcStream) * (size_t)n + 16 + sizeof(uint32_t) * kClasses + 16 +
                   sizeof(spz::HufJob) * njobs + 16 + 8 * (size_t)nhent + 16;
    for (int c = 0; c < kClasses; ++c) {
        const uint32_t spw = spz::pc_spw(class_D(c), spz::kPcProducers, spz::kPcConsumers);
        while (ent[c].size() % spw) ent[c].push_back(~0ull);
        bytes += ent[c].size() * 8 + gs[c].size() * 4 + 16;
    }
    b->host.assign(bytes, 0);
    std::vector<uint8_t> &host = b->host;
    size_t off = 0;
    auto carve = [&](size_t sz) { const size_t o = off; off = (off + sz + 15) & ~size_t(15); return o; };
    const size_t o_streams = carve(sizeof(spz::PcStream) * (size_t)n);
    spz::PcStream *hs = reinterpret_cast<spz::PcStream *>(host.data() + o_streams);
    for (uint32_t i = 0; i < n; ++i) {
        const spz_info &in = infos[i];
        const spz::Geom &g = geoms[i];
        spz::PcStream &st = hs[i];
        st.src = (const uint8_t *)srcof(i);
        st.dst = (uint8_t *)items[i].d_dst;
        st.data_start = g.data_start;
        st.data_bytes = g.data_bytes;
        st.rows = in.rows;
        st.nseg = in.nseg;
        st.S = in.params.seg_rows;
        st.sh = g.sh;
        st.acc_lo = g.acc_lo;
        st.acc_hi = g.acc_hi;
        st.pad = 0;
    }
    size_t o_ent[kClasses], o_gs[kClasses];
    for (int c = 0; c < kClasses; ++c) {
        o_ent[c] = carve(ent[c].size() * 8);
        if (!ent[c].empty()) memcpy(host.data() + o_ent[c], ent[c].data(), ent[c].size() * 8);
        o_gs[c] = carve(gs[c].size() * 4);
        if (!gs[c].empty()) memcpy(host.data() + o_gs[c], gs[c].data(), gs[c].size() * 4);
    }
    const size_t o_q = carve(sizeof(uint32_t) * kClasses);
    const size_t o_jobs = carve(sizeof(spz::HufJob) * njobs);
    const size_t o_hent = carve(8 * (size_t)nhent);
    {
        spz::HufJob *hj = reinterpret_cast<spz::HufJob *>(host.data() + o_jobs);
        uint64_t *he = reinterpret_cast<uint64_t *>(host.data() + o_hent);
        uint32_t j = 0;
        uint64_t q = 0;
        for (uint32_t i = 0; i < n; ++i) {
            if (!pstride[i]) continue;
            spz::HufJob &job = hj[j];
            job.src = (const uint8_t *)items[i].d_src;
            job.plain = base + poff[i];
            job.src_size = items[i].src_size;
            job.data_start = cgeoms[i].data_start;
            job.data_bytes = cgeoms[i].data_bytes;
            job.stride = pstride[i];
            job.nseg = infos[i].nseg;
            job.table = 1;
            job.status = i;
            job.pad = 0;
            for (uint32_t sg = 0; sg < infos[i].nseg; ++sg) he[q++] = ((uint64_t)j << 32) | sg;
            ++j;
        }
    }
    uint8_t *const tb = base + P;   // the tables, after the plain containers
    b->img_off = P;
    b->total = P + host.size();
    b->hjobs = (spz::HufJob *)(tb + o_jobs);
    b->hentries = (uint64_t *)(tb + o_hent);
    b->nhent = (uint32_t)nhent;
    b->streams = (spz::PcStream *)(tb + o_streams);
    b->queues = (uint32_t *)(tb + o_q);
    for (int c = 0; c < kClasses; ++c) {
        b->entries[c] = (uint64_t *)(tb + o_ent[c]);
        b->group_s[c] = (uint32_t *)(tb + o_gs[c]);
        b->ngroups[c] = (uint32_t)gs[c].size();
        uint32_t cap = 1;
#define SPZ_CAP(W_, F_, D_) if (class_w(c) == W_ && class_fire(c) == F_ && class_D(c) == D_) cap = batch_grid_cap<W_, F_, D_>();
#define SPZ_CAPD(W_, F_)                                                                                \
    SPZ_CAP(W_, F_, 1) SPZ_CAP(W_, F_, 2) SPZ_CAP(W_, F_, 3) SPZ_CAP(W_, F_, 4) SPZ_CAP(W_, F_, 5) SPZ_CAP(W_, F_, 6)   \
    SPZ_CAP(W_, F_, 7) SPZ_CAP(W_, F_, 8) SPZ_CAP(W_, F_, 9) SPZ_CAP(W_, F_, 10) SPZ_CAP(W_, F_, 11)               \
    SPZ_CAP(W_, F_, 12) SPZ_CAP(W_, F_, 13) SPZ_CAP(W_, F_, 14) SPZ_CAP(W_, F_, 15) SPZ_CAP(W_, F_, 16)
        if (b->ngroups[c]) { SPZ_CAPD(8, false) SPZ_CAPD(8, true) SPZ_CAPD(16, false) SPZ_CAPD(16, true) }
#undef SPZ_CAPD
#undef SPZ_CAP
        b->grid[c] = std::min(b->ngroups[c], cap);
        double wk = 0;
        for (uint32_t gi = 0; gi < gs[c].size(); ++gi) wk += (double)gs[c][gi];
        b->work[c] = wk * spz::pc_spw(class_D(c), spz::kPcProducers, spz::kPcConsumers) * (class_D(c) + 4.0);
    }
    b->nfallback = (uint32_t)fb.size();
    b->fallback = nullptr;
    if (!fb.empty()) {
        b->fallback = new (std::nothrow) spz_batch::Fallback[fb.size()];
        if (!b->fallback) return SPZ_ENOMEM;
        std::copy(fb.begin(), fb.end(), b->fallback);
    }
    return SPZ_OK;
}

}  // namespace

extern "C" {

size_t sprintz_batch_workspace_size(const spz_batch_item *items, const spz_info *infos, uint32_t n) {
    if (n > 0 && (!items || !infos)) return 0;
    spz_batch b{};
    if (build_plan(items, infos, n, &b, nullptr) != SPZ_OK) { delete[] b.fallback; return 0; }
    delete[] b.fallback;
    return b.total;
}

spz_status sprintz_batch_create(const spz_batch_item *items, const spz_info *infos, uint32_t n, spz_batch **out) {
    if (!out || (n > 0 && (!items || !infos))) return SPZ_EINVAL;
    *out = nullptr;
    spz_batch *b = new (std::nothrow) spz_batch();
    if (!b) return SPZ_ENOMEM;
    spz_status st = build_plan(items, infos, n, b, nullptr);   // size first
    if (st != SPZ_OK) { delete[] b->fallback; delete b; return st; }
    delete[] b->fallback;
    b->fallback = nullptr;
    if (hipMalloc(&b->dmem, b->total) != hipSuccess) { delete b; return SPZ_ENOMEM; }
    b->owns = true;
    st = build_plan(items, infos, n, b, (uint8_t *)b->dmem);
    if (st == SPZ_OK && hipMemcpy((uint8_t *)b->dmem + b->img_off, b->host.data(), b->host.size(),
                                  hipMemcpyHostToDevice) != hipSuccess)
        st = SPZ_EHIP;
    if (st == SPZ_OK && b->lanes.create() != hipSuccess) st = SPZ_EHIP;
    if (st != SPZ_OK) { b->lanes.destroy(); (void)hipFree(b->dmem); delete[] b->fallback; delete b; return st; }
    *out = b;
    return SPZ_OK;
}

spz_status sprintz_batch_create_in(const spz_batch_item *items, const spz_info *infos, uint32_t n, void *d_ws,
                                   size_t ws_size, hipStream_t stream, spz_batch **out) {
    if (!out || (n > 0 && (!items || !infos)) || !d_ws || ((uintptr_t)d_ws & 15)) return SPZ_EINVAL;
    *out = nullptr;
    spz_batch *b = new (std::nothrow) spz_batch();
    if (!b) return SPZ_ENOMEM;
    spz_status st = build_plan(items, infos, n, b, (uint8_t *)d_ws);
    if (st == SPZ_OK && b->total > ws_size) st = SPZ_ENOSPC;
    if (st == SPZ_OK && hipMemcpyAsync((uint8_t *)d_ws + b->img_off, b->host.data(), b->host.size(),
                                       hipMemcpyHostToDevice, stream) != hipSuccess)
        st = SPZ_EHIP;
    if (st == SPZ_OK && b->lanes.create() != hipSuccess) st = SPZ_EHIP;
    if (st != SPZ_OK) { b->lanes.destroy(); delete[] b->fallback; delete b; return st; }
    b->dmem = d_ws;
    b->owns = false;
    *out = b;
    return SPZ_OK;
}


spz_status sprintz_batch_decompress(const spz_batch *b, int32_t *d_status, hipStream_t stream) {
    if (!b) return SPZ_EINVAL;
    hipLaunchKernelGGL(spz::k_zero_u32, dim3(1), dim3(64), 0, stream, b->queues, (uint32_t)kClasses);
    // entropy-coded items: every segment Huffman-decoded into its plain
    // container (and the containers' tables written) in one launch
    if (b->nhent)
        hipLaunchKernelGGL(spz::k_huff_decode_batch, dim3((b->nhent + spz::kHufSegsPerWave - 1) / spz::kHufSegsPerWave),
                           dim3(64), 0, stream, b->hjobs, b->hentries, b->nhent, d_status);
    int order[kClasses];
    const int ncls = lane_order(b->ngroups, [&](int c) { return b->work[c]; }, order);
    const int used = std::min(ncls, kLanes);
    hipStream_t ls[kLanes];
    if (b->lanes.begin(stream, used, ls) != hipSuccess) return SPZ_EHIP;
    for (int oi = 0; oi < ncls; ++oi) {
        const int c = order[oi];
        hipStream_t cs = ls[oi % used];
        hipError_t e = hipSuccess;
#define SPZ_BL(W_, F_, D_)                                                                                      \
    if (class_w(c) == W_ && class_fire(c) == F_ && class_D(c) == D_)                                            \
        e = launch_batch_class<W_, F_, D_>(b->streams, b->entries[c], b->group_s[c], b->ngroups[c], b->queues + c, \
                                           d_status, b->grid[c], cs);
#define SPZ_BLD(W_, F_)                                                                                   \
    SPZ_BL(W_, F_, 1) SPZ_BL(W_, F_, 2) SPZ_BL(W_, F_, 3) SPZ_BL(W_, F_, 4) SPZ_BL(W_, F_, 5) SPZ_BL(W_, F_, 6)         \
    SPZ_BL(W_, F_, 7) SPZ_BL(W_, F_, 8) SPZ_BL(W_, F_, 9) SPZ_BL(W_, F_, 10) SPZ_BL(W_, F_, 11)                     \
    SPZ_BL(W_, F_, 12) SPZ_BL(W_, F_, 13) SPZ_BL(W_, F_, 14) SPZ_BL(W_, F_, 15) SPZ_BL(W_, F_, 16)
        SPZ_BLD(8, false) SPZ_BLD(8, true) SPZ_BLD(16, false) SPZ_BLD(16, true)
#undef SPZ_BLD
#undef SPZ_BL
        if (e != hipSuccess) return SPZ_EHIP;
    }
    if (b->lanes.end(used, ls) != hipSuccess) return SPZ_EHIP;
    for (uint32_t k = 0; k < b->nfallback; ++k) {
        const spz_batch::Fallback &f = b->fallback[k];
        if (launch_decode_any(f.src, &f.info, f.g, f.dst, d_status ? d_status + f.index : nullptr, stream) != hipSuccess)
            return SPZ_EHIP;
    }
    return hipGetLastError() == hipSuccess ? SPZ_OK : SPZ_EHIP;
}

void sprintz_batch_destroy(spz_batch *b) {
    if (!b) return;
    b->lanes.destroy();
    if (b->owns) (void)hipFree(b->dmem);
    delete[] b->fallback;
    delete b;
}

}  // extern "C"

// ---- Batched compression ------------------------------------------------------

struct spz_cbatch {
    uint32_t n;
    std::vector<uint8_t> host;                     // image of the device tables (kept for the upload)
    spz::EsStream *streams;                        // batched series
    uint2 *groups[kClasses];                       // per class: (series, first segment)
    uint32_t ngroups[kClasses], grid[kClasses];
    uint32_t *queues;
    uint32_t *scan_list;                           // batched series, one scan workgroup each
    uint32_t nscan;
    uint4 *cgroups;                                // compaction groups (series, first segment, count)
    uint32_t ncgroups;
    struct Fallback { spz_compress_item item; void *ws; size_t ws_size; uint32_t index; };
    std::vector<Fallback> fallback;                // series the batched kernels do not take
    double work[kClasses];                         // launch order weight per class
    Lanes lanes;
    ~spz_cbatch() { lanes.destroy(); }
};

namespace {

template <int W, bool FIRE, int D>
uint32_t cbatch_grid_cap() {
    static std::mutex mu;
    static std::map<int, uint32_t> cache;
    int per_cu = 0, dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(dev);
        if (it != cache.end()) return it->second;
    }
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)spz::k_encode_sp_batch<W, FIRE, D>,
                                                     spz::es_threads(D), 0) != hipSuccess)
        return 1;
    const uint32_t cap = (uint32_t)(per_cu > 0 ? per_cu : 1) * (uint32_t)(cus > 0 ? cus : 1);
    std::lock_guard<std::mutex> lk(mu);
    cache[dev] = cap;
    return cap;
}

spz_status check_compress_item(const spz_compress_item &it) {
    const spz_dtype dt = (spz_dtype)it.dtype;
    const uint32_t w = bits_of(dt);
    if (w == 0 || it.D == 0) return SPZ_EINVAL;
    spz_status st = check_params(&it.params);   // seg_rows 0 is not taken: tune first
    if (st != SPZ_OK) return st;
    if (it.D > kMaxD) return SPZ_EUNSUPPORTED;
    if (num_segments(it.rows, it.params.seg_rows) > 0xFFFFFFFFull) return SPZ_EUNSUPPORTED;
    if (!it.d_dst || !it.d_out_size || (it.rows > 0 && !it.d_src)) return SPZ_EINVAL;
    if (((uintptr_t)it.d_dst & 15) || ((uintptr_t)it.d_src & (w / 8 - 1)) || ((uintptr_t)it.d_out_size & 7))
        return SPZ_EINVAL;
    if (it.dst_cap < sprintz_compress_bound(it.rows, it.D, dt, &it.params)) return SPZ_ENOSPC;
    if (!it.d_ws || ((uintptr_t)it.d_ws & 15)) return SPZ_EINVAL;
    if (it.ws_size < sprintz_workspace_size_min(it.rows, it.D, dt, &it.params)) return SPZ_ENOSPC;
    return SPZ_OK;
}

bool cbatch_takes(const spz_compress_item &it) {
    const uint32_t w = bits_of((spz_dtype)it.dtype);
    return it.params.entropy == 0 && it.params.hdr_group == 0 && it.D >= 1 && it.D <= 16 && it.rows > 0 &&
           !((uintptr_t)it.d_src & 15) && ((uint64_t)it.params.seg_rows * it.D * (w / 8)) % 16 == 0 &&
           it.ws_size >= sp_workspace_bytes(num_segments(it.rows, it.params.seg_rows), it.params.seg_rows, it.D, w);
}

// Builds the plan's tables (b->host) with pointers relative to the device
// address `base`; returns their bytes in *total. Every series codes into its
// own workspace.
spz_status build_cplan(const spz_compress_item *items, uint32_t n, spz_cbatch *b, uint8_t *base, size_t *total) {
    b->n = n;
    for (int c = 0; c < kClasses; ++c) b->work[c] = 0;
    std::vector<int> cls(n, -1);
    uint32_t nb = 0;
    for (uint32_t i = 0; i < n; ++i) {
        const spz_status st = check_compress_item(items[i]);
        if (st != SPZ_OK) return st;
        if (cbatch_takes(items[i])) {
            cls[i] = class_of(bits_of((spz_dtype)items[i].dtype), items[i].params.forecaster == SPZ_FIRE, items[i].D);
            ++nb;
        }
    }
    std::vector<std::vector<uint2>> grp(kClasses);
    std::vector<uint4> cg;
    std::vector<uint32_t> scan;
    std::vector<uint32_t> sidx(n, ~0u);
    uint32_t k = 0;
    for (uint32_t i = 0; i < n; ++i) {
        if (cls[i] < 0) continue;
        sidx[i] = k;
        const uint32_t D = items[i].D, S = items[i].params.seg_rows, w = bits_of((spz_dtype)items[i].dtype);
        const uint32_t nseg = (uint32_t)num_segments(items[i].rows, S);
        const uint32_t spw = 64 / spz::pc_pow2(D);
        for (uint32_t s0 = 0; s0 < nseg; s0 += spw) grp[cls[i]].push_back(make_uint2(k, s0));
        b->work[cls[i]] += (double)items[i].rows * (D + 4.0);
        const uint64_t units = sp_slot_stride(S, D, w) / 16;
        const uint32_t K = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(256, 2048 / units));
        for (uint32_t s0 = 0; s0 < nseg; s0 += K) cg.push_back(make_uint4(k, s0, K, 0));
        scan.push_back(k);
        ++k;
    }
    size_t off = 0;
    auto carve = [&](size_t sz) { const size_t o = off; off = (off + sz + 255) & ~size_t(255); return o; };
    const size_t o_streams = carve(sizeof(spz::EsStream) * (size_t)nb);
    size_t o_grp[kClasses];
    for (int c = 0; c < kClasses; ++c) o_grp[c] = carve(grp[c].size() * sizeof(uint2));
    const size_t o_q = carve(sizeof(uint32_t) * kClasses);
    const size_t o_scan = carve(scan.size() * sizeof(uint32_t));
    const size_t o_cg = carve(cg.size() * sizeof(uint4));
    b->host.assign(off, 0);
    // per-series workspace regions after the tables
    spz::EsStream *hs = reinterpret_cast<spz::EsStream *>(b->host.data() + o_streams);
    b->fallback.clear();
    for (uint32_t i = 0; i < n; ++i) {
        const spz_compress_item &it = items[i];
        const uint32_t w = bits_of((spz_dtype)it.dtype);
        if (cls[i] < 0) {
            b->fallback.push_back({it, it.d_ws, it.ws_size, i});
            continue;
        }
        const uint32_t S = it.params.seg_rows;
        spz::EsStream &st = hs[sidx[i]];
        const spz::Geom g = make_geom(it.rows, it.D, w, S, 0, it.params.learn_shift);
        st.src = (const uint8_t *)it.d_src;
        st.dst = (uint8_t *)it.d_dst;
        st.out_size = it.d_out_size;
        st.rows = it.rows;
        st.cap = it.dst_cap;
        st.data_start = g.data_start;
        st.slot_stride = sp_slot_stride(S, it.D, w);
        st.D = it.D; st.S = S; st.nseg = g.nseg; st.w = w; st.dtype = it.dtype;
        st.forecaster = it.params.forecaster; st.learn_shift = it.params.learn_shift; st.sh = g.sh;
        st.acc_lo = g.acc_lo; st.acc_hi = g.acc_hi;
        st.status = i; st.pad = 0;
        st.info = reinterpret_cast<spz::u32x4 *>(it.d_ws);
        st.slots = (uint8_t *)it.d_ws + align256(16 * (size_t)g.nseg);
    }
    *total = off;
    for (int c = 0; c < kClasses; ++c)
        if (!grp[c].empty()) memcpy(b->host.data() + o_grp[c], grp[c].data(), grp[c].size() * sizeof(uint2));
    if (!scan.empty()) memcpy(b->host.data() + o_scan, scan.data(), scan.size() * sizeof(uint32_t));
    if (!cg.empty()) memcpy(b->host.data() + o_cg, cg.data(), cg.size() * sizeof(uint4));
    b->streams = reinterpret_cast<spz::EsStream *>(base + o_streams);
    b->queues = reinterpret_cast<uint32_t *>(base + o_q);
    b->scan_list = reinterpret_cast<uint32_t *>(base + o_scan);
    b->nscan = (uint32_t)scan.size();
    b->cgroups = reinterpret_cast<uint4 *>(base + o_cg);
    b->ncgroups = (uint32_t)cg.size();
    for (int c = 0; c < kClasses; ++c) {
        b->groups[c] = reinterpret_cast<uint2 *>(base + o_grp[c]);
        b->ngroups[c] = (uint32_t)grp[c].size();
        uint32_t cap = 1;
        if (b->ngroups[c] && base) {
#define SPZ_CCAP(W_, F_, D_) if (class_w(c) == W_ && class_fire(c) == F_ && class_D(c) == D_) cap = cbatch_grid_cap<W_, F_, D_>();
#define SPZ_CCAPD(W_, F_)                                                                                        \
    SPZ_CCAP(W_, F_, 1) SPZ_CCAP(W_, F_, 2) SPZ_CCAP(W_, F_, 3) SPZ_CCAP(W_, F_, 4) SPZ_CCAP(W_, F_, 5)            \
    SPZ_CCAP(W_, F_, 6) SPZ_CCAP(W_, F_, 7) SPZ_CCAP(W_, F_, 8) SPZ_CCAP(W_, F_, 9) SPZ_CCAP(W_, F_, 10)           \
    SPZ_CCAP(W_, F_, 11) SPZ_CCAP(W_, F_, 12) SPZ_CCAP(W_, F_, 13) SPZ_CCAP(W_, F_, 14) SPZ_CCAP(W_, F_, 15)       \
    SPZ_CCAP(W_, F_, 16)
            SPZ_CCAPD(8, false) SPZ_CCAPD(8, true) SPZ_CCAPD(16, false) SPZ_CCAPD(16, true)
#undef SPZ_CCAPD
#undef SPZ_CCAP
        }
        b->grid[c] = std::min(b->ngroups[c], cap);
    }
    return SPZ_OK;
}

}  // namespace

extern "C" {

size_t sprintz_compress_batch_workspace_size(const spz_compress_item *items, uint32_t n) {
    if (n > 0 && !items) return 0;
    spz_cbatch b{};
    size_t total = 0;
    if (build_cplan(items, n, &b, nullptr, &total) != SPZ_OK) return 0;
    return std::max<size_t>(total, 256);
}

spz_status sprintz_compress_batch_create_in(const spz_compress_item *items, uint32_t n, void *d_ws, size_t ws_size,
                                            hipStream_t stream, spz_cbatch **out) {
    if (!out || (n > 0 && !items) || !d_ws || ((uintptr_t)d_ws & 255)) return SPZ_EINVAL;
    *out = nullptr;
    spz_cbatch *b = new (std::nothrow) spz_cbatch();
    if (!b) return SPZ_ENOMEM;
    size_t total = 0;
    spz_status st = build_cplan(items, n, b, (uint8_t *)d_ws, &total);
    if (st == SPZ_OK && total > ws_size) st = SPZ_ENOSPC;
    if (st == SPZ_OK && !b->host.empty() &&
        hipMemcpyAsync(d_ws, b->host.data(), b->host.size(), hipMemcpyHostToDevice, stream) != hipSuccess)
        st = SPZ_EHIP;
    if (st == SPZ_OK && b->lanes.create() != hipSuccess) st = SPZ_EHIP;
    if (st != SPZ_OK) { delete b; return st; }
    *out = b;
    return SPZ_OK;
}

spz_status sprintz_compress_batch(const spz_cbatch *b, int32_t *d_status, hipStream_t stream) {
    if (!b) return SPZ_EINVAL;
    hipLaunchKernelGGL(spz::k_zero_u32, dim3(1), dim3(64), 0, stream, b->queues, (uint32_t)kClasses);
    int order[kClasses];
    const int ncls = lane_order(b->ngroups, [&](int c) { return b->work[c]; }, order);
    const int used = std::min(ncls, kLanes);
    hipStream_t ls[kLanes];
    if (b->lanes.begin(stream, used, ls) != hipSuccess) return SPZ_EHIP;
    for (int oi = 0; oi < ncls; ++oi) {
        const int c = order[oi];
        hipStream_t cs = ls[oi % used];
#define SPZ_CBL(W_, F_, D_)                                                                                      \
    if (class_w(c) == W_ && class_fire(c) == F_ && class_D(c) == D_)                                             \
        hipLaunchKernelGGL((spz::k_encode_sp_batch<W_, F_, D_>), dim3(b->grid[c]), dim3(spz::es_threads(D_)), 0, \
                           cs, b->streams, b->groups[c], b->ngroups[c], b->queues + c);
#define SPZ_CBLD(W_, F_)                                                                                  \
    SPZ_CBL(W_, F_, 1) SPZ_CBL(W_, F_, 2) SPZ_CBL(W_, F_, 3) SPZ_CBL(W_, F_, 4) SPZ_CBL(W_, F_, 5)          \
    SPZ_CBL(W_, F_, 6) SPZ_CBL(W_, F_, 7) SPZ_CBL(W_, F_, 8) SPZ_CBL(W_, F_, 9) SPZ_CBL(W_, F_, 10)         \
    SPZ_CBL(W_, F_, 11) SPZ_CBL(W_, F_, 12) SPZ_CBL(W_, F_, 13) SPZ_CBL(W_, F_, 14) SPZ_CBL(W_, F_, 15)     \
    SPZ_CBL(W_, F_, 16)
        SPZ_CBLD(8, false) SPZ_CBLD(8, true) SPZ_CBLD(16, false) SPZ_CBLD(16, true)
#undef SPZ_CBLD
#undef SPZ_CBL
    }
    if (b->lanes.end(used, ls) != hipSuccess) return SPZ_EHIP;
    if (b->nscan) hipLaunchKernelGGL(spz::k_enc_scan_batch, dim3(b->nscan), dim3(256), 0, stream, b->streams,
                                     b->scan_list, d_status);
    if (b->ncgroups) hipLaunchKernelGGL(spz::k_enc_compact_batch, dim3(b->ncgroups), dim3(256), 0, stream, b->streams,
                                        b->cgroups, d_status);
    for (const spz_cbatch::Fallback &f : b->fallback) {
        const spz_compress_item &it = f.item;
        const spz_status st = sprintz_compress(it.d_src, it.rows, it.D, (spz_dtype)it.dtype, &it.params, it.d_dst,
                                               it.dst_cap, it.d_out_size, f.ws, f.ws_size,
                                               d_status ? d_status + f.index : nullptr, stream);
        if (st != SPZ_OK) return st;
    }
    return hipGetLastError() == hipSuccess ? SPZ_OK : SPZ_EHIP;
}

void sprintz_compress_batch_destroy(spz_cbatch *b) { delete b; }

const char *sprintz_strerror(spz_status s) {
    switch (s) {
        case SPZ_OK: return "ok";
        case SPZ_EINVAL: return "invalid argument";
        case SPZ_ENOSPC: return "destination or workspace too small";
        case SPZ_ECORRUPT: return "corrupt container header";
        case SPZ_EUNSUPPORTED: return "outside the GPU limits (D <= 128)";
        case SPZ_EHIP: return "HIP runtime error";
        case SPZ_ENOMEM: return "out of memory";
        default: return "unknown status";
    }
}

int sprintz_format_version(void) { return 1; }

}  // extern "C"

// Entropy stage of the gfx950 Sprintz codec: Huffman coding of every
// segment's packed bytes.
//
// Paper: Section 4.4 closes the pipeline with a byte-oriented Huffman coder
// run over the bit-packed headers and payloads (bytes are the symbols,
// whatever the data's bit width). The coder and its byte format are this
// library's own (the paper uses an external coder):
//   - one code per segment, from the byte counts of the plain segment;
//   - code lengths by the two-queue Huffman construction over the present
//     byte values in (count, value) order, a leaf taken before an internal
//     node of equal weight; if a length exceeds 11 bits every count c becomes
//     (c + 1) / 2 and the construction runs again; a lone value gets length 1;
//   - canonical codes in (length, value) order;
//   - 16 sub-streams per segment, sub-stream k coding plain bytes
//     [k n/16, (k+1) n/16) as a byte-aligned LSB-first bit string, every code
//     stored from its first (most significant) bit on.
// Coded segment: u32 n | u8 len[128] (4 bits per value, even values low) |
// u32 size[16] | the 16 sub-streams | zero pad to 16 bytes.
//
// Compression runs the plain encoder into a workspace container, then
//   k_huff_size   one wavefront per segment: byte histogram, code
//                 lengths, sub-stream bits from a second pass, coded size
//   k_huff_scan   offsets of the coded segments, container header
//   k_huff_write  one workgroup per segment: canonical codes, every byte's
//                 code OR-ed into an LDS image of the coded segment at its
//                 bit offset (scans over the byte ranges), 16-byte stores;
//                 a coded segment larger than the LDS image is OR-ed into
//                 its (cleared) place in the container directly.
// Decompression runs
//   k_huff_decode one wavefront per four segments, 16 lanes per segment: a
//                 2048-entry table (11-bit lookup) per segment in LDS, one
//                 sub-stream per lane read with aligned 16-byte loads kept
//                 four blocks ahead, plain bytes stored at a fixed stride
//   k_huff_plain_table  the workspace container's header and offset table,
// and then the plain decoder over the workspace container.
#pragma once

#include "spz_device.h"

namespace spz {

constexpr uint32_t kHufMaxLen = 11;
constexpr uint32_t kHufSub = 16;
constexpr uint32_t kHufFixed = 4 + 128 + 4 * kHufSub;   // n, lengths, sub-stream sizes
constexpr uint32_t kHufInfo = 256;                      // per-segment record in the encoder workspace
constexpr uint32_t kHufSegsPerWave = 4;                 // decoder: segments per wavefront

// Upper bound of a coded segment for a plain segment of n bytes.
__host__ __device__ inline uint64_t huff_segment_bound(uint64_t n) {
    return (kHufFixed + (n * kHufMaxLen + 7) / 8 + kHufSub + 15) & ~15ull;
}

__device__ __forceinline__ uint32_t huff_rev(uint32_t code, uint32_t len) {
    return __builtin_bitreverse32(code) >> (32 - len);
}

// ---- size pass -----------------------------------------------------------
// plain: plain container (offset table at +64, data at +data_start); info:
// kHufInfo bytes per segment: len nibbles [0,128), sub-stream bytes
// [128,192), coded segment bytes at 192.
__global__ __launch_bounds__(64) void k_huff_size(const uint8_t *__restrict__ plain, uint64_t data_start,
                                                  uint32_t nseg, uint8_t *__restrict__ info,
                                                  int32_t *__restrict__ status) {
    // One wavefront per segment, about 7 KB of LDS, so that many segments'
    // serial merges run on a CU at once. The four byte histograms (lanes
    // spread over them) become the merge's weights and parent links once
    // the counts are summed.
    __shared__ uint32_t hist[4 * 256];
    __shared__ u32x4 f4[64];                     // counts, four per entry
    __shared__ uint32_t order[256];
    __shared__ uint32_t len[256];
    __shared__ uint32_t sub_bits[kHufSub];
    __shared__ uint32_t nsym, maxlen;
    uint32_t *const weight = hist;               // [512], after the counts are summed
    uint32_t *const parent = hist + 512;         // [512]
    const uint32_t t = threadIdx.x, s = blockIdx.x;
    if (s >= nseg) return;
    const uint64_t a = gld64(plain + 64 + 8ull * s), b = gld64(plain + 64 + 8ull * (s + 1));
    const uint8_t *seg = plain + data_start + a;
    const uint32_t n = (uint32_t)(b - a);
    const uint32_t m16 = n / kHufSub;
    for (uint32_t k = t; k < 4 * 256; k += 64) hist[k] = 0;
    if (t < kHufSub) sub_bits[t] = 0;
    wave_sync();
    // byte histogram (16-byte loads)
    {
        uint32_t *const h = hist + 256 * (t & 3);
        for (uint32_t q = t; q < n / 16; q += 64) {
            const u32x4 v = gld128(seg + 16 * q);
            const uint32_t wds[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int i = 0; i < 16; ++i) atomicAdd(&h[(wds[i >> 2] >> (8 * (i & 3))) & 0xFFu], 1u);
        }
    }
    wave_sync();
    uint32_t *const f = reinterpret_cast<uint32_t *>(f4);
#pragma unroll
    for (uint32_t r = 0; r < 4; ++r) {
        const uint32_t v = t + 64 * r;
        f[v] = hist[v] + hist[256 + v] + hist[512 + v] + hist[768 + v];
    }
    wave_sync();
    // code lengths: two-queue construction, repeated on halved counts while
    // a length exceeds the limit; lane t holds values t, t+64, t+128, t+192
    uint32_t fv[4], rank[4], lv[4];
    for (;;) {
        if (t == 0) { nsym = 0; maxlen = 0; }
        wave_sync();
#pragma unroll
        for (uint32_t r = 0; r < 4; ++r) { fv[r] = f[t + 64 * r]; rank[r] = 0; }
        // rank by (count, value): 16-byte reads of all counts
        for (uint32_t u4 = 0; u4 < 64; ++u4) {
            const u32x4 c = f4[u4];
            const uint32_t fu[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
            for (uint32_t q = 0; q < 4; ++q) {
                const uint32_t u = 4 * u4 + q;
#pragma unroll
                for (uint32_t r = 0; r < 4; ++r) {
                    const uint32_t v = t + 64 * r;
                    rank[r] += (fu[q] != 0 && (fu[q] < fv[r] || (fu[q] == fv[r] && u < v))) ? 1u : 0u;
                }
            }
        }
#pragma unroll
        for (uint32_t r = 0; r < 4; ++r)
            if (fv[r]) { order[rank[r]] = t + 64 * r; atomicAdd(&nsym, 1u); }
        wave_sync();
        const uint32_t m = nsym;
        if (m == 1) {
#pragma unroll
            for (uint32_t r = 0; r < 4; ++r) { lv[r] = fv[r] ? 1u : 0u; len[t + 64 * r] = lv[r]; }
            wave_sync();
            break;
        }
        if (t == 0) {
            // serial two-queue merge; the next leaf's weight is read one
            // pick ahead and a fresh internal node is kept in a register
            for (uint32_t k = 0; k < m; ++k) weight[k] = f[order[k]];
            uint32_t leaf = 0, inner = m, next = m;
            uint32_t lw = weight[0];
            for (uint32_t step = 0; step + 1 < m; ++step) {
                uint32_t pick[2], wsum = 0;
                for (int q = 0; q < 2; ++q) {
                    const uint32_t iw = inner < next ? weight[inner] : 0u;
                    const bool use_leaf = leaf < m && (inner >= next || lw <= iw);
                    if (use_leaf) {
                        pick[q] = leaf++;
                        wsum += lw;
                        lw = leaf < m ? weight[leaf] : 0u;
                    } else {
                        pick[q] = inner++;
                        wsum += iw;
                    }
                }
                weight[next] = wsum;
                parent[pick[0]] = next;
                parent[pick[1]] = next;
                ++next;
            }
        }
        wave_sync();
        uint32_t dmax = 0;
#pragma unroll
        for (uint32_t r = 0; r < 4; ++r) {
            uint32_t d = 0;
            if (fv[r]) {
                const uint32_t root = 2 * m - 2;
                for (uint32_t q = rank[r]; q != root; q = parent[q]) ++d;
            }
            lv[r] = d;
            len[t + 64 * r] = d;
            dmax = max(dmax, d);
        }
        atomicMax(&maxlen, dmax);
        wave_sync();
        if (maxlen <= kHufMaxLen) break;
#pragma unroll
        for (uint32_t r = 0; r < 4; ++r) f[t + 64 * r] = (fv[r] + 1) >> 1;
        wave_sync();
    }
    // bits of every sub-stream: a second pass over the segment's bytes
    // (sub-stream k holds bytes [k m16, (k+1) m16))
    for (uint32_t q = t; q < n / 16; q += 64) {
        const u32x4 v = gld128(seg + 16 * q);
        const uint32_t wds[4] = {v.x, v.y, v.z, v.w};
        uint32_t pos = 16 * q, k = pos / m16, bits = 0;
#pragma unroll
        for (int i = 0; i < 16; ++i, ++pos) {
            if (pos >= (k + 1) * m16) {
                atomicAdd(&sub_bits[k], bits);
                bits = 0;
                while (pos >= (k + 1) * m16) ++k;
            }
            bits += len[(wds[i >> 2] >> (8 * (i & 3))) & 0xFFu];
        }
        atomicAdd(&sub_bits[min(k, kHufSub - 1)], bits);
    }
    wave_sync();
    uint8_t *rec = info + (uint64_t)s * kHufInfo;
#pragma unroll
    for (uint32_t r = 0; r < 2; ++r) {
        const uint32_t b2 = t + 64 * r;   // byte of the nibble table: values 2 b2 and 2 b2 + 1
        rec[b2] = (uint8_t)(len[2 * b2] | (len[2 * b2 + 1] << 4));
    }
    if (t < kHufSub) reinterpret_cast<uint32_t *>(rec + 128)[t] = (sub_bits[t] + 7) >> 3;
    if (t == 0) {
        uint32_t tot = kHufFixed;
        for (uint32_t k = 0; k < kHufSub; ++k) tot += (sub_bits[k] + 7) >> 3;
        reinterpret_cast<uint32_t *>(rec + 192)[0] = (tot + 15) & ~15u;
        if ((n % 16 || n == 0) && status) atomicOr(status, 2);
    }
}

// ---- offsets and header --------------------------------------------------
__global__ __launch_bounds__(1024) void k_huff_scan(const uint8_t *__restrict__ plain, uint32_t nseg,
                                                    uint64_t data_start, const uint8_t *__restrict__ info,
                                                    uint8_t *__restrict__ dst, uint64_t cap,
                                                    uint64_t *__restrict__ out_size, int32_t *__restrict__ status) {
    __shared__ uint64_t wsum[16];
    const uint32_t t = threadIdx.x, lane = t & 63, wv = t >> 6;
    uint64_t *tab = reinterpret_cast<uint64_t *>(dst + 64);
    uint64_t carry = 0;
    for (uint32_t base = 0; base < nseg; base += 1024) {
        const uint32_t k = base + t;
        const uint32_t v = k < nseg ? reinterpret_cast<const uint32_t *>(info + (uint64_t)k * kHufInfo + 192)[0] : 0u;
        uint64_t incl = v;
        for (uint32_t d = 1; d < 64; d <<= 1) {
            const uint64_t o = (uint64_t)__shfl_up((unsigned long long)incl, d, 64);
            if (lane >= d) incl += o;
        }
        if (lane == 63) wsum[wv] = incl;
        __syncthreads();
        uint64_t before = carry, total = carry;
        for (uint32_t q = 0; q < 16; ++q) {
            const uint64_t ws = wsum[q];
            if (q < wv) before += ws;
            total += ws;
        }
        if (k < nseg) tab[k] = before + incl - v;
        carry = total;
        __syncthreads();
    }
    if (t == 0) tab[nseg] = carry;
    if (t < 16) {
        // the plain header with entropy 1 and the coded data size
        uint32_t word = reinterpret_cast<const uint32_t *>(plain)[t];
        if (t == 2) word = (word & 0x00FFFFFFu) | (1u << 24);
        if (t == 8) word = (uint32_t)carry;
        if (t == 9) word = (uint32_t)(carry >> 32);
        reinterpret_cast<uint32_t *>(dst)[t] = word;
    }
    const uint64_t pad0 = 64 + 8ull * (nseg + 1);
    if (t < data_start - pad0) dst[pad0 + t] = 0;
    if (t == 0) {
        *out_size = data_start + carry;
        if (data_start + carry > cap && status) atomicOr(status, 2);
    }
}

// ---- write pass ----------------------------------------------------------
// Dynamic LDS: the coded segment image (ldsb bytes, a multiple of 16).
__global__ __launch_bounds__(256) void k_huff_write(const uint8_t *__restrict__ plain, uint64_t data_start,
                                                    uint32_t nseg, const uint8_t *__restrict__ info,
                                                    uint8_t *__restrict__ dst, uint32_t ldsb,
                                                    int32_t *__restrict__ status) {
    extern __shared__ u32x4 img4[];
    __shared__ uint32_t len[256], rcode[256], cntl[kHufMaxLen + 1], first[kHufMaxLen + 1];
    __shared__ uint32_t sub_base[kHufSub];
    const uint32_t t = threadIdx.x, s = blockIdx.x;
    if (s >= nseg) return;
    const uint64_t a = gld64(plain + 64 + 8ull * s), b = gld64(plain + 64 + 8ull * (s + 1));
    const uint8_t *seg = plain + data_start + a;
    const uint32_t n = (uint32_t)(b - a), m16 = n / kHufSub;
    const uint8_t *rec = info + (uint64_t)s * kHufInfo;
    const uint32_t coded = reinterpret_cast<const uint32_t *>(rec + 192)[0];
    const uint64_t ta = gld64(dst + 64 + 8ull * s);
    uint8_t *const out = dst + data_start + ta;
    // the coded image: in LDS when it fits (ldsb bytes), else the destination
    // itself, cleared first (the offsets are final: the scan ran before)
    const bool in_lds = coded <= ldsb;
    auto body = [&](uint32_t *img) {
        for (uint32_t k = t; k < coded / 4; k += 256) img[k] = 0;
        if (!in_lds) __threadfence();
        const uint32_t lv = (gld8(rec + (t >> 1)) >> (4 * (t & 1))) & 15u;
        len[t] = lv;
        if (t <= kHufMaxLen) cntl[t] = 0;
        __syncthreads();
        if (lv) atomicAdd(&cntl[lv], 1u);
        if (t < kHufSub) {
            uint32_t base = kHufFixed;
            for (uint32_t k = 0; k < t; ++k) base += reinterpret_cast<const uint32_t *>(rec + 128)[k];
            sub_base[t] = base;
        }
        __syncthreads();
        if (t == 0) {
            uint32_t c = 0;
            for (uint32_t l = 1; l <= kHufMaxLen; ++l) {
                first[l] = c;
                c = (c + cntl[l]) << 1;
            }
        }
        __syncthreads();
        {
            uint32_t r = 0;
            for (uint32_t u = 0; u < t; ++u) r += len[u] == lv ? 1u : 0u;
            rcode[t] = lv ? huff_rev(first[lv] + r, lv) : 0u;
        }
        // fixed part: n, lengths, sub-stream sizes (bytes 0..195; streams start at 196)
        if (t < 49) {
            uint32_t word;
            if (t == 0) word = n;
            else if (t <= 32) word = gld32(rec + 4 * (t - 1));
            else word = reinterpret_cast<const uint32_t *>(rec + 128)[t - 33];
            img[t] = word;
        }
        __syncthreads();
        // thread = (sub-stream k, part p): bit offsets by a scan over the parts
        const uint32_t k = t >> 4, p = t & 15;
        const uint32_t q = (m16 + 15) / 16;
        const uint32_t lo = min(p * q, m16), hi = min(lo + q, m16);
        const uint8_t *src = seg + k * m16;
        uint32_t bits = 0;
        for (uint32_t i = lo; i < hi; ++i) bits += len[gld8(src + i)];
        uint32_t incl = bits;
#pragma unroll
        for (uint32_t d = 1; d < 16; d <<= 1) {
            const uint32_t o = (uint32_t)__shfl_up((int)incl, d, 16);
            if (p >= d) incl += o;
        }
        uint32_t pos = 8 * sub_base[k] + incl - bits;
        for (uint32_t i = lo; i < hi; ++i) {
            const uint32_t v = gld8(src + i);
            const uint32_t l = len[v], rc = rcode[v];
            atomicOr(&img[pos >> 5], rc << (pos & 31));
            if ((pos & 31) + l > 32) atomicOr(&img[(pos >> 5) + 1], rc >> (32 - (pos & 31)));
            pos += l;
        }
    };
    if (in_lds) {
        body(reinterpret_cast<uint32_t *>(img4));
        __syncthreads();
        for (uint32_t u = t; u < coded / 16; u += 256) gst128(out + 16 * u, img4[u]);
    } else {
        body(reinterpret_cast<uint32_t *>(out));
    }
}

// ---- decode --------------------------------------------------------------
// One entropy-coded container whose segments a decode wavefront takes.
struct HufJob {
    const uint8_t *src;         // coded container
    uint8_t *plain;             // plain container at a fixed segment stride
    uint64_t src_size, data_start, data_bytes, stride;
    uint32_t nseg, table;       // segments; nonzero: also write the plain header and offset table
    uint32_t status, pad;       // index of its status word
};

// Lanes (segment g of the wavefront's four, sub-stream k). Plain segment s
// of job jb goes to jb.plain + data_start + s * stride; `have` is false for
// lanes whose group has no segment (they take part in the wave's syncs).
// With jb.table the group of segment s also writes its offset-table entries
// (and segment 0's group the header: the coded one's, entropy 0, data bytes
// nseg * stride).
__device__ __forceinline__ void huff_decode_wave(const HufJob &jb, uint32_t s, bool have, int32_t *__restrict__ statuses) {
    __shared__ uint16_t lut[kHufSegsPerWave][1u << kHufMaxLen];
    __shared__ uint32_t cnt[kHufSegsPerWave][kHufSub][kHufMaxLen + 1];
    __shared__ uint32_t first[kHufSegsPerWave][kHufMaxLen + 1];
    __shared__ uint32_t index[kHufSegsPerWave][kHufMaxLen + 1];   // first position of each length in code order
    __shared__ uint32_t codes_end[kHufSegsPerWave];              // end of the used 11-bit code space
    __shared__ uint8_t sorted[kHufSegsPerWave][256];             // values in (length, value) order
    const uint32_t lane = threadIdx.x & 63, g = lane >> 4, k = lane & 15;
    const uint8_t *const src = jb.src;
    uint8_t *const plain = jb.plain;
    const uint64_t src_size = jb.src_size, data_start = jb.data_start, data_bytes = jb.data_bytes;
    const uint64_t stride = jb.stride;
    const uint32_t nseg = jb.nseg;
    int32_t *const status = statuses ? statuses + jb.status : nullptr;
    if (have && jb.table && s < nseg) {
        uint64_t *const tab = reinterpret_cast<uint64_t *>(plain + 64);
        if (k == 0) tab[s] = (uint64_t)s * stride;
        if (k == 1 && s + 1 == nseg) tab[nseg] = (uint64_t)nseg * stride;
        if (s == 0) {
            uint32_t word = gld32(src + 4 * k);
            if (k == 2) word &= 0x00FFFFFFu;   // entropy 0
            if (k == 8) word = (uint32_t)(stride * nseg);
            if (k == 9) word = (uint32_t)((stride * nseg) >> 32);
            reinterpret_cast<uint32_t *>(plain)[k] = word;
        }
    }
    bool ok = have && s < nseg;
    uint64_t a = 0, b = 0;
    if (ok) {
        a = gld64(src + 64 + 8ull * s);
        b = gld64(src + 64 + 8ull * (s + 1));
        ok = a <= b && b <= data_bytes && !((a | b) & 15u) && b - a >= kHufFixed && data_start + b <= src_size;
    }
    const uint8_t *seg = src + data_start + a;
    const uint32_t n = ok ? gld32(seg) : 0u;
    if (ok && (n % 16 || n == 0 || n > stride)) ok = false;
    // this lane's 16 values: lengths, counts per length
    uint32_t lw[2] = {0u, 0u};
    if (ok) { lw[0] = gld32(seg + 4 + 8 * k); lw[1] = gld32(seg + 8 + 8 * k); }
    uint32_t lc[kHufMaxLen + 1];
#pragma unroll
    for (uint32_t l = 0; l <= kHufMaxLen; ++l) lc[l] = 0;
#pragma unroll
    for (uint32_t i = 0; i < 16; ++i) {
        const uint32_t l = (lw[i >> 3] >> (4 * (i & 7))) & 15u;
#pragma unroll
        for (uint32_t q = 1; q <= kHufMaxLen; ++q) lc[q] += l == q ? 1u : 0u;
        if (l > kHufMaxLen) ok = false;
    }
#pragma unroll
    for (uint32_t l = 0; l <= kHufMaxLen; ++l) cnt[g][k][l] = lc[l];
    wave_sync();
    if (k == 0) {
        uint32_t c = 0, pos = 0, end = 0;
        for (uint32_t l = 1; l <= kHufMaxLen; ++l) {
            first[g][l] = c;
            index[g][l] = pos;
            uint32_t tot = 0;
            for (uint32_t q = 0; q < kHufSub; ++q) tot += cnt[g][q][l];
            if (tot) end = (c + tot) << (kHufMaxLen - l);
            pos += tot;
            c = (c + tot) << 1;
        }
        codes_end[g] = end;
    }
    wave_sync();
    // canonical code of each value: first code of its length + values of that
    // length before it (earlier lanes, then earlier values of this lane)
    uint32_t seen[kHufMaxLen + 1];
#pragma unroll
    for (uint32_t l = 1; l <= kHufMaxLen; ++l) {
        uint32_t before = 0;
        for (uint32_t q = 0; q < k; ++q) before += cnt[g][q][l];
        seen[l] = first[g][l] + before;
    }
#pragma unroll
    for (uint32_t i = 0; i < 16; ++i) {
        const uint32_t l = (lw[i >> 3] >> (4 * (i & 7))) & 15u;
        if (l == 0 || l > kHufMaxLen) continue;
        uint32_t code = 0;
#pragma unroll
        for (uint32_t q = 1; q <= kHufMaxLen; ++q)
            if (q == l) { code = seen[q]; seen[q] = code + 1; }
        if (code >= (1u << l)) { ok = false; continue; }
        sorted[g][(index[g][l] + code - first[g][l]) & 255u] = (uint8_t)(16 * k + i);
    }
    wave_sync();
    // table entries: an 11-bit window (first code bit lowest) read most
    // significant bit first falls in the left-aligned range of exactly one
    // code length; the value is found by its offset in that range
    {
        uint32_t lj[kHufMaxLen + 1], ix[kHufMaxLen + 1];
#pragma unroll
        for (uint32_t l = 1; l <= kHufMaxLen; ++l) {
            lj[l] = first[g][l] << (kHufMaxLen - l);
            ix[l] = index[g][l];
        }
        const uint32_t end = codes_end[g];
        for (uint32_t e = k; e < (1u << kHufMaxLen); e += kHufSub) {
            const uint32_t M = __builtin_bitreverse32(e) >> (32 - kHufMaxLen);
            uint32_t len_of = 0, base = 0, off = 0;
#pragma unroll
            for (uint32_t l = 1; l <= kHufMaxLen; ++l) {
                // the range of length l is [lj[l], lj[l+1]); an empty length
                // starts where the next one does, so the last start <= M wins
                if (M >= lj[l]) { len_of = l; base = ix[l]; off = (M - lj[l]) >> (kHufMaxLen - l); }
            }
            uint16_t v = 0;
            if (M < end && len_of) v = (uint16_t)(sorted[g][(base + off) & 255u] | (len_of << 8));
            lut[g][e] = v;
        }
    }
    wave_sync();
    // this lane's sub-stream
    uint32_t size = ok ? gld32(seg + 132 + 4 * k) : 0u;
    uint32_t incl = size;
#pragma unroll
    for (uint32_t d = 1; d < 16; d <<= 1) {
        const uint32_t o = (uint32_t)__shfl_up((int)incl, d, 16);
        if (k >= d) incl += o;
    }
    const uint64_t sbeg = a + kHufFixed + incl - size;   // data-relative byte offset
    if (ok && sbeg + size > b) ok = false;
    const uint32_t m16 = n / kHufSub;
    const uint32_t count = ok ? m16 : 0u;
    uint8_t *out = plain + data_start + (uint64_t)s * stride + (uint64_t)k * m16;
    // The sub-stream in aligned 16-byte blocks through a buffer resource
    // bounded to this segment (blocks past its end read as zero). Four
    // slots are reloaded as soon as their last dword is taken, so every
    // load has three blocks of decoding to arrive; the slots never move
    // between registers, so no wait is forced early.
    const Buf sb = make_buf(seg, ok ? (uint32_t)(b - a) : 0u);
    uint32_t boff = (uint32_t)(sbeg - a) & ~15u;
    u32x4 qa = buf_ld128(sb, boff), qb = buf_ld128(sb, boff + 16), qc = buf_ld128(sb, boff + 32),
          qd = buf_ld128(sb, boff + 48);
    boff += 64;
    uint32_t skipw = (uint32_t)(sbeg & 15) >> 2;   // dwords of the first block before the stream
    uint32_t skipb = 8 * ((uint32_t)sbeg & 3);     // then bytes of the first dword
    uint64_t bb = 0;
    uint32_t nb = 0, i = 0, used = 0, bad = 0;
    // output: bytes up to the lane's first 16-byte boundary one by one, then
    // whole 16-byte units from four staging words, then the tail
    const uint32_t head = min((uint32_t)((16 - ((uintptr_t)out & 15)) & 15), count);
    uint32_t w0 = 0, w1 = 0, w2 = 0, w3 = 0;
    auto take = [&](uint32_t wd) {
        if (skipw) { --skipw; return; }
        if (i >= count) return;   // past the last symbol: nb would grow past 64
        bb |= (uint64_t)wd << nb;
        nb += 32;
        bb >>= skipb;
        nb -= skipb;
        skipb = 0;
        while (nb >= kHufMaxLen && i < count) {
            const uint32_t e = lut[g][(uint32_t)bb & ((1u << kHufMaxLen) - 1)];
            const uint32_t l = e >> 8;
            bad |= l == 0 ? 1u : 0u;
            bb >>= l;
            nb -= l;
            used += l;
            const uint32_t sym = e & 0xFFu;
            if (i < head) {
                gst8(out + i, sym);
            } else {
                const uint32_t j = i - head, q = j & 15, v = sym << (8 * (q & 3));
                w0 |= (q >> 2) == 0 ? v : 0u;
                w1 |= (q >> 2) == 1 ? v : 0u;
                w2 |= (q >> 2) == 2 ? v : 0u;
                w3 |= (q >> 2) == 3 ? v : 0u;
                if (q == 15) {
                    u32x4 u;
                    u.x = w0; u.y = w1; u.z = w2; u.w = w3;
                    gst128(out + head + j - 15, u);
                    w0 = w1 = w2 = w3 = 0;
                }
            }
            ++i;
        }
    };
    while (i < count) {
        take(qa.x); take(qa.y); take(qa.z); take(qa.w);
        qa = buf_ld128(sb, boff);
        take(qb.x); take(qb.y); take(qb.z); take(qb.w);
        qb = buf_ld128(sb, boff + 16);
        take(qc.x); take(qc.y); take(qc.z); take(qc.w);
        qc = buf_ld128(sb, boff + 32);
        take(qd.x); take(qd.y); take(qd.z); take(qd.w);
        qd = buf_ld128(sb, boff + 48);
        boff += 64;
    }
    if (count > head) {
        const uint32_t rem = (count - head) & 15, base = count - rem;
        for (uint32_t q = 0; q < rem; ++q) {
            const uint32_t wd = (q >> 2) == 0 ? w0 : (q >> 2) == 1 ? w1 : (q >> 2) == 2 ? w2 : w3;
            gst8(out + base + q, wd >> (8 * (q & 3)));
        }
    }
    if (bad || used > 8u * size) ok = false;
    if (have && s < nseg && !ok && status) atomicOr(status, 4);
}

__global__ __launch_bounds__(64) void k_huff_decode(const uint8_t *__restrict__ src, uint64_t src_size,
                                                    uint64_t data_start, uint64_t data_bytes, uint32_t nseg,
                                                    uint8_t *__restrict__ plain, uint64_t stride,
                                                    int32_t *__restrict__ status) {
    HufJob jb;
    jb.src = src; jb.plain = plain;
    jb.src_size = src_size; jb.data_start = data_start; jb.data_bytes = data_bytes; jb.stride = stride;
    jb.nseg = nseg; jb.table = 0; jb.status = 0; jb.pad = 0;
    huff_decode_wave(jb, blockIdx.x * kHufSegsPerWave + (threadIdx.x >> 4), true, status);
}

// Many containers: entry e = job << 32 | segment; a wavefront takes four
// consecutive entries and also writes the plain containers' tables. Corrupt
// coded segments of job j set bit 2 of status[jobs[j].status].
__global__ __launch_bounds__(64) void k_huff_decode_batch(const HufJob *__restrict__ jobs,
                                                          const uint64_t *__restrict__ entries, uint32_t nent,
                                                          int32_t *__restrict__ status) {
    const uint32_t q = blockIdx.x * kHufSegsPerWave + (threadIdx.x >> 4);
    const bool have = q < nent;
    const uint64_t e = have ? entries[q] : 0ull;
    huff_decode_wave(jobs[have ? (uint32_t)(e >> 32) : 0u], (uint32_t)e, have, status);
}

// Header and offset table of the workspace (plain) container.
__global__ void k_huff_plain_table(const uint8_t *__restrict__ src, uint32_t nseg, uint64_t stride,
                                   uint8_t *__restrict__ plain) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < 16) {
        uint32_t word = gld32(src + 4 * t);
        if (t == 2) word &= 0x00FFFFFFu;   // entropy 0
        if (t == 8) word = (uint32_t)(stride * nseg);
        if (t == 9) word = (uint32_t)((stride * nseg) >> 32);
        reinterpret_cast<uint32_t *>(plain)[t] = word;
    }
    if (t <= nseg) reinterpret_cast<uint64_t *>(plain + 64)[t] = (uint64_t)t * stride;
}

}  // namespace spz

// Sprintz encoder kernels for gfx950.
//
// Paper: Algorithm 1 (encodeBlock) applied to every 8-row block of a
// segment; forecasters of Section 4.2 (delta; FIRE as Algorithm 3 with the
// practical changes of Section 4.2.2: alpha once per block, one summed
// gradient update per block from every other sample); zigzag, bit widths,
// log2(w)-bit headers and column-/row-major payloads of Section 4.3;
// run-length records for all-zero blocks (Algorithm 1).
//
// Two passes over the same per-lane walk: pass 1 (WRITE = false) only sizes
// every segment; a single-workgroup scan turns the sizes into the offset
// table; pass 2 (WRITE = true) repeats the walk and writes the bytes. A lane
// walks one column, or two (j and j + 64) when D exceeds 64, so that a
// segment's lane group stays inside one wavefront.
#pragma once

#include "spz_device.h"

namespace spz {

// Bytes of the record headers of a segment with nrec records (all groups,
// each padded to a byte).
__device__ __forceinline__ uint32_t header_bytes(uint32_t nrec, uint32_t D, uint32_t HB, uint32_t G) {
    if (G == 0) return (nrec * D * HB + 7) >> 3;
    uint32_t full = nrec / G, rest = nrec % G;
    return full * ((G * D * HB + 7) >> 3) + ((rest * D * HB + 7) >> 3);
}

// Ring of header words per lane group (enough for one record plus a byte).
__device__ __forceinline__ uint32_t ring_words(uint32_t Dp) { return Dp >= 8 ? Dp / 4 : 2; }

template <int W, bool FIRE, bool COLMAJOR, bool WRITE>
__global__ __launch_bounds__(kThreads) void k_encode(const typename Elem<W>::T *__restrict__ src, Geom g,
                                                     uint32_t *__restrict__ seg_info, uint8_t *__restrict__ dst,
                                                     int32_t *__restrict__ status) {
    using T = typename Elem<W>::T;
    constexpr uint32_t HB = W == 8 ? 3 : 4;
    constexpr uint32_t WB = W / 8;
    __shared__ uint32_t hring[512];
    __shared__ uint32_t pbuf[COLMAJOR ? 1 : 2 * kThreads * W / 4];

    const uint32_t Dp = 1u << g.dp_log2;          // padded columns of a segment
    const uint32_t lg = min(g.dp_log2, 6u);
    const uint32_t Dl = 1u << lg;                 // lanes of a segment
    const uint32_t gid = blockIdx.x * kThreads + threadIdx.x;
    const uint32_t seg = gid >> lg;
    const uint32_t j = gid & (Dl - 1);
    if (seg >= g.nseg) return;  // whole lane groups leave together
    const uint32_t D = g.D;
    constexpr uint32_t CPL = 2;                   // column slots of a lane: j and j + 64
    const uint32_t ncs = D > Dl ? 2u : 1u;
    bool col[CPL];
    for (uint32_t c = 0; c < CPL; ++c) col[c] = c < ncs && j + 64 * c < D;

    const uint64_t row0 = (uint64_t)seg * g.S;
    const uint32_t nr = (uint32_t)min((uint64_t)g.S, g.rows - row0);
    const uint32_t nblk = nr >> 3, tail = nr & 7u;
    const T *xs = src + row0 * D + j;

    // write state
    const uint32_t gw = threadIdx.x >> lg;         // lane group within the workgroup
    const uint32_t RW = ring_words(Dp);
    uint32_t *ring = hring + gw * RW;
    uint32_t *pay = pbuf + (COLMAJOR ? 0 : gw * (Dp * W / 4));
    uint64_t base = 0;
    uint32_t nrec_total = 0, seg_size = 0;
    uint32_t cursor = 4, grp_left = 0, hstart = 0, hbit = 0, hflushed = 0, r = 0;
    bool overflow = false;
    auto st = [&](uint64_t pos, uint32_t v) {
        if (pos < g.cap) dst[pos] = (uint8_t)v;
        else overflow = true;
    };
    if (WRITE) {
        base = g.data_start + ld_u64_aligned(dst + 64 + 8ull * seg);
        seg_size = seg_info[2 * seg];
        nrec_total = seg_info[2 * seg + 1];
        for (uint32_t k = j; k < RW; k += Dl) ring[k] = 0;
        if (!COLMAJOR)
            for (uint32_t k = j; k < Dp * W / 4; k += Dl) pay[k] = 0;
        if (j == 0) {
            if (base + 4 <= g.cap) *reinterpret_cast<uint32_t *>(dst + base) = nrec_total;
            else overflow = true;
        }
    }

    uint32_t nrec = 0, payload = 0, run = 0;
    uint32_t prev[CPL] = {0, 0};
    int32_t delta[CPL] = {0, 0}, acc[CPL] = {0, 0};

    // Emit one record: header codes of this lane's columns, payload bytes.
    auto emit = [&](const uint32_t *codes, bool is_rle, uint32_t count, const uint32_t (*zz)[8], const uint32_t *widths,
                    const uint32_t *offs, uint32_t wsum) {
        if (grp_left == 0) {
            uint32_t cnt = g.G ? min(g.G, nrec_total - r) : nrec_total;
            hstart = cursor;
            cursor += (cnt * D * HB + 7) >> 3;
            hbit = 0;
            hflushed = 0;
            grp_left = cnt;
        }
        for (uint32_t c = 0; c < ncs; ++c) {
            const uint32_t code = codes[c];
            if (code == 0) continue;
            uint32_t p = hbit + (j + 64 * c) * HB;
            uint32_t w0 = (p >> 5) & (RW - 1), s = p & 31u;
            atomicOr(&ring[w0], code << s);
            if (s + HB > 32) atomicOr(&ring[(w0 + 1) & (RW - 1)], code >> (32 - s));
        }
        hbit += D * HB;
        if (is_rle) {
            if (j == 0) {
                st(base + cursor, count & 0xFFu);
                st(base + cursor + 1, count >> 8);
            }
            cursor += 2;
        } else if (COLMAJOR) {
            // column j: its 8 values, width bits each, LSB first = width bytes
            const uint32_t *z = zz[0];
            const uint32_t width = widths[0], off = offs[0];
            uint64_t lo = 0, hi = 0;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                uint32_t pos = (uint32_t)i * width;
                if (pos < 64) {
                    lo |= (uint64_t)z[i] << pos;
                    if (pos + width > 64) hi |= (uint64_t)z[i] >> (64 - pos);
                } else {
                    hi |= (uint64_t)z[i] << (pos - 64);
                }
            }
            for (uint32_t k = 0; k < width; ++k) {
                uint32_t byte = k < 8 ? (uint32_t)(lo >> (8 * k)) : (uint32_t)(hi >> (8 * (k - 8)));
                st(base + cursor + off + k, byte & 0xFFu);
            }
            cursor += wsum;
        } else {
            // row-major: row i = fields of all columns, padded to a byte
            const uint32_t R = (wsum + 7) >> 3;
            for (uint32_t c = 0; c < ncs; ++c) {
                const uint32_t width = widths[c], off = offs[c];
                if (width == 0) continue;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    uint32_t p = (uint32_t)i * 8 * R + off;
                    uint32_t w0 = p >> 5, s = p & 31u;
                    atomicOr(&pay[w0], zz[c][i] << s);
                    if (s + width > 32) atomicOr(&pay[w0 + 1], zz[c][i] >> (32 - s));
                }
            }
            for (uint32_t k = j; k < 8 * R; k += Dl) {
                uint32_t sh = (k & 3u) * 8;
                uint32_t old = atomicAnd(&pay[k >> 2], ~(0xFFu << sh));
                st(base + cursor + k, (old >> sh) & 0xFFu);
            }
            cursor += 8 * R;
        }
        grp_left--;
        r++;
        uint32_t complete = grp_left == 0 ? (hbit + 7) >> 3 : hbit >> 3;
        for (uint32_t k = hflushed + j; k < complete; k += Dl) {
            uint32_t wi = (k >> 2) & (RW - 1), sh = (k & 3u) * 8;
            uint32_t old = atomicAnd(&ring[wi], ~(0xFFu << sh));
            st(base + hstart + k, (old >> sh) & 0xFFu);
        }
        hflushed = complete;
    };

    const uint32_t zcodes[CPL] = {0, 0}, zw[CPL] = {0, 0};
    for (uint32_t b = 0; b < nblk; ++b) {
        uint32_t z[CPL][8], code[CPL] = {0, 0}, width[CPL] = {0, 0}, off[CPL] = {0, 0};
        uint32_t wsum = 0;
        for (uint32_t c = 0; c < ncs; ++c) {
            const int32_t alpha = FIRE ? (acc[c] >> g.sh) : 0;
            int32_t grad = 0;
            uint32_t orz = 0;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const uint32_t x = col[c] ? (uint32_t)xs[(uint64_t)(8 * b + i) * D + 64 * c] : 0u;
                int32_t pred = (int32_t)prev[c];
                if (FIRE) pred += __mul24(alpha, delta[c]) >> W;
                const int32_t e = sext<W>((int32_t)x - pred);
                if (FIRE && (i & 1)) grad += __mul24(sgn(e), delta[c]);
                delta[c] = sext<W>((int32_t)x - (int32_t)prev[c]);
                prev[c] = x;
                z[c][i] = zigzag(e);
                orz |= z[c][i];
            }
            if (FIRE) acc[c] = min(max(acc[c] + grad, g.acc_lo), g.acc_hi);
            code[c] = min(bitlen(orz), (uint32_t)W - 1);
            width[c] = code[c] < (uint32_t)W - 1 ? code[c] : (uint32_t)W;
            // columns j + 64 follow all of the first 64 in the row
            const uint32_t incl = group_incl_sum(width[c], Dl, j);
            off[c] = wsum + incl - width[c];
            wsum += group_last(incl, Dl);
        }
        if (wsum == 0) {
            run++;
            if (run == kRleMax) {
                if (WRITE) emit(zcodes, true, run, z, zw, zw, 0);
                nrec++;
                payload += 2;
                run = 0;
            }
            continue;
        }
        if (run > 0) {
            if (WRITE) emit(zcodes, true, run, z, zw, zw, 0);
            nrec++;
            payload += 2;
            run = 0;
        }
        if (WRITE) emit(code, false, 0, z, width, off, wsum);
        nrec++;
        payload += COLMAJOR ? wsum : 8 * ((wsum + 7) >> 3);
    }
    if (run > 0) {
        const uint32_t z0[CPL][8] = {};
        if (WRITE) emit(zcodes, true, run, z0, zw, zw, 0);
        nrec++;
        payload += 2;
    }

    const uint32_t tail_bytes = tail * D * WB;
    if (!WRITE) {
        if (j == 0) {
            uint32_t size = 4 + header_bytes(nrec, D, HB, g.G) + payload + tail_bytes;
            seg_info[2 * seg] = (size + 15) & ~15u;
            seg_info[2 * seg + 1] = nrec;
        }
        return;
    }
    // raw tail rows (last segment only), then zero padding to 16 bytes
    for (uint32_t c = 0; c < ncs; ++c) {
        if (!col[c]) continue;
        for (uint32_t t = 0; t < tail; ++t) {
            uint32_t x = (uint32_t)xs[(uint64_t)(8 * nblk + t) * D + 64 * c];
            uint32_t pos = cursor + (t * D + j + 64 * c) * WB;
            for (uint32_t q = 0; q < WB; ++q) st(base + pos + q, (x >> (8 * q)) & 0xFFu);
        }
    }
    cursor += tail_bytes;
    const uint32_t end = (cursor + 15) & ~15u;
    for (uint32_t k = cursor + j; k < end; k += Dl) st(base + k, 0);
    if (j == 0 && (end != seg_size || r != nrec_total)) overflow = true;
    if (overflow && status) atomicOr(status, 2);
}

// Exclusive scan of the per-segment sizes into the container's offset
// table, plus the 64-byte container header and *out_size. One workgroup.
__global__ __launch_bounds__(1024) void k_scan_sizes(const uint32_t *__restrict__ seg_info, Geom g, uint32_t w,
                                                     uint32_t dtype, uint32_t forecaster, uint32_t learn_shift,
                                                     uint8_t *__restrict__ dst, uint64_t *__restrict__ out_size,
                                                     int32_t *__restrict__ status) {
    // Exclusive scan of the segment byte sizes into the offset table, 1024
    // entries per step (coalesced loads, wavefront shuffle scans, one LDS
    // exchange of the 16 wavefront totals), then the container header.
    __shared__ uint64_t wsum[16];
    const uint32_t t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const uint32_t n = g.nseg;
    uint64_t *tab = reinterpret_cast<uint64_t *>(dst + 64);
    uint64_t carry = 0;
    for (uint32_t base = 0; base < n; base += 1024) {
        const uint32_t k = base + t;
        const uint32_t v = k < n ? seg_info[2 * k] : 0u;
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
        if (k < n) tab[k] = before + incl - v;
        carry = total;
        __syncthreads();
    }
    if (t == 0) tab[n] = carry;
    if (t < 16) {
        // 64-byte header as 16 dwords (reading R18: the container layout)
        uint32_t word = 0;
        switch (t) {
            case 0: word = 0x315A5053u; break;                                            // "SPZ1"
            case 1: word = 1u | (w << 16) | (dtype << 24); break;                          // version, w, dtype
            case 2: word = forecaster | (learn_shift << 8) | (g.G << 16); break;           // entropy 0
            case 3: word = g.D; break;
            case 4: word = (uint32_t)g.rows; break;
            case 5: word = (uint32_t)(g.rows >> 32); break;
            case 6: word = g.S; break;
            case 7: word = n; break;
            case 8: word = (uint32_t)carry; break;
            case 9: word = (uint32_t)(carry >> 32); break;
            default: word = 0; break;
        }
        reinterpret_cast<uint32_t *>(dst)[t] = word;
    }
    // zero padding between the offset table and the data
    const uint64_t pad0 = 64 + 8ull * (n + 1);
    if (t < g.data_start - pad0) dst[pad0 + t] = 0;
    if (t == 0) {
        *out_size = g.data_start + carry;
        if (g.data_start + carry > g.cap && status) atomicOr(status, 2);
    }
}

}  // namespace spz

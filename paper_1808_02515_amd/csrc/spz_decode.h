// Sprintz decoder kernel for gfx950.
//
// Paper: Algorithm 2 (decodeBlock) for every record of a segment. A record
// whose header codes are all zero is a run of all-zero blocks: the samples
// are the forecaster's predictions (the forecaster keeps its delta in step
// with the encoder, which also trains on those rows). Otherwise the payload
// is unpacked with the per-column widths of Section 4.3 and x = err + x_hat.
//
// One lane per (segment, column); a lane walks its segment's records in
// order, so header groups of any size need no extra pass. Every read of the
// container is clamped inside the segment's extent, so a corrupt container
// can only produce wrong samples and a status bit, never a stray access.
#pragma once

#include "spz_device.h"

namespace spz {

template <int W, bool FIRE, bool COLMAJOR>
__global__ __launch_bounds__(kThreads) void k_decode(const uint8_t *__restrict__ src, Geom g,
                                                     typename Elem<W>::T *__restrict__ dst,
                                                     int32_t *__restrict__ status) {
    using T = typename Elem<W>::T;
    constexpr uint32_t HB = W == 8 ? 3 : 4;
    constexpr uint32_t WB = W / 8;
    constexpr uint32_t MASK = (1u << W) - 1;

    const uint32_t Dp = 1u << g.dp_log2;
    const uint32_t gid = blockIdx.x * kThreads + threadIdx.x;
    const uint32_t seg = gid >> g.dp_log2;
    const uint32_t j = gid & (Dp - 1);
    if (seg >= g.nseg) return;
    const bool col = j < g.D;
    const uint32_t D = g.D;

    const uint64_t a = ld_u64_aligned(src + 64 + 8ull * seg);
    const uint64_t b = ld_u64_aligned(src + 64 + 8ull * seg + 8);
    if (a > b || b > g.data_bytes || ((a | b) & 15u) || b - a < 16 || b - a > 0x7FFFFFF0ull) {
        if (j == 0 && status) atomicOr(status, 1);
        return;
    }
    const uint32_t *segw = reinterpret_cast<const uint32_t *>(src + g.data_start + a);
    const uint32_t nwm1 = (uint32_t)((b - a) >> 2) - 1;
    const uint32_t ext = (uint32_t)(b - a);
    // bits [p, p + width) of the segment, width <= 16
    auto getbits = [&](uint32_t p, uint32_t width) -> uint32_t {
        const uint32_t wi = p >> 5;
        const uint32_t lo = segw[min(wi, nwm1)];
        const uint32_t hi = segw[min(wi + 1, nwm1)];
        const uint32_t v = __builtin_amdgcn_alignbit(hi, lo, p & 31u);
        return __builtin_amdgcn_ubfe(v, 0u, width);
    };

    const uint64_t row0 = (uint64_t)seg * g.S;
    const uint32_t nr = (uint32_t)min((uint64_t)g.S, g.rows - row0);
    const uint32_t nblk = nr >> 3, tail = nr & 7u;
    T *out = dst + row0 * D + (col ? j : 0);

    const uint32_t nrec = segw[0];
    if (nrec > nblk) {  // every record covers at least one block
        if (j == 0 && status) atomicOr(status, 1);
        return;
    }
    uint32_t cursor = 4;        // byte position in the segment
    uint32_t r = 0, grp_left = 0, hpos = 0, rle_left = 0;
    uint32_t width = 0, off = 0, stride = 0, p0 = 0;
    bool is_rle = false, ok = true;

    uint32_t prev = 0;
    int32_t delta = 0, acc = 0;

    for (uint32_t blk = 0; blk < nblk; ++blk) {
        if (rle_left == 0) {
            if (r >= nrec) { ok = false; break; }
            if (grp_left == 0) {
                const uint32_t cnt = g.G ? min(g.G, nrec - r) : nrec;
                hpos = cursor * 8;
                cursor += (uint32_t)(((uint64_t)cnt * D * HB + 7) >> 3);
                grp_left = cnt;
            }
            const uint32_t code = col ? getbits(hpos + j * HB, HB) : 0u;
            hpos += D * HB;
            grp_left--;
            r++;
            width = code < (uint32_t)W - 1 ? code : (uint32_t)W;
            const uint32_t incl = group_incl_sum(width, Dp, j);
            const uint32_t wsum = group_last(incl, Dp);
            off = incl - width;
            if (wsum == 0) {
                const uint32_t cnt16 = getbits(cursor * 8, 16);
                cursor += 2;
                if (cnt16 == 0) { ok = false; break; }
                rle_left = cnt16;
                is_rle = true;
            } else {
                if (COLMAJOR) {
                    p0 = (cursor + off) * 8;   // column j: width bytes, values back to back
                    stride = width;
                    cursor += wsum;
                } else {
                    const uint32_t R = (wsum + 7) >> 3;  // bytes per packed row
                    p0 = cursor * 8 + off;
                    stride = 8 * R;
                    cursor += 8 * R;
                }
                rle_left = 1;
                is_rle = false;
            }
        }
        rle_left--;
        const uint32_t wd = is_rle ? 0u : width;
        const int32_t alpha = FIRE ? (acc >> g.sh) : 0;
        int32_t grad = 0;
        T vals[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const uint32_t z = getbits(p0 + (uint32_t)i * stride, wd);
            const int32_t e = unzigzag(z);
            int32_t s = e;
            if (FIRE) s += __mul24(alpha, delta) >> W;
            if (FIRE && (i & 1)) grad += __mul24(sgn(e), delta);
            if (FIRE) delta = sext<W>(s);
            prev = (prev + (uint32_t)s) & MASK;
            vals[i] = (T)prev;
        }
        if (FIRE) acc = min(max(acc + grad, g.acc_lo), g.acc_hi);
        if (col) {
#pragma unroll
            for (int i = 0; i < 8; ++i) out[(uint64_t)(8 * blk + i) * D] = vals[i];
        }
    }
    if (ok && (rle_left != 0 || r != nrec)) ok = false;
    if (ok) {
        if (col) {
            for (uint32_t t = 0; t < tail; ++t) {
                const uint32_t x = getbits((cursor + (t * D + j) * WB) * 8, W);
                out[(uint64_t)(8 * nblk + t) * D] = (T)x;
            }
        }
        cursor += tail * D * WB;
        if (cursor > ext) ok = false;
    }
    if (!ok && j == 0 && status) atomicOr(status, 1);
}

}  // namespace spz

// Sprintz decoder kernel for gfx950.
//
// Paper: Algorithm 2 (decodeBlock) for every record of a segment. A record
// whose header codes are all zero is a run of all-zero blocks: the samples
// are the forecaster's predictions (the forecaster keeps its delta in step
// with the encoder, which also trains on those rows). Otherwise the payload
// is unpacked with the per-column widths of Section 4.3 and x = err + x_hat.
//
// One lane per (segment, column), or per two columns j and j + 64 when D
// exceeds 64 (a segment's lane group never outgrows a wavefront); a lane
// walks its segment's records in order, so header groups of any size need
// no extra pass. Every read of the container is clamped inside the segment's
// extent, so a corrupt container can only produce wrong samples and a status
// bit, never a stray access.
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

    const uint32_t lg = min(g.dp_log2, 6u);
    const uint32_t Dl = 1u << lg;                 // lanes of a segment
    const uint32_t gid = blockIdx.x * kThreads + threadIdx.x;
    const uint32_t seg = gid >> lg;
    const uint32_t j = gid & (Dl - 1);
    if (seg >= g.nseg) return;
    const uint32_t D = g.D;
    constexpr uint32_t CPL = 2;                   // column slots of a lane: j and j + 64
    const uint32_t ncs = D > Dl ? 2u : 1u;
    bool col[CPL];
    for (uint32_t c = 0; c < CPL; ++c) col[c] = c < ncs && j + 64 * c < D;

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
    T *out = dst + row0 * D + j;

    const uint32_t nrec = segw[0];
    if (nrec > nblk) {  // every record covers at least one block
        if (j == 0 && status) atomicOr(status, 1);
        return;
    }
    uint32_t cursor = 4;        // byte position in the segment
    uint32_t r = 0, grp_left = 0, hpos = 0, rle_left = 0;
    uint32_t width[CPL] = {0, 0}, off[CPL] = {0, 0}, p0[CPL] = {0, 0}, stride = 0;
    bool is_rle = false, ok = true;

    uint32_t prev[CPL] = {0, 0};
    int32_t delta[CPL] = {0, 0}, acc[CPL] = {0, 0};

    for (uint32_t blk = 0; blk < nblk; ++blk) {
        if (rle_left == 0) {
            if (r >= nrec) { ok = false; break; }
            if (grp_left == 0) {
                const uint32_t cnt = g.G ? min(g.G, nrec - r) : nrec;
                hpos = cursor * 8;
                cursor += (uint32_t)(((uint64_t)cnt * D * HB + 7) >> 3);
                grp_left = cnt;
            }
            // the widths of the lane's columns; columns j + 64 follow all of
            // the first 64 in the row
            uint32_t wsum = 0;
            for (uint32_t c = 0; c < ncs; ++c) {
                const uint32_t code = col[c] ? getbits(hpos + (j + 64 * c) * HB, HB) : 0u;
                width[c] = code < (uint32_t)W - 1 ? code : (uint32_t)W;
                const uint32_t incl = group_incl_sum(width[c], Dl, j);
                off[c] = wsum + incl - width[c];
                wsum += group_last(incl, Dl);
            }
            hpos += D * HB;
            grp_left--;
            r++;
            if (wsum == 0) {
                const uint32_t cnt16 = getbits(cursor * 8, 16);
                cursor += 2;
                if (cnt16 == 0) { ok = false; break; }
                rle_left = cnt16;
                is_rle = true;
            } else {
                if (COLMAJOR) {
                    p0[0] = (cursor + off[0]) * 8;   // column j: width bytes, values back to back
                    stride = width[0];
                    cursor += wsum;
                } else {
                    const uint32_t R = (wsum + 7) >> 3;  // bytes per packed row
                    for (uint32_t c = 0; c < ncs; ++c) p0[c] = cursor * 8 + off[c];
                    stride = 8 * R;
                    cursor += 8 * R;
                }
                rle_left = 1;
                is_rle = false;
            }
        }
        rle_left--;
        for (uint32_t c = 0; c < ncs; ++c) {
            const uint32_t wd = is_rle ? 0u : width[c];
            const int32_t alpha = FIRE ? (acc[c] >> g.sh) : 0;
            int32_t grad = 0;
            T vals[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const uint32_t z = getbits(p0[c] + (uint32_t)i * stride, wd);
                const int32_t e = unzigzag(z);
                int32_t s = e;
                if (FIRE) s += __mul24(alpha, delta[c]) >> W;
                if (FIRE && (i & 1)) grad += __mul24(sgn(e), delta[c]);
                if (FIRE) delta[c] = sext<W>(s);
                prev[c] = (prev[c] + (uint32_t)s) & MASK;
                vals[i] = (T)prev[c];
            }
            if (FIRE) acc[c] = min(max(acc[c] + grad, g.acc_lo), g.acc_hi);
            if (col[c]) {
#pragma unroll
                for (int i = 0; i < 8; ++i) out[(uint64_t)(8 * blk + i) * D + 64 * c] = vals[i];
            }
        }
    }
    if (ok && (rle_left != 0 || r != nrec)) ok = false;
    if (ok) {
        for (uint32_t c = 0; c < ncs; ++c) {
            if (!col[c]) continue;
            for (uint32_t t = 0; t < tail; ++t) {
                const uint32_t x = getbits((cursor + (t * D + j + 64 * c) * WB) * 8, W);
                out[(uint64_t)(8 * nblk + t) * D + 64 * c] = (T)x;
            }
        }
        cursor += tail * D * WB;
        if (cursor > ext) ok = false;
    }
    if (!ok && j == 0 && status) atomicOr(status, 1);
}

}  // namespace spz

// Chunked, phase-split Sprintz decoder for gfx950 (header group = whole
// segment).
//
// Paper: Algorithm 2 (decodeBlock). The only step that is inherently serial
// is the forecaster recurrence of each column (Section 5.4: the serial
// dependence between decoding one sample and predicting the next is the
// limit). This kernel moves everything else off the serial path and hides
// memory latency by staging the next chunk while the current one decodes:
//
//   per chunk of up to 16 blocks of every segment of the workgroup
//   1. parse   (lanes = candidate records, from LDS): header codes -> widths,
//              column bit offsets, record sizes; group scans give payload
//              offsets and the block -> record map; run counts read here.
//   2. stage   (all lanes): 16-byte loads of the NEXT chunk's header and
//              payload windows are issued into registers; they land while
//      unpack  (lanes = (segment, block, column)) turns this chunk's bit
//              fields into errors e, stored as e * 2^w (FIRE) or e (delta).
//   3. serial  (one wavefront, lane = column chain): for FIRE
//                t = alpha * delta + e * 2^w      (v_mad_i32_i24)
//                delta = bits [w, 2w) of t, signed (v_bfe_i32)
//                x += delta
//              which equals x_hat + e with x_hat = x_{i-1} + floor(alpha *
//              delta / 2^w) modulo 2^w; the gradient sign(e) * delta_{i-1}
//              is summed on odd rows and the accumulator saturates once per
//              block (practical FIRE, Section 4.2.2).
//   4. output  (all lanes): samples leave row-major with 16-byte stores; the
//              staged registers replace the consumed windows in LDS.
//
// A workgroup holds 64 chains: 64 / Dp segments of Dp = next_pow2(D) lanes.
// Every global access goes through a bounded buffer resource.
#pragma once

#include "spz_device.h"

namespace spz {

constexpr int kChunkBlocks = 16;                 // blocks per chunk per segment (max)
constexpr int kChunkRows = kChunkBlocks * 8;     // 128
constexpr int kChainStride = kChunkRows + 4;     // dwords per chain in LDS (bank padding)
constexpr uint32_t kRleMark = 0xFFu;
constexpr int kStageUnits = 1120;                // 16-byte units per staging buffer (max over D, w)
constexpr int kStagePerThread = (kStageUnits + kThreads - 1) / kThreads;
constexpr int kUnpackPerThread = 64 * kChunkBlocks / kThreads;  // (segment, block, column) items

struct SegSlot {
    uint32_t ra;           // segment byte offset relative to the workgroup's first segment
    uint32_t ext;          // segment extent in bytes
    uint32_t nrec, nblk, tail;
    uint32_t r;            // next unread record
    uint32_t cursor;       // payload byte position of record r
    uint32_t rle_rem;      // blocks of a run continuing into this chunk
    uint32_t ok;
    uint32_t hbase;        // staged header window: segment byte offset (16-aligned)
    uint32_t pbase;        // staged payload window: segment byte offset (16-aligned)
};

// Staging geometry per segment, in 16-byte units: header window for CB
// records and payload window for CB records of at most 8*D*(w/8) bytes.
struct StageGeom {
    uint32_t hu, pu, nu;
    uint64_t nu_magic;  // ceil(2^32 / nu)
};

__host__ __device__ inline StageGeom stage_geom(uint32_t D, uint32_t w, uint32_t CB) {
    const uint32_t hb = w == 8 ? 3 : 4;
    StageGeom sg;
    sg.hu = ((CB * D * hb + 7) / 8 + 47) / 16;
    sg.pu = (CB * 8 * D * (w / 8) + 31 + 15) / 16;
    sg.nu = sg.hu + sg.pu;
    sg.nu_magic = ((1ull << 32) + sg.nu - 1) / sg.nu;
    return sg;
}

__host__ __device__ inline uint32_t chunk_blocks(uint32_t dp_log2) {
    const uint32_t v = 4u << dp_log2;
    return v < (uint32_t)kChunkBlocks ? v : (uint32_t)kChunkBlocks;
}

template <int W, bool FIRE, bool COLMAJOR>
__global__ __launch_bounds__(kThreads) void k_decode_chunked(const uint8_t *__restrict__ src, Geom g,
                                                             typename Elem<W>::T *__restrict__ dst,
                                                             uint64_t div_magic, int32_t *__restrict__ status) {
    constexpr uint32_t HB = W == 8 ? 3 : 4;
    constexpr uint32_t WB = W / 8;
    constexpr uint32_t CPW = 32 / HB;  // header codes per 32-bit window

    __shared__ int32_t E[64 * kChainStride];       // [chain][row]: errors, then samples
    __shared__ u32x4 STG[kStageUnits];              // staged header + payload windows of one chunk
    __shared__ uint32_t colmeta[64 * kChunkBlocks]; // [segment][record][column]: off | width << 24
    __shared__ uint32_t recbits[256];               // [segment][record]: payload bit offset in the window
    __shared__ uint32_t recstride[256];             // [segment][record]: bits per packed row
    __shared__ uint32_t blkrec[256];                // [segment][block]: record index or kRleMark
    __shared__ SegSlot slots[2][64];                // per-segment state, double buffered by chunk

    const uint32_t tid = threadIdx.x;
    const uint32_t lg = g.dp_log2;
    const uint32_t Dp = 1u << lg;
    const uint32_t SPW = 64u >> lg;                      // segments per workgroup
    const uint32_t CB = chunk_blocks(lg);
    const uint32_t CR = CB * 8;
    const uint32_t D = g.D;
    const uint32_t seg0 = blockIdx.x * SPW;
    const uint32_t nsw = min(SPW, g.nseg - seg0);         // segments of this workgroup
    const StageGeom sg = stage_geom(D, W, CB);
    // blocks of segment s (of this workgroup) in chunk c, from the geometry alone
    auto blocks_in_chunk = [&](uint32_t s, uint32_t c) -> uint32_t {
        const uint32_t nb = (uint32_t)min((uint64_t)g.S, g.rows - (uint64_t)(seg0 + s) * g.S) >> 3;
        return c * CB < nb ? min(CB, nb - c * CB) : 0u;
    };
    const uint32_t ups0 = (CR * D * WB + 15) / 16;
    const uint64_t ups_magic = ((1ull << 32) + ups0 - 1) / ups0;

    // bounded views: offset table, this workgroup's container span, its output rows
    const Buf tab = make_buf(src + 64, 8u * (g.nseg + 1));
    auto tab_ld = [&](uint32_t k) -> uint64_t {
        return (uint64_t)buf_ld32(tab, 8 * k) | ((uint64_t)buf_ld32(tab, 8 * k + 4) << 32);
    };
    const uint64_t a_wg = uniform64(tab_ld(seg0));
    const uint64_t b_wg = uniform64(tab_ld(seg0 + nsw));
    const bool wg_ok = a_wg <= b_wg && b_wg <= g.data_bytes && b_wg - a_wg <= 0x7FFFFFF0ull;
    const Buf in = make_buf(src + g.data_start + (wg_ok ? a_wg : 0), wg_ok ? (uint32_t)(b_wg - a_wg) : 0u);
    const uint64_t wrow0 = (uint64_t)seg0 * g.S;
    const uint64_t wrows = min((uint64_t)nsw * g.S, g.rows - wrow0);
    const Buf out = make_buf(reinterpret_cast<uint8_t *>(dst) + wrow0 * D * WB, (uint32_t)(wrows * D * WB));

    // staging: issue loads of the windows described by slot state st into regs
    u32x4 reg[kStagePerThread];
    auto stage_issue = [&](const SegSlot *st) {
#pragma unroll
        for (int t = 0; t < kStagePerThread; ++t) {
            const uint32_t u = tid + (uint32_t)t * kThreads;
            u32x4 v = {0u, 0u, 0u, 0u};
            if (u < nsw * sg.nu) {
                const uint32_t s = (uint32_t)(((uint64_t)u * sg.nu_magic) >> 32);
                const uint32_t k = u - s * sg.nu;
                const SegSlot &sl = st[s];
                if (sl.ok) {
                    const uint32_t off = k < sg.hu ? sl.hbase + 16 * k : sl.pbase + 16 * (k - sg.hu);
                    v = buf_ld128(in, sl.ra + off);
                }
            }
            reg[t] = v;
        }
    };
    auto stage_commit = [&](u32x4 *buf) {
#pragma unroll
        for (int t = 0; t < kStagePerThread; ++t) {
            const uint32_t u = tid + (uint32_t)t * kThreads;
            if (u < nsw * sg.nu) buf[u] = reg[t];
        }
    };
    auto window_bases = [&](SegSlot &sl) {
        sl.hbase = (4 + (uint32_t)(((uint64_t)sl.r * D * HB) >> 3)) & ~15u;
        sl.pbase = sl.cursor & ~15u;
    };

    // ---- per-segment setup ----------------------------------------------
    if (tid < SPW) {
        SegSlot sl;
        sl.ok = 0; sl.nblk = 0; sl.tail = 0; sl.nrec = 0; sl.ext = 0; sl.ra = 0;
        sl.r = 0; sl.cursor = 0; sl.rle_rem = 0; sl.hbase = 0; sl.pbase = 0;
        if (tid < nsw) {
            const uint32_t seg = seg0 + tid;
            const uint64_t a = tab_ld(seg);
            const uint64_t b = tab_ld(seg + 1);
            const uint32_t nr = (uint32_t)min((uint64_t)g.S, g.rows - (uint64_t)seg * g.S);
            sl.nblk = nr >> 3;
            sl.tail = nr & 7u;
            if (wg_ok && a_wg <= a && a <= b && b <= b_wg && !((a | b) & 15u) && b - a >= 16) {
                sl.ra = (uint32_t)(a - a_wg);
                sl.ext = (uint32_t)(b - a);
                sl.nrec = buf_ld32(in, sl.ra);
                sl.cursor = 4 + (uint32_t)(((uint64_t)sl.nrec * D * HB + 7) >> 3);
                sl.ok = sl.nrec <= sl.nblk ? 1u : 0u;
            }
            if (!sl.ok && status) atomicOr(status, 1);
            window_bases(sl);
        }
        slots[0][tid] = sl;
    }
    __syncthreads();
    stage_issue(slots[0]);
    stage_commit(STG);
    __syncthreads();

    // FIRE / delta state of the chain owned by this lane of wave 0
    uint32_t xprev = 0;
    int32_t delta = 0, acc = 0;

    const uint32_t nchunks = ((g.S >> 3) + CB - 1) / CB;
    for (uint32_t c = 0; c < nchunks; ++c) {
        const SegSlot *cur = slots[c & 1];
        SegSlot *nxt = slots[(c + 1) & 1];
        const uint32_t *stw = reinterpret_cast<const uint32_t *>(STG);
        // ---- 1. parse candidate records --------------------------------
        if (tid < SPW * CB) {
            const uint32_t s = tid / CB, k = tid % CB;
            const SegSlot sl = cur[s];
            const uint32_t nb = sl.ok ? sl.nblk : 0u;
            const uint32_t bic = c * CB < nb ? min(CB, nb - c * CB) : 0u;
            const uint32_t hw0 = s * sg.nu * 4;                 // first header word of segment s
            const uint32_t hwl = hw0 + sg.hu * 4 - 2;           // last header word readable as a pair
            const uint32_t pw0 = hw0 + sg.hu * 4;               // first payload word
            const uint32_t pwl = pw0 + sg.pu * 4 - 2;
            auto hbits32 = [&](uint32_t p) -> uint32_t {       // p: bit offset in the header window
                const uint32_t wi = min(hw0 + (p >> 5), hwl);
                return __builtin_amdgcn_alignbit(stw[wi + 1], stw[wi], p & 31u);
            };
            auto pbits32 = [&](uint32_t p) -> uint32_t {       // p: bit offset in the payload window
                const uint32_t wi = min(pw0 + (p >> 5), pwl);
                return __builtin_amdgcn_alignbit(stw[wi + 1], stw[wi], p & 31u);
            };
            const uint32_t rr = sl.r + k;
            const bool cand = bic > 0 && rr < sl.nrec;
            uint32_t total = 0;
            if (cand) {
                const uint32_t hp = 32 + rr * D * HB - 8 * sl.hbase;
                uint32_t win = 0;
                for (uint32_t j = 0; j < D; ++j) {
                    const uint32_t jj = j % CPW;
                    if (jj == 0) win = hbits32(hp + j * HB);
                    const uint32_t code = __builtin_amdgcn_ubfe(win, jj * HB, HB);
                    const uint32_t width = code < (uint32_t)W - 1 ? code : (uint32_t)W;
                    colmeta[(s * CB + k) * Dp + j] = (COLMAJOR ? 8 * total : total) | (width << 24);
                    total += width;
                }
            }
            const bool zero = cand && total == 0;
            const uint32_t size = !cand ? 0u : zero ? 2u : (COLMAJOR ? total : 8 * ((total + 7) >> 3));
            const uint32_t incl = group_incl_sum(size, CB, k);
            const uint32_t off = sl.cursor + incl - size;        // segment byte offset of the payload
            uint32_t nblocks = 0;
            if (cand) nblocks = zero ? (pbits32(8 * (off - sl.pbase)) & 0xFFFFu) : 1u;
            const bool bad = cand && (nblocks == 0 || off + size > sl.ext);
            const uint32_t bincl = group_incl_sum(nblocks, CB, k);
            const uint32_t start = sl.rle_rem + bincl - nblocks;
            const uint32_t end = start + nblocks;
            const bool used = cand && start < bic;
            if (used) {
                recbits[s * CB + k] = 8 * (off - sl.pbase);
                recstride[s * CB + k] = 8 * ((total + 7) >> 3);
                const uint32_t mark = zero ? kRleMark : k;
                for (uint32_t q = start; q < min(end, bic); ++q) blkrec[s * CB + q] = mark;
            }
            if (k == 0)
                for (uint32_t q = 0; q < min(sl.rle_rem, bic); ++q) blkrec[s * CB + q] = kRleMark;
            // new segment state: records used, payload consumed, carried run
            const uint32_t nused = group_incl_sum(used ? 1u : 0u, CB, k);
            const uint32_t n_used = group_last(nused, CB);
            const uint32_t used_size = group_last(group_incl_sum(used ? size : 0u, CB, k), CB);
            const uint32_t last_end = group_last(group_incl_sum(used && nused == n_used ? end : 0u, CB, k), CB);
            const uint32_t any_bad = group_last(group_incl_sum(used && bad ? 1u : 0u, CB, k), CB);
            if (k == 0) {
                SegSlot ns = sl;
                if (bic > 0) {
                    ns.r = sl.r + n_used;
                    ns.cursor = sl.cursor + used_size;
                    const uint32_t covered = n_used ? last_end : sl.rle_rem;
                    if (covered < bic || any_bad) {
                        ns.ok = 0;  // records ran out, a zero run count, or a payload past the segment
                        if (status) atomicOr(status, 1);
                    }
                    ns.rle_rem = covered >= bic ? covered - bic : 0u;
                    window_bases(ns);
                }
                nxt[s] = ns;
            }
        }
        __syncthreads();

        // ---- 2. stage the next chunk; unpack this one --------------------
        if (c + 1 < nchunks) stage_issue(nxt);
#pragma unroll
        for (int ti = 0; ti < kUnpackPerThread; ++ti) {
            const uint32_t it = tid + (uint32_t)ti * kThreads;
            const uint32_t j = it & (Dp - 1);
            const uint32_t q = (it >> lg) % CB;
            const uint32_t s = (it >> lg) / CB;
            if (s >= nsw || j >= D || q >= blocks_in_chunk(s, c)) continue;
            int32_t *e = &E[(s * Dp + j) * kChainStride + q * 8];
            const uint32_t k = blkrec[s * CB + q];
            int32_t v[8];
            if (k >= CB || !nxt[s].ok) {
#pragma unroll
                for (int i = 0; i < 8; ++i) v[i] = 0;
            } else {
                const uint32_t pw0 = s * sg.nu * 4 + sg.hu * 4;
                const uint32_t pwl = pw0 + sg.pu * 4 - 2;
                const uint32_t cm = colmeta[(s * CB + k) * Dp + j];
                const uint32_t width = cm >> 24;
                const uint32_t p0 = recbits[s * CB + k] + (cm & 0xFFFFFFu);
                const uint32_t stride = COLMAJOR ? width : recstride[s * CB + k];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const uint32_t p = p0 + (uint32_t)i * stride;
                    const uint32_t wi = min(pw0 + (p >> 5), pwl);
                    const uint32_t z =
                        __builtin_amdgcn_ubfe(__builtin_amdgcn_alignbit(stw[wi + 1], stw[wi], p & 31u), 0u, width);
                    const int32_t er = unzigzag(z);
                    v[i] = FIRE ? (int32_t)((uint32_t)er << W) : er;
                }
            }
            *reinterpret_cast<int4 *>(e) = make_int4(v[0], v[1], v[2], v[3]);
            *reinterpret_cast<int4 *>(e + 4) = make_int4(v[4], v[5], v[6], v[7]);
        }
        __syncthreads();

        // ---- 3. serial recurrence (wave 0) ------------------------------
        if (tid < 64) {
            const uint32_t s = tid >> lg, j = tid & (Dp - 1);
            const uint32_t bic = s < nsw ? blocks_in_chunk(s, c) : 0u;
            if (j < D) {
                int32_t *e = &E[tid * kChainStride];
                for (uint32_t q = 0; q < bic; ++q) {
                    int4 a = *reinterpret_cast<int4 *>(e + q * 8);
                    int4 b = *reinterpret_cast<int4 *>(e + q * 8 + 4);
                    int32_t v[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
                    if (FIRE) {
                        const int32_t alpha = acc >> g.sh;
                        int32_t grad = 0;
#pragma unroll
                        for (int i = 0; i < 8; ++i) {
                            // low 32 bits of alpha * delta + e * 2^w (both factors fit 24 bits)
                            const int32_t tt = (int32_t)((uint32_t)__mul24(alpha, delta) + (uint32_t)v[i]);
                            const int32_t dn = __builtin_amdgcn_sbfe(tt, (uint32_t)W, (uint32_t)W);
                            if (i & 1) grad += __mul24(sgn_med3(v[i]), delta);
                            delta = dn;
                            xprev += (uint32_t)dn;
                            v[i] = (int32_t)xprev;
                        }
                        acc = min(max(acc + grad, g.acc_lo), g.acc_hi);
                    } else {
#pragma unroll
                        for (int i = 0; i < 8; ++i) {
                            xprev += (uint32_t)v[i];
                            v[i] = (int32_t)xprev;
                        }
                    }
                    *reinterpret_cast<int4 *>(e + q * 8) = make_int4(v[0], v[1], v[2], v[3]);
                    *reinterpret_cast<int4 *>(e + q * 8 + 4) = make_int4(v[4], v[5], v[6], v[7]);
                }
            }
        }
        __syncthreads();

        // ---- 4. output: row-major, 16-byte units; commit the staging ----
        {
            constexpr uint32_t VPU = 16 / WB;             // values per 16-byte unit
            const uint32_t ups = (CR * D * WB + 15) / 16;  // units per full chunk of one segment
            for (uint32_t u = tid; u < nsw * ups; u += kThreads) {
                const uint32_t s = (uint32_t)(((uint64_t)u * ups_magic) >> 32);  // u / ups
                const uint32_t f0 = (u - s * ups) * VPU;
                const uint32_t nvals = blocks_in_chunk(s, c) * 8 * D;
                if (f0 >= nvals) continue;
                uint32_t row = (uint32_t)(((uint64_t)f0 * div_magic) >> 32);  // f0 / D
                uint32_t j = f0 - row * D;
                uint32_t w4[4] = {0, 0, 0, 0};
#pragma unroll
                for (uint32_t t = 0; t < VPU; ++t) {
                    // rows past the chunk read padding of the same chain: harmless, never stored
                    const uint32_t x = (uint32_t)E[(s * Dp + j) * kChainStride + min(row, (uint32_t)kChunkRows - 1)];
                    w4[t / (4 / WB)] |= (x & ((1u << W) - 1)) << (W * (t % (4 / WB)));
                    const bool wrap = ++j == D;
                    j = wrap ? 0u : j;
                    row += wrap ? 1u : 0u;
                }
                const uint32_t obase = (s * g.S + c * CR) * D * WB;  // byte offset in the workgroup's rows
                if (f0 + VPU <= nvals) {
                    u32x4 v4 = {w4[0], w4[1], w4[2], w4[3]};
                    buf_st128(out, obase + f0 * WB, v4);
                } else {
                    for (uint32_t t = 0; t < nvals - f0; ++t) {
                        const uint32_t x = w4[t / (4 / WB)] >> (W * (t % (4 / WB)));
                        if (WB == 1) buf_st8(out, obase + (f0 + t), x);
                        else buf_st16(out, obase + (f0 + t) * 2, x);
                    }
                }
            }
        }
        // this chunk's windows were last read by the unpack: reuse the buffer
        if (c + 1 < nchunks) stage_commit(STG);
        __syncthreads();
    }

    // ---- raw tail rows and final checks ---------------------------------
    if (tid < nsw) {
        const SegSlot sl = slots[nchunks & 1][tid];
        if (sl.ok) {
            const uint32_t tb = sl.tail * D * WB;
            if (sl.r != sl.nrec || sl.rle_rem != 0 || sl.cursor + tb > sl.ext) {
                if (status) atomicOr(status, 1);
            } else {
                const uint32_t obase = (tid * g.S + sl.nblk * 8) * D * WB;
                for (uint32_t t = 0; t < tb; ++t) {
                    const uint32_t pos = sl.ra + sl.cursor + t;
                    buf_st8(out, obase + t, buf_ld32(in, pos & ~3u) >> (8 * (pos & 3u)));
                }
            }
        }
    }
}

}  // namespace spz

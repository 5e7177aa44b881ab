// Chunked, phase-split Sprintz encoder for gfx950 (header group = whole
// segment).
//
// Paper: Algorithm 1 (encodeBlock) for every 8-row block; forecasters of
// Section 4.2 with FIRE's practical changes (alpha once per block, one summed
// gradient update per block from every other sample, Section 4.2.2); zigzag,
// per-column bit widths, log2(w)-bit headers, column- or row-major payloads
// (Section 4.3); runs of all-zero blocks become run-length records.
//
// Compression has one serial dependence: FIRE's coefficient of block b+1
// needs the residual signs of block b. Everything else is data parallel, so
// a workgroup of 64 column chains (64 / Dp segments) walks its segments in
// chunks of up to 8 blocks:
//   stage   16-byte loads of the chunk's rows into LDS (issued one chunk ahead)
//   delta   (lanes = segment, block, column): delta_i = sext(x_i - x_{i-1})
//   alpha   (one wavefront, lane = chain, FIRE only): the coefficient chain
//   resid   (lanes = segment, block, column): e_i, zigzag, bit width; group
//           sums over the columns give each column's bit offset
//   records (lanes = segment, block): runs, records, payload offsets
//   pack    (WRITE pass only): fields OR-ed into an LDS staging buffer, then
//           copied to the container; headers go out when the segment ends.
// The size pass (WRITE = false) reports each segment's byte size and record
// count; a scan turns them into the offset table; the write pass repeats the
// walk and writes every byte of each segment exactly once.
#pragma once

#include "spz_device.h"

namespace spz {

constexpr int kEncChunkBlocks = 8;                    // blocks per chunk per segment (max)
constexpr int kEncChunkRows = kEncChunkBlocks * 8;    // 64
constexpr int kEncChainStride = kEncChunkRows + 4;    // dwords per chain in LDS (bank padding)
constexpr int kEncXsBytes = 64 * kEncChunkRows * 2;   // staged input rows (64 chains, 16-bit)
constexpr int kEncOutWords = 3072;                    // payload staging (12 KiB)
constexpr int kEncHdrBytes = 8192;                    // whole-segment header arrays of the workgroup
constexpr int kEncItemsPerThread = 64 * kEncChunkBlocks / kThreads;

struct EncSlot {
    uint32_t nblk, tail;
    uint32_t r;         // records emitted so far
    uint32_t cursor;    // payload bytes emitted so far
    uint32_t run;       // zero blocks pending (not yet emitted)
    uint32_t nrec_total, hdr_bytes;  // write pass: from the size pass
    uint32_t pad;
    uint64_t base;      // write pass: container byte offset of the segment
};

__host__ __device__ inline uint32_t enc_chunk_blocks(uint32_t) { return (uint32_t)kEncChunkBlocks; }

// Header bytes of a whole segment with nblk blocks at most (fast-path limit).
__host__ __device__ inline uint32_t enc_hdr_cap(uint32_t nblk, uint32_t D, uint32_t w) {
    return (nblk * D * (w == 8 ? 3u : 4u) + 7) / 8 + 4;
}

template <int W, bool FIRE, bool COLMAJOR, bool WRITE>
__global__ __launch_bounds__(kThreads) void k_encode_chunked(const uint8_t *__restrict__ src, Geom g,
                                                             uint32_t *__restrict__ seg_info,
                                                             uint8_t *__restrict__ dst,
                                                             int32_t *__restrict__ status) {
    constexpr uint32_t HB = W == 8 ? 3 : 4;
    constexpr uint32_t WB = W / 8;

    __shared__ u32x4 XS[kEncXsBytes / 16];              // staged rows: [segment][row][column]
    __shared__ int32_t DL[64 * kEncChainStride];        // [chain][row]: delta, then zigzag code
    __shared__ int32_t ALPHA[64 * kEncChunkBlocks];     // [chain][block]
    __shared__ uint32_t CM[64 * kEncChunkBlocks];       // [segment][block][column]: code | width<<8 | off<<16
    __shared__ uint32_t BW[64 * kEncChunkBlocks];       // [segment][block]: summed width of the block
    __shared__ uint32_t BREC[64 * kEncChunkBlocks];     // [segment][block]: record index of the block
    __shared__ uint32_t BOFF[64 * kEncChunkBlocks];     // [segment][block]: payload byte offset (chunk-relative)
    __shared__ uint32_t BRUN[64 * kEncChunkBlocks];     // [segment][block]: zero blocks emitted before it
    __shared__ uint32_t PREVX[2][64];                   // last sample of the previous chunk, per chain
    __shared__ int32_t PREVD[2][64];                    // last delta of the previous chunk, per chain
    __shared__ uint32_t OUTP[kEncOutWords];             // chunk payload bytes, per segment
    __shared__ uint32_t OUTH[kEncHdrBytes / 4];         // header arrays, per segment
    __shared__ EncSlot slots[64];

    const uint32_t tid = threadIdx.x;
    const uint32_t lg = g.dp_log2;
    const uint32_t Dp = 1u << lg;
    const uint32_t SPW = 64u >> lg;
    const uint32_t CB = enc_chunk_blocks(lg);
    const uint32_t CR = CB * 8;
    const uint32_t D = g.D;
    const uint32_t seg0 = blockIdx.x * SPW;
    const uint32_t nsw = min(SPW, g.nseg - seg0);
    const uint32_t xs_seg = CR * D * WB;                        // staged bytes per segment
    const uint32_t out_seg = (CB * 8 * D * WB + 6 * CB + 15) & ~15u;  // payload staging bytes per segment
    const uint32_t hdr_seg = (enc_hdr_cap(g.S >> 3, D, W) + 15) & ~15u;
    // container words one segment's chunk payload can touch (a misaligned
    // start adds one), and the magic multiplier dividing by that count
    const uint32_t out_wps = out_seg / 4 + 1;
    const uint64_t wps_magic = ((1ull << 32) + out_wps - 1) / out_wps;

    // bounded views: this workgroup's input rows and the whole container
    const uint64_t wrow0 = (uint64_t)seg0 * g.S;
    const uint64_t wrows = min((uint64_t)nsw * g.S, g.rows - wrow0);
    const uint32_t in_bytes = (uint32_t)(wrows * D * WB);
    const Buf in = make_buf(src + wrow0 * D * WB, in_bytes);
    auto blocks_in_chunk = [&](uint32_t s, uint32_t c) -> uint32_t {
        const uint32_t nb = (uint32_t)min((uint64_t)g.S, g.rows - (uint64_t)(seg0 + s) * g.S) >> 3;
        return c * CB < nb ? min(CB, nb - c * CB) : 0u;
    };

    // ---- setup --------------------------------------------------------------
    if (tid < SPW) {
        EncSlot sl;
        sl.nblk = 0; sl.tail = 0; sl.r = 0; sl.cursor = 0; sl.run = 0; sl.nrec_total = 0; sl.hdr_bytes = 0;
        sl.pad = 0; sl.base = 0;
        if (tid < nsw) {
            const uint32_t seg = seg0 + tid;
            const uint32_t nr = (uint32_t)min((uint64_t)g.S, g.rows - (uint64_t)seg * g.S);
            sl.nblk = nr >> 3;
            sl.tail = nr & 7u;
            if (WRITE) {
                sl.nrec_total = seg_info[2 * seg + 1];
                sl.hdr_bytes = (uint32_t)(((uint64_t)sl.nrec_total * D * HB + 7) >> 3);
                sl.base = g.data_start + ld_u64_aligned(dst + 64 + 8ull * seg);
            }
        }
        slots[tid] = sl;
    }
    for (uint32_t k = tid; k < kEncOutWords; k += kThreads) OUTP[k] = 0;
    if (WRITE)
        for (uint32_t k = tid; k < kEncHdrBytes / 4; k += kThreads) OUTH[k] = 0;
    if (tid < 64) { PREVX[0][tid] = 0; PREVD[0][tid] = 0; }

    // staging of a chunk's input rows: 16-byte units, issued one chunk ahead
    constexpr int kStPer = (kEncXsBytes / 16 + kThreads - 1) / kThreads;
    u32x4 reg[kStPer];
    const uint32_t units_seg = xs_seg / 16;
    const uint64_t us_magic = ((1ull << 32) + units_seg - 1) / units_seg;
    auto stage_issue = [&](uint32_t c) {
#pragma unroll
        for (int t = 0; t < kStPer; ++t) {
            const uint32_t u = tid + (uint32_t)t * kThreads;
            u32x4 v = {0u, 0u, 0u, 0u};
            if (u < nsw * units_seg) {
                const uint32_t s = (uint32_t)(((uint64_t)u * us_magic) >> 32);
                const uint32_t k = u - s * units_seg;
                const uint32_t off = (s * g.S + c * CR) * D * WB + 16 * k;
                if (off + 16 <= in_bytes) {
                    v = buf_ld128(in, off);
                } else if (off < in_bytes) {
                    // the unit crosses the end of the input: block rows end on
                    // an 8-byte boundary, so every dword they use is whole
                    v.x = buf_ld32(in, off);
                    v.y = buf_ld32(in, off + 4);
                    v.z = buf_ld32(in, off + 8);
                    v.w = buf_ld32(in, off + 12);
                }
            }
            reg[t] = v;
        }
    };
    auto stage_commit = [&]() {
#pragma unroll
        for (int t = 0; t < kStPer; ++t) {
            const uint32_t u = tid + (uint32_t)t * kThreads;
            if (u < nsw * units_seg) XS[u] = reg[t];
        }
    };
    const uint8_t *xsb = reinterpret_cast<const uint8_t *>(XS);
    auto xs_val = [&](uint32_t s, uint32_t row, uint32_t j) -> uint32_t {
        const uint32_t off = s * xs_seg + (row * D + j) * WB;
        return WB == 1 ? (uint32_t)xsb[off] : (uint32_t)*reinterpret_cast<const uint16_t *>(xsb + off);
    };

    stage_issue(0);
    __syncthreads();
    stage_commit();
    __syncthreads();

    // FIRE coefficient chain of the lane's column (wave 0)
    int32_t acc = 0;
    uint32_t any_err = 0;

    const uint32_t nchunks = ((g.S >> 3) + CB - 1) / CB;
    for (uint32_t c = 0; c < nchunks; ++c) {
        const uint32_t par = c & 1;
        // ---- delta phase ----------------------------------------------------
#pragma unroll
        for (int ti = 0; ti < kEncItemsPerThread; ++ti) {
            const uint32_t it = tid + (uint32_t)ti * kThreads;
            const uint32_t j = it & (Dp - 1);
            const uint32_t q = (it >> lg) % CB;
            const uint32_t s = (it >> lg) / CB;
            if (s >= nsw || j >= D) continue;
            const uint32_t bic = blocks_in_chunk(s, c);
            if (q >= bic) continue;
            const uint32_t ch = s * Dp + j;
            uint32_t xp = q == 0 ? PREVX[par][ch] : xs_val(s, 8 * q - 1, j);
            int32_t d[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const uint32_t x = xs_val(s, 8 * q + i, j);
                d[i] = sext<W>((int32_t)(x - xp));
                xp = x;
            }
            int32_t *dl = &DL[ch * kEncChainStride + 8 * q];
            *reinterpret_cast<int4 *>(dl) = make_int4(d[0], d[1], d[2], d[3]);
            *reinterpret_cast<int4 *>(dl + 4) = make_int4(d[4], d[5], d[6], d[7]);
            if (q == bic - 1) {
                PREVX[par ^ 1][ch] = xp;
                PREVD[par ^ 1][ch] = d[7];
            }
        }
        __syncthreads();
        if (c + 1 < nchunks) stage_issue(c + 1);

        // ---- FIRE coefficient chain (wave 0) ------------------------------
        if (FIRE && tid < 64) {
            const uint32_t s = tid >> lg, j = tid & (Dp - 1);
            const uint32_t bic = s < nsw && j < D ? blocks_in_chunk(s, c) : 0u;
            const int32_t *dl = &DL[tid * kEncChainStride];
            for (uint32_t q = 0; q < bic; ++q) {
                const int4 a = *reinterpret_cast<const int4 *>(dl + 8 * q);
                const int4 b = *reinterpret_cast<const int4 *>(dl + 8 * q + 4);
                const int32_t d[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
                const int32_t alpha = acc >> g.sh;
                ALPHA[tid * kEncChunkBlocks + q] = alpha;
                int32_t grad = 0;
#pragma unroll
                for (int i = 1; i < 8; i += 2) {
                    const int32_t e = sext<W>(d[i] - (__mul24(alpha, d[i - 1]) >> W));
                    grad += __mul24(sgn_med3(e), d[i - 1]);
                }
                acc = min(max(acc + grad, g.acc_lo), g.acc_hi);
            }
        }
        __syncthreads();

        // ---- residual phase: zigzag codes and bit widths ------------------
        // Codes replace the deltas in place once every item has read its
        // inputs (an item reads the last delta of the block before it).
        uint32_t zr[kEncItemsPerThread][8];
        bool zw[kEncItemsPerThread];
#pragma unroll
        for (int ti = 0; ti < kEncItemsPerThread; ++ti) {
            zw[ti] = false;
            const uint32_t it = tid + (uint32_t)ti * kThreads;
            const uint32_t j = it & (Dp - 1);
            const uint32_t q = (it >> lg) % CB;
            const uint32_t s = (it >> lg) / CB;
            // whole lane groups (one segment block) stay together for the scan
            const uint32_t bic = s < nsw ? blocks_in_chunk(s, c) : 0u;
            if (q >= bic) continue;
            const uint32_t ch = s * Dp + j;
            uint32_t orz = 0;
            if (j < D) {
                const int32_t *dl = &DL[ch * kEncChainStride + 8 * q];
                const int4 a = *reinterpret_cast<const int4 *>(dl);
                const int4 b = *reinterpret_cast<const int4 *>(dl + 4);
                const int32_t d[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
                int32_t dm = q == 0 ? PREVD[par][ch] : dl[-1];
                const int32_t alpha = FIRE ? ALPHA[ch * kEncChunkBlocks + q] : 0;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int32_t e = FIRE ? sext<W>(d[i] - (__mul24(alpha, dm) >> W)) : d[i];
                    dm = d[i];
                    zr[ti][i] = zigzag(e);
                    orz |= zr[ti][i];
                }
                zw[ti] = true;
            }
            const uint32_t code = min(bitlen(orz), (uint32_t)W - 1);
            const uint32_t width = code < (uint32_t)W - 1 ? code : (uint32_t)W;
            const uint32_t incl = group_incl_sum(width, Dp, j);
            if (j < D) CM[(s * CB + q) * Dp + j] = code | (width << 8) | ((incl - width) << 16);
            if (j == Dp - 1) BW[s * CB + q] = incl;
        }
        __syncthreads();
#pragma unroll
        for (int ti = 0; ti < kEncItemsPerThread; ++ti) {
            if (!zw[ti]) continue;
            const uint32_t it = tid + (uint32_t)ti * kThreads;
            const uint32_t j = it & (Dp - 1);
            const uint32_t q = (it >> lg) % CB;
            const uint32_t s = (it >> lg) / CB;
            int32_t *dl = &DL[(s * Dp + j) * kEncChainStride + 8 * q];
            *reinterpret_cast<int4 *>(dl) = make_int4((int)zr[ti][0], (int)zr[ti][1], (int)zr[ti][2], (int)zr[ti][3]);
            *reinterpret_cast<int4 *>(dl + 4) = make_int4((int)zr[ti][4], (int)zr[ti][5], (int)zr[ti][6], (int)zr[ti][7]);
        }
        __syncthreads();

        // ---- records: runs, record indices, payload offsets ----------------
        // lanes = (segment, block); whole lane groups of CB stay together
        for (uint32_t rl = tid; rl < SPW * CB; rl += kThreads) {
            const uint32_t s = rl / CB, q = rl % CB;
            const uint32_t bic = s < nsw ? blocks_in_chunk(s, c) : 0u;
            const EncSlot sl = slots[s];
            const bool act = q < bic;
            const uint32_t wsum = act ? BW[s * CB + q] : 0u;
            const bool nz = act && wsum != 0;
            // last nonzero block before q in this chunk (or -1): max-scan
            int32_t last = nz ? (int32_t)q : -1;
            for (uint32_t k = 1; k < CB; k <<= 1) {
                const int32_t t = __shfl_up(last, k, (int)CB);
                if (q >= k) last = max(last, t);
            }
            int32_t prev_nz = __shfl_up(last, 1, (int)CB);
            if (q == 0) prev_nz = -1;
            const uint32_t run = nz ? (prev_nz < 0 ? sl.run + q : q - (uint32_t)prev_nz - 1) : 0u;
            const uint32_t nrle = (run + kRleMax - 1) / kRleMax;
            const uint32_t size = COLMAJOR ? wsum : 8 * ((wsum + 7) >> 3);
            const uint32_t nrec_q = nz ? nrle + 1 : 0u;
            const uint32_t pay_q = nz ? 2 * nrle + size : 0u;
            const uint32_t rinc = group_incl_sum(nrec_q, CB, q);
            const uint32_t pinc = group_incl_sum(pay_q, CB, q);
            if (nz) {
                BREC[s * CB + q] = sl.r + rinc - 1;       // record index of the block itself
                BOFF[s * CB + q] = pinc - pay_q;          // chunk-relative payload offset (its runs first)
                BRUN[s * CB + q] = run;
            }
            const int32_t last_all = __shfl(last, (int)(CB - 1), (int)CB);
            const uint32_t nrec_c = group_last(rinc, CB);
            const uint32_t pay_c = group_last(pinc, CB);
            if (q == 0 && s < nsw) {
                EncSlot ns = sl;
                if (bic > 0) {
                    ns.r = sl.r + nrec_c;
                    ns.cursor = sl.cursor + pay_c;
                    ns.run = last_all < 0 ? sl.run + bic : bic - 1 - (uint32_t)last_all;
                }
                // pass-through of the payload start of this chunk for the pack phase
                ns.pad = sl.cursor;
                slots[s] = ns;
            }
        }
        __syncthreads();

        if (WRITE) {
            // ---- pack: payload fields and header codes into LDS ------------
#pragma unroll
            for (int ti = 0; ti < kEncItemsPerThread; ++ti) {
                const uint32_t it = tid + (uint32_t)ti * kThreads;
                const uint32_t j = it & (Dp - 1);
                const uint32_t q = (it >> lg) % CB;
                const uint32_t s = (it >> lg) / CB;
                if (s >= nsw || j >= D) continue;
                if (q >= blocks_in_chunk(s, c)) continue;
                const uint32_t wsum = BW[s * CB + q];
                if (wsum == 0) continue;
                uint32_t *op = &OUTP[s * (out_seg / 4)];
                const uint32_t boff = BOFF[s * CB + q];
                const uint32_t run = BRUN[s * CB + q];
                const uint32_t nrle = (run + kRleMax - 1) / kRleMax;
                if (j == 0) {
                    for (uint32_t k = 0; k < nrle; ++k) {
                        const uint32_t cnt = k + 1 < nrle ? kRleMax : run - kRleMax * (nrle - 1);
                        const uint32_t pb = 8 * (boff + 2 * k);
                        atomicOr(&op[pb >> 5], cnt << (pb & 31));
                        if ((pb & 31) > 16) atomicOr(&op[(pb >> 5) + 1], cnt >> (32 - (pb & 31)));
                    }
                }
                const uint32_t cm = CM[(s * CB + q) * Dp + j];
                const uint32_t code = cm & 0xFF, width = (cm >> 8) & 0xFF, off = cm >> 16;
                const uint32_t rec = BREC[s * CB + q];
                if (code != 0) {
                    const uint32_t hp = (rec * D + j) * HB;
                    uint32_t *hh = &OUTH[s * (hdr_seg / 4)];
                    atomicOr(&hh[hp >> 5], code << (hp & 31));
                    if ((hp & 31) + HB > 32) atomicOr(&hh[(hp >> 5) + 1], code >> (32 - (hp & 31)));
                }
                if (width == 0) continue;
                const uint32_t pstart = 8 * (boff + 2 * nrle);
                const int32_t *dl = &DL[(s * Dp + j) * kEncChainStride + 8 * q];
                const uint32_t rbits = 8 * ((wsum + 7) >> 3);
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const uint32_t z = (uint32_t)dl[i];
                    const uint32_t p = COLMAJOR ? pstart + 8 * off + (uint32_t)i * width : pstart + (uint32_t)i * rbits + off;
                    atomicOr(&op[p >> 5], z << (p & 31));
                    if ((p & 31) + width > 32) atomicOr(&op[(p >> 5) + 1], z >> (32 - (p & 31)));
                }
            }
            __syncthreads();

            // ---- payload bytes out; clear the staging -----------------------
            // staging byte b of segment s belongs at container byte o0 + b;
            // lanes = (segment, container word), all segments at once
            for (uint32_t it = tid; it < nsw * out_wps; it += kThreads) {
                const uint32_t s = (uint32_t)(((uint64_t)it * wps_magic) >> 32);
                const uint32_t k = it - s * out_wps;
                const EncSlot sl = slots[s];
                const uint32_t n = sl.cursor - sl.pad;     // payload bytes of this chunk
                const uint64_t o0 = sl.base + 4 + sl.hdr_bytes + sl.pad;
                const uint32_t mis = (uint32_t)(o0 & 3);
                const uint32_t nw = n == 0 ? 0u : (mis + n + 3) >> 2;    // container words touched
                if (k >= nw) continue;
                const uint32_t *op = &OUTP[s * (out_seg / 4)];
                // container word k holds staging bytes 4k - mis .. 4k - mis + 3
                const uint32_t cur = k < (n + 3) / 4 ? op[k] : 0u;
                const uint32_t word = mis == 0 ? cur
                                               : __builtin_amdgcn_alignbit(cur, k > 0 ? op[k - 1] : 0u, 8 * (4 - mis));
                const uint64_t addr = (o0 & ~3ull) + 4ull * k;
                const int32_t b0 = 4 * (int32_t)k - (int32_t)mis;
                if (b0 >= 0 && (uint32_t)b0 + 4 <= n) {
                    if (addr + 4 <= g.cap) *reinterpret_cast<uint32_t *>(dst + addr) = word;
                    else any_err = 1;
                } else {
                    for (uint32_t t = 0; t < 4; ++t) {
                        const int32_t bb = b0 + (int32_t)t;
                        if (bb < 0 || (uint32_t)bb >= n) continue;
                        if (addr + t < g.cap) dst[addr + t] = (uint8_t)(word >> (8 * t));
                        else any_err = 1;
                    }
                }
            }
            __syncthreads();
            for (uint32_t k = tid; k < nsw * (out_seg / 4); k += kThreads) OUTP[k] = 0;
        }
        if (c + 1 < nchunks) stage_commit();
        __syncthreads();
    }

    // ---- segment end: trailing run, sizes or final bytes ------------------------
    if (tid < nsw) {
        EncSlot sl = slots[tid];
        const uint32_t seg = seg0 + tid;
        const uint32_t nrle = (sl.run + kRleMax - 1) / kRleMax;
        const uint32_t nrec = sl.r + nrle;
        const uint32_t tail_bytes = sl.tail * D * WB;
        const uint32_t hdr = (uint32_t)(((uint64_t)nrec * D * HB + 7) >> 3);
        const uint32_t size = (4 + hdr + sl.cursor + 2 * nrle + tail_bytes + 15) & ~15u;
        if (!WRITE) {
            seg_info[2 * seg] = size;
            seg_info[2 * seg + 1] = nrec;
        } else {
            if (nrec != sl.nrec_total || size != seg_info[2 * seg]) any_err = 1;
            // trailing run records: counts after the chunked payload
            for (uint32_t k = 0; k < nrle; ++k) {
                const uint32_t cnt = k + 1 < nrle ? kRleMax : sl.run - kRleMax * (nrle - 1);
                const uint64_t p = sl.base + 4 + hdr + sl.cursor + 2 * k;
                if (p + 2 <= g.cap) { dst[p] = (uint8_t)cnt; dst[p + 1] = (uint8_t)(cnt >> 8); }
                else any_err = 1;
            }
            if (sl.base + 4 <= g.cap) *reinterpret_cast<uint32_t *>(dst + sl.base) = nrec;
            else any_err = 1;
            sl.cursor += 2 * nrle;   // payload bytes including the trailing run
            sl.pad = size;
            slots[tid] = sl;
        }
    }
    if (WRITE) {
        __syncthreads();
        // header arrays (dword aligned start); lanes = (segment, header word)
        const uint32_t hwps = hdr_seg / 4;
        const uint64_t hw_magic = ((1ull << 32) + hwps - 1) / hwps;
        for (uint32_t it = tid; it < nsw * hwps; it += kThreads) {
            const uint32_t s = (uint32_t)(((uint64_t)it * hw_magic) >> 32);
            const uint32_t k = it - s * hwps;
            const EncSlot sl = slots[s];
            const uint32_t hdr = sl.hdr_bytes;
            if (4 * k >= hdr) continue;
            const uint32_t hv = OUTH[s * hwps + k];
            const uint64_t addr = sl.base + 4 + 4ull * k;
            if (4 * k + 4 <= hdr) {
                if (addr + 4 <= g.cap) *reinterpret_cast<uint32_t *>(dst + addr) = hv;
                else any_err = 1;
            } else {
                for (uint32_t t = 0; 4 * k + t < hdr; ++t) {
                    if (addr + t < g.cap) dst[addr + t] = (uint8_t)(hv >> (8 * t));
                    else any_err = 1;
                }
            }
        }
        // raw tail rows and zero padding to the 16-byte segment end;
        // lanes = (segment, byte): fewer than 8 rows plus 15 bytes each
        const uint32_t tbps = 7 * D * WB + 16;
        const uint64_t tb_magic = ((1ull << 32) + tbps - 1) / tbps;
        for (uint32_t it = tid; it < nsw * tbps; it += kThreads) {
            const uint32_t s = (uint32_t)(((uint64_t)it * tb_magic) >> 32);
            const uint32_t t = it - s * tbps;
            const EncSlot sl = slots[s];
            const uint32_t seg = seg0 + s;
            const uint32_t tail_bytes = sl.tail * D * WB;
            const uint64_t tpos = sl.base + 4 + sl.hdr_bytes + sl.cursor;
            const uint64_t end = sl.base + sl.pad;
            const uint64_t p = tpos + t;
            if (p >= end) continue;
            const uint64_t trow = (uint64_t)seg * g.S + (uint64_t)sl.nblk * 8;
            uint32_t v = 0;
            if (t < tail_bytes) v = buf_ld8(in, (uint32_t)((trow - wrow0) * D * WB + t));
            if (p < g.cap) dst[p] = (uint8_t)v;
            else any_err = 1;
        }
    }
    if (WRITE && any_err && status) atomicOr(status, 2);
}

}  // namespace spz

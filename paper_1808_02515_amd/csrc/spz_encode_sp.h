// Single-pass Sprintz encoder for gfx950 (header group = whole segment,
// D up to 16).
//
// Paper: Algorithm 1 (encodeBlock) for every 8-row block, the forecasters of
// Section 4.2 (delta coding; FIRE with the practical changes of Section
// 4.2.2: alpha once per block, one summed gradient update per block from
// every other sample), zigzag residuals, per-column bit widths behind
// log2(w)-bit headers and column- or row-major payloads (Section 4.3), runs
// of all-zero blocks as run-length records (Algorithm 1).
//
// Compression has one serial dependence: FIRE's coefficient of block b+1
// needs the residual signs of block b. A workgroup holds SPW = 64 / Dp
// segments (64 column chains) and walks them in chunks of CB blocks with one
// barrier per chunk:
//   alpha wave (FIRE)  chunk t: lane = column chain, the coefficient chain
//                      over the chunk's blocks (registers carry it on)
//   item waves         chunk t-1 (t for delta): lanes = (segment, block,
//                      column): deltas, residuals, zigzag codes and the
//                      column's bit width; DPP sums over the columns of a
//                      block give bit offsets, the record's header code word
//                      and its payload size. Lanes = (segment, block) then
//                      scan the chunk's records (run-length records, record
//                      indices, payload byte offsets). Fields and header
//                      codes are OR-ed into per-segment LDS staging; whole
//                      16-byte units (whole header dwords) go out, the
//                      partial last one stays for the next chunk.
//   item waves also    16-byte loads of chunk t+1's rows into registers,
//                      stored to LDS staging after the chunk's work.
// A wave tile (64 item lanes) covers whole segment-chunks, so the record
// scans and the staging flushes are wave-local: the only workgroup barrier
// is the one per chunk.
//
// Every segment goes to a slot of the workspace: the u32 record count and
// the header array from byte 0, the payload and the raw tail rows from byte
// P0 (the largest header, rounded up). Its sizes go to a 16-byte info record;
// k_enc_scan turns the sizes into the offset table and k_enc_compact copies
// each segment to its place in the container. The input is read once.
//
// Global accesses go through buffer resources bounded to the workgroup's
// input rows, its workspace slots and (compaction) its part of the container.
#pragma once

#include "spz_decode_pc.h"
#include "spz_device.h"

namespace spz {

// item waves of a workgroup (eight measured slower: the record scans and
// flushes then run once per tile instead of once per two tiles)
__host__ __device__ constexpr uint32_t es_item_waves(uint32_t) { return 4u; }
__host__ __device__ constexpr uint32_t es_threads(uint32_t D) { return 64 * (es_item_waves(D) + 1); }

// Inclusive max over an aligned group of N <= 16 lanes (values >= 0).
template <int N> __device__ __forceinline__ uint32_t es_incl_max(uint32_t v, uint32_t i) {
    if constexpr (N >= 2) { const uint32_t t = pc_dpp<0x111>(v); v = i >= 1 ? max(v, t) : v; }
    if constexpr (N >= 4) { const uint32_t t = pc_dpp<0x112>(v); v = i >= 2 ? max(v, t) : v; }
    if constexpr (N >= 8) { const uint32_t t = pc_dpp<0x114>(v); v = i >= 4 ? max(v, t) : v; }
    if constexpr (N >= 16) { const uint32_t t = pc_dpp<0x118>(v); v = i >= 8 ? max(v, t) : v; }
    return v;
}

// The value of lane i-1 of an aligned group (0 in the group's first lane).
__device__ __forceinline__ uint32_t es_prev(uint32_t v, uint32_t i) {
    const uint32_t t = pc_dpp<0x111>(v);   // row_shr:1
    return i >= 1 ? t : 0u;
}

template <int W, int D> struct EsGeom {
    static constexpr uint32_t HB = W == 8 ? 3 : 4;
    static constexpr uint32_t WB = W / 8;
    static constexpr uint32_t DP = pc_pow2(D);                     // item lanes per block
    static constexpr uint32_t SPW = 64 / DP;                       // segments per workgroup
    static constexpr uint32_t CB = DP <= 8 ? 8 : 64 / DP;          // blocks per chunk
    static constexpr uint32_t CR = 8 * CB;                         // rows per chunk
    static constexpr uint32_t SEGB = CR * D * WB;                  // staged bytes of a segment-chunk
    // staged rows carry 16 bytes of padding after every group of GB bytes
    // (whole blocks, whole 16-byte units), so that the lanes of one row
    // read, which belong to different blocks, fall into different banks
    static constexpr uint32_t GB = (8 * D * WB) % 16 == 0 ? 8 * D * WB : 16 * D * WB;
    static constexpr uint32_t RG = GB / (D * WB);                  // rows per padded group (8 or 16)
    static constexpr uint32_t SSTR = SEGB + 16 * (SEGB / GB) + 16; // LDS stride of a segment-chunk
    static constexpr uint32_t UNITS = SEGB / 16;                   // 16-byte input units
    static constexpr uint32_t UG = GB / 16;                        // units per padded group
    static constexpr uint32_t SPT = 64 / (CB * DP);                // segments per wave tile
    static constexpr uint32_t NBS = 64 / DP;                       // block slots per wave tile
    static constexpr uint32_t IW = es_item_waves(D);               // item waves
    static constexpr uint32_t PASSES = CB / IW;                    // wave tiles per item wave
    static constexpr uint32_t MAXBLK = 8 * D * WB;                 // largest block payload
    // Records in one chunk of one segment: its nonzero blocks, the runs
    // between them, and the pieces of a run carried in from earlier chunks
    // (a segment has at most 2^17 blocks, so at most 3 pieces of 65,535).
    static constexpr uint32_t MAXREC = CB + 4;
    // payload staging per segment: the carried partial unit, one chunk of
    // payloads and run records; at the segment's end the trailing run
    // records and the raw tail rows
    static constexpr uint32_t PBYTES = 16 + CB * MAXBLK + 2 * MAXREC + 7 * D * WB;
    static constexpr uint32_t PUNITS = (PBYTES + 15) / 16;
    static constexpr uint32_t PSTR = PUNITS * 4;                   // dwords
    // header staging: the carried partial dword and one chunk of records
    static constexpr uint32_t HSTR = (32 + MAXREC * D * HB + 31) / 32 + 1;   // dwords
    static constexpr uint32_t NT = es_threads(D);
    static_assert(SEGB % 16 == 0 && CB % IW == 0 && PASSES >= 1 && SPT >= 1 && SPT * CB * DP == 64 &&
                      (RG == 8 || RG == 16) && SEGB % GB == 0, "geometry");
};

// Largest header array of a segment with nblk blocks, and the slot layout.
__host__ __device__ inline uint64_t es_hdr_cap(uint64_t nblk, uint32_t D, uint32_t w) {
    return (nblk * D * (w == 8 ? 3u : 4u) + 7) / 8;
}
__host__ __device__ inline uint64_t es_p0(uint64_t nblk, uint32_t D, uint32_t w) {
    return (4 + es_hdr_cap(nblk, D, w) + 4 + 15) & ~15ull;
}
__host__ __device__ inline uint64_t es_slot_bytes(uint64_t nblk, uint32_t D, uint32_t w) {
    // full-width payloads, run records of a segment, raw tail rows, and the
    // whole last staged unit
    return (es_p0(nblk, D, w) + nblk * D * w + 8 + 7ull * D * (w / 8) + 32 + 15) & ~15ull;
}

// Per-segment encoding state in LDS.
struct EsSeg {
    uint32_t nblk, tail;      // whole blocks, raw tail rows
    uint32_t r, cursor, run;  // records so far, payload bytes so far, zero blocks pending
    uint32_t r0, cursor0;     // the same at the start of the current chunk
    uint32_t pad;
};

__host__ __device__ constexpr uint32_t es_pow2(uint32_t v) { return v <= 1 ? 1u : 2 * es_pow2((v + 1) / 2); }

// One workgroup's job: up to SPW consecutive segments of one series.
struct EsJob {
    const uint8_t *src;   // the series' rows
    uint8_t *slots;       // its workspace slots (slot_stride bytes each)
    u32x4 *info;          // its segment info records
    uint64_t rows, slot_stride;
    uint32_t S, nseg, seg0, sh;
    int32_t acc_lo, acc_hi;
};

template <int W, bool FIRE, int D> __device__ __forceinline__ void es_encode_group(const EsJob &jb) {
    using G = EsGeom<W, D>;
    constexpr uint32_t HB = G::HB, WB = G::WB, DP = G::DP, SPW = G::SPW, CB = G::CB, CR = G::CR;
    constexpr uint32_t SSTR = G::SSTR, SPT = G::SPT, NBS = G::NBS, P = G::PASSES;
    constexpr bool COL = D * W <= 32;   // column-major payloads (reading R13)
    constexpr uint32_t NBUF = FIRE ? 3 : 2;
    constexpr uint32_t LAG = FIRE ? 1 : 0;   // item waves work one chunk behind the alpha wave
    // payload and header staging are rings (powers of two) over the
    // segment's byte and header-bit positions: a unit goes out and is
    // cleared as soon as it is complete, the partial last one stays in place
    constexpr uint32_t PR = es_pow2(G::PUNITS);   // 16-byte units per segment
    constexpr uint32_t HR = es_pow2(G::HSTR);     // header dwords per segment
    constexpr uint32_t WSEG = SPT * P;            // segments of one item wave
    constexpr uint32_t WSLOT = NBS * P;           // block slots of one item wave

    __shared__ u32x4 STG[NBUF * SPW * SSTR / 16];          // staged rows: [buffer][segment][row][column]
    __shared__ int32_t ALPHA[FIRE ? 2 * 64 * CB : 1];       // [parity][chain][block]
    __shared__ uint32_t PREVX[2][64];                       // a chain's last sample before the chunk
    __shared__ int32_t PREVD[2][64];                        // and its last delta
    __shared__ u32x4 PST4[SPW * PR];                        // payload rings
    __shared__ uint32_t HST[SPW * HR];                      // header rings
    __shared__ u32x4 BLK[G::IW][WSLOT];                     // wave-local block records
    __shared__ EsSeg SEG[SPW];
    uint32_t *const PST = reinterpret_cast<uint32_t *>(PST4);
    uint8_t *const PSTB = reinterpret_cast<uint8_t *>(PST4);
    const uint8_t *const stgb = reinterpret_cast<const uint8_t *>(STG);

    const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    constexpr uint32_t IW = G::IW;
    const bool alpha_wave = wave == IW;
    const uint32_t seg0 = jb.seg0;
    const uint8_t *const src = jb.src;
    uint8_t *const slots = jb.slots;
    u32x4 *const info = jb.info;
    const uint64_t slot_stride = jb.slot_stride;
    const uint32_t nsw = min(SPW, jb.nseg - seg0);

    // bounded views: this workgroup's input rows and its workspace slots
    const uint64_t wrow0 = (uint64_t)seg0 * jb.S;
    const uint64_t wrows = min((uint64_t)nsw * jb.S, jb.rows - wrow0);
    const uint32_t in_bytes = (uint32_t)(wrows * D * WB);
    const Buf in = make_buf(src + wrow0 * D * WB, in_bytes);
    const uint32_t sstride = (uint32_t)slot_stride;
    const Buf out = make_buf(slots + (uint64_t)seg0 * slot_stride, nsw * sstride);
    const uint32_t p0 = (uint32_t)es_p0(jb.S >> 3, D, W);

    // the wave's k-th segment and block slot q's segment (in the workgroup)
    auto wseg = [&](uint32_t k) -> uint32_t { return ((k / SPT) * IW + wave) * SPT + k % SPT; };

    // ---- setup ------------------------------------------------------------------
    if (tid < SPW) {
        EsSeg sg;
        const uint32_t nr = tid < nsw ? (uint32_t)min((uint64_t)jb.S, jb.rows - (uint64_t)(seg0 + tid) * jb.S) : 0u;
        sg.nblk = nr >> 3;
        sg.tail = nr & 7u;
        sg.r = 0; sg.cursor = 0; sg.run = 0; sg.r0 = 0; sg.cursor0 = 0; sg.pad = 0;
        SEG[tid] = sg;
    }
    for (uint32_t k = tid; k < SPW * PR * 4; k += G::NT) PST[k] = 0;
    for (uint32_t k = tid; k < SPW * HR; k += G::NT) HST[k] = 0;
    if (tid < 64) { PREVX[0][tid] = 0; PREVD[0][tid] = 0; }

    // staging of a chunk's rows: 16-byte units over the item lanes
    constexpr uint32_t NIT = 64 * IW;
    constexpr uint32_t SUN = (SPW * G::UNITS + NIT - 1) / NIT;
    u32x4 reg[SUN];
    auto stage_issue = [&](uint32_t c) {
#pragma unroll
        for (uint32_t t = 0; t < SUN; ++t) {
            const uint32_t u = tid + t * NIT;
            const uint32_t s = u / G::UNITS, k = u % G::UNITS;
            u32x4 v = {0u, 0u, 0u, 0u};
            if (u < SPW * G::UNITS && s < nsw) {
                const uint32_t off = (s * jb.S + c * CR) * D * WB + 16 * k;
                if (off + 16 <= in_bytes) {
                    v = buf_ld128(in, off);
                } else if (off < in_bytes) {
                    // a unit across the end of the input (rows end on 8-byte
                    // boundaries at least, so its dwords are whole or absent)
                    v.x = buf_ld32(in, off);
                    v.y = buf_ld32(in, off + 4);
                    v.z = buf_ld32(in, off + 8);
                    v.w = buf_ld32(in, off + 12);
                }
            }
            reg[t] = v;
        }
    };
    auto stage_commit = [&](uint32_t c) {
        u32x4 *const dstg = STG + (c % NBUF) * (SPW * SSTR / 16);
#pragma unroll
        for (uint32_t t = 0; t < SUN; ++t) {
            const uint32_t u = tid + t * NIT;
            const uint32_t s = u / G::UNITS, k = u % G::UNITS;
            if (u < SPW * G::UNITS) dstg[s * (SSTR / 16) + k + k / G::UG] = reg[t];
        }
    };
    auto xval = [&](uint32_t buf, uint32_t s, uint32_t row, uint32_t j) -> uint32_t {
        const uint32_t off = (buf * SPW + s) * SSTR + (row * D + j) * WB + 16 * (row / G::RG);
        return WB == 1 ? (uint32_t)stgb[off] : (uint32_t)*reinterpret_cast<const uint16_t *>(stgb + off);
    };
    // a u16 run count at payload byte pos of segment s
    auto put_count = [&](uint32_t s, uint32_t pos, uint32_t cnt) {
        uint8_t *const pb = PSTB + s * PR * 16;
        pb[pos & (PR * 16 - 1)] = (uint8_t)cnt;
        pb[(pos + 1) & (PR * 16 - 1)] = (uint8_t)(cnt >> 8);
    };

    if (!alpha_wave) {
        stage_issue(0);
        stage_commit(0);
    }
    __syncthreads();

    const uint32_t nchunks = ((jb.S >> 3) + CB - 1) / CB;

    // alpha wave state: one column chain per lane
    const uint32_t a_s = lane / DP, a_j = lane % DP;
    const bool a_on = alpha_wave && a_j < (uint32_t)D && a_s < nsw;
    uint32_t a_x = 0;
    int32_t a_d = 0, acc = 0;

    for (uint32_t t = 0; t < nchunks + LAG; ++t) {
        if (alpha_wave) {
            if (FIRE && t < nchunks && a_on) {
                // ---- the coefficient chain over chunk t ------------------------
                const uint32_t buf = t % NBUF;
                const uint32_t nb = SEG[a_s].nblk;
                const uint32_t bic = t * CB < nb ? min(CB, nb - t * CB) : 0u;
                for (uint32_t b = 0; b < bic; ++b) {
                    uint32_t xs[8];
#pragma unroll
                    for (int i = 0; i < 8; ++i) xs[i] = xval(buf, a_s, 8 * b + i, a_j);
                    const int32_t alpha = acc >> jb.sh;
                    ALPHA[((t & 1) * 64 + lane) * CB + b] = alpha;
                    int32_t grad = 0;
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        const int32_t d = sext<W>((int32_t)(xs[i] - a_x));
                        if (i & 1) {
                            const int32_t e = sext<W>(d - (__mul24(alpha, a_d) >> W));
                            grad += __mul24(sgn_med3(e), a_d);
                        }
                        a_d = d;
                        a_x = xs[i];
                    }
                    acc = min(max(acc + grad, jb.acc_lo), jb.acc_hi);
                }
            }
        } else {
            if (t + 1 < nchunks) stage_issue(t + 1);
            if (t >= LAG) {
                const uint32_t c = t - LAG;
                const uint32_t buf = c % NBUF;
                // ---- item lanes: (segment, block, column), every tile of the wave --
                const uint32_t sl = lane / (CB * DP), b = (lane / DP) % CB, j = lane % DP;
                const uint32_t bslot = lane / DP;
                uint32_t z[P][8], width[P], off[P], wsum[P], cwl[P], cwh[P];
                bool valid[P];
#pragma unroll
                for (uint32_t pass = 0; pass < P; ++pass) {
                    const uint32_t s = (pass * IW + wave) * SPT + sl;
                    const uint32_t nblk_s = SEG[s].nblk;
                    const uint32_t bic = c * CB < nblk_s ? min(CB, nblk_s - c * CB) : 0u;
                    valid[pass] = s < nsw && b < bic;
                    const bool act = valid[pass] && j < (uint32_t)D;
                    const uint32_t ch = s * DP + j;
                    uint32_t orz = 0;
                    if (act) {
                        uint32_t xp = b == 0 ? PREVX[c & 1][ch] : xval(buf, s, 8 * b - 1, j);
                        int32_t dp = 0;
                        if (FIRE) dp = b == 0 ? PREVD[c & 1][ch] : sext<W>((int32_t)(xp - xval(buf, s, 8 * b - 2, j)));
                        const int32_t alpha = FIRE ? ALPHA[((c & 1) * 64 + ch) * CB + b] : 0;
#pragma unroll
                        for (int i = 0; i < 8; ++i) {
                            const uint32_t x = xval(buf, s, 8 * b + i, j);
                            const int32_t d = sext<W>((int32_t)(x - xp));
                            const int32_t e = FIRE ? sext<W>(d - (__mul24(alpha, dp) >> W)) : d;
                            z[pass][i] = zigzag(e);
                            orz |= z[pass][i];
                            dp = d;
                            xp = x;
                        }
                        if (b == bic - 1) {
                            PREVX[(c + 1) & 1][ch] = xp;
                            PREVD[(c + 1) & 1][ch] = dp;
                        }
                    } else {
#pragma unroll
                        for (int i = 0; i < 8; ++i) z[pass][i] = 0;
                    }
                    const uint32_t code = min(bitlen(orz), (uint32_t)W - 1);
                    width[pass] = code < (uint32_t)W - 1 ? code : (uint32_t)W;
                    wsum[pass] = pc_total<DP>(width[pass]);
                    off[pass] = pc_incl<DP>(width[pass], j) - width[pass];
                    // header code word of the block: D fields of HB bits, LSB first
                    const uint32_t cb0 = j * HB;
                    cwl[pass] = pc_total<DP>(cb0 < 32 ? code << cb0 : 0u);
                    cwh[pass] = 0;
                    if constexpr (D * HB > 32)
                        cwh[pass] = pc_total<DP>(cb0 + HB <= 32 ? 0u : cb0 >= 32 ? code << (cb0 - 32) : code >> (32 - cb0));
                    if (j == 0) {
                        u32x4 v;
                        v.x = wsum[pass]; v.y = 0; v.z = 0; v.w = valid[pass] ? 1u : 0u;
                        BLK[wave][pass * NBS + bslot] = v;
                    }
                }
                wave_sync();
                // ---- block lanes: (segment, block); records of the chunk -----------
                // every lane takes part in the scans (lanes past the wave's
                // slots form groups of their own and write nothing)
#pragma unroll
                for (uint32_t rr = 0; rr < (WSLOT + 63) / 64; ++rr) {
                    const uint32_t qr = lane + 64 * rr;
                    const bool qa = qr < WSLOT;
                    const uint32_t q = qa ? qr : 0u;
                    {
                        const uint32_t bb = qr % CB;
                        const uint32_t ss = wseg(q / CB);
                        const EsSeg sq = SEG[ss];
                        const u32x4 bv = BLK[wave][q];
                        const bool nz = qa && bv.w != 0 && bv.x != 0;
                        const uint32_t qbic = c * CB < sq.nblk ? min(CB, sq.nblk - c * CB) : 0u;
                        // last nonzero block up to this one, 1-based (0 = none)
                        const uint32_t lastin = es_incl_max<CB>(nz ? bb + 1 : 0u, bb);
                        const uint32_t prevnz = es_prev(lastin, bb);
                        const uint32_t run = !nz ? 0u : prevnz == 0 ? sq.run + bb : bb - prevnz;
                        const uint32_t nrle = (run + kRleMax - 1) / kRleMax;
                        const uint32_t psize = COL ? bv.x : 8 * ((bv.x + 7) >> 3);
                        const uint32_t nrec_b = nz ? nrle + 1 : 0u;
                        const uint32_t pay_b = nz ? 2 * nrle + psize : 0u;
                        const uint32_t rinc = pc_incl<CB>(nrec_b, bb);
                        const uint32_t pinc = pc_incl<CB>(pay_b, bb);
                        const uint32_t nrec_c = pc_total<CB>(nrec_b);
                        const uint32_t pay_c = pc_total<CB>(pay_b);
                        const uint32_t lastall = pc_total<CB>(bb == CB - 1 ? lastin : 0u);
                        const uint32_t prun = sq.cursor + pinc - pay_b;   // its run records
                        for (uint32_t k = 0; k < nrle; ++k)
                            put_count(ss, prun + 2 * k, k + 1 < nrle ? kRleMax : run - kRleMax * (nrle - 1));
                        u32x4 res;
                        res.x = sq.r + rinc - 1;    // record index of the block
                        res.y = prun + 2 * nrle;    // payload byte of the block
                        res.z = 0;
                        res.w = 0;
                        wave_sync();
                        if (qa) BLK[wave][q] = res;
                        if (qa && bb == 0 && ss < nsw) {
                            EsSeg &ns = SEG[ss];
                            ns.r0 = sq.r;
                            ns.cursor0 = sq.cursor;
                            if (qbic > 0) {
                                ns.r = sq.r + nrec_c;
                                ns.cursor = sq.cursor + pay_c;
                                ns.run = lastall == 0 ? sq.run + qbic : qbic - lastall;
                            }
                        }
                    }
                }
                wave_sync();
                // ---- pack: fields and header codes into the rings -------------------
#pragma unroll
                for (uint32_t pass = 0; pass < P; ++pass) {
                    const uint32_t s = (pass * IW + wave) * SPT + sl;
                    // row-major: the fields of columns j and j + 1 of a row lie side
                    // by side; even lanes take their odd neighbour's field and width
                    // (every lane, before any lane-dependent branch) and write both
                    // with one pair of atomics
                    uint32_t zn[COL ? 1 : 8], wn = 0;
                    if constexpr (!COL) {
#pragma unroll
                        for (int i = 0; i < 8; ++i) zn[i] = pc_dpp<0xF5>(z[pass][i]);   // quad_perm [1,1,3,3]
                        wn = pc_dpp<0xF5>(width[pass]);
                    }
                    if (valid[pass] && wsum[pass] != 0) {
                        const u32x4 res = BLK[wave][pass * NBS + bslot];
                        uint32_t *const pw = PST + s * PR * 4;
                        const uint32_t pbit = 8 * res.y;
                        const uint32_t wd = width[pass];
                        const uint32_t rbits = 8 * ((wsum[pass] + 7) >> 3);
                        if (COL && j < (uint32_t)D && wd != 0) {
                            // column-major: the column's fields lie side by side, so 32/w
                            // of them (at most 32 bits) go in with one pair of atomics
                            constexpr uint32_t FG = 32 / W;
#pragma unroll
                            for (uint32_t k = 0; k < 8 / FG; ++k) {
                                uint32_t v = z[pass][k * FG];
#pragma unroll
                                for (uint32_t g = 1; g < FG; ++g) v |= z[pass][k * FG + g] << (g * wd);
                                const uint32_t fwd = FG * wd;
                                const uint32_t p = pbit + 8 * off[pass] + k * fwd;
                                const uint32_t sb = p & 31u;
                                atomicOr(&pw[(p >> 5) & (PR * 4 - 1)], v << sb);
                                if (sb + fwd > 32) atomicOr(&pw[((p >> 5) + 1) & (PR * 4 - 1)], v >> (32 - sb));
                            }
                        }
                        if constexpr (!COL) {
                            if (!(j & 1) && j < (uint32_t)D && wd + wn != 0) {
                                const uint32_t fwd = wd + wn;   // at most 2w <= 32 bits
#pragma unroll
                                for (int i = 0; i < 8; ++i) {
                                    const uint32_t v = z[pass][i] | zn[i] << wd;
                                    const uint32_t p = pbit + (uint32_t)i * rbits + off[pass];
                                    const uint32_t sb = p & 31u;
                                    atomicOr(&pw[(p >> 5) & (PR * 4 - 1)], v << sb);
                                    if (sb + fwd > 32) atomicOr(&pw[((p >> 5) + 1) & (PR * 4 - 1)], v >> (32 - sb));
                                }
                            }
                        }
                        if (j == 0) {
                            const uint32_t lb = res.x * D * HB;
                            uint32_t *const hw = HST + s * HR;
                            const uint32_t q0 = lb >> 5, sb = lb & 31u;
                            const uint32_t cl = cwl[pass], chh = cwh[pass];
                            if (cl) atomicOr(&hw[q0 & (HR - 1)], cl << sb);
                            if constexpr (D * HB > 32) {
                                const uint32_t w1 = (sb ? cl >> (32 - sb) : 0u) | (chh << sb);
                                if (w1) atomicOr(&hw[(q0 + 1) & (HR - 1)], w1);
                                if (sb && (chh >> (32 - sb))) atomicOr(&hw[(q0 + 2) & (HR - 1)], chh >> (32 - sb));
                            } else {
                                if (sb + D * HB > 32 && (cl >> (32 - sb))) atomicOr(&hw[(q0 + 1) & (HR - 1)], cl >> (32 - sb));
                            }
                        }
                    }
                }
                wave_sync();
                // ---- flush: units and header dwords completed in this chunk ---------
                // (each goes out and is cleared in place)
                constexpr uint32_t FU = (WSEG * G::PUNITS + 63) / 64;
#pragma unroll
                for (uint32_t k = 0; k < FU; ++k) {
                    const uint32_t f = lane + 64 * k;
                    const uint32_t fs = f / G::PUNITS, u = f % G::PUNITS;
                    const uint32_t ss = wseg(fs);
                    if (f < WSEG * G::PUNITS && ss < nsw) {
                        const EsSeg sq = SEG[ss];
                        const uint32_t ua = (sq.cursor0 >> 4) + u;
                        if (ua < (sq.cursor >> 4)) {
                            u32x4 *const pu = PST4 + ss * PR + (ua & (PR - 1));
                            buf_st128(out, ss * sstride + p0 + 16 * ua, *pu);
                            *pu = u32x4{0u, 0u, 0u, 0u};
                        }
                    }
                }
                constexpr uint32_t FH = (WSEG * G::HSTR + 63) / 64;
#pragma unroll
                for (uint32_t k = 0; k < FH; ++k) {
                    const uint32_t f = lane + 64 * k;
                    const uint32_t fs = f / G::HSTR, qd = f % G::HSTR;
                    const uint32_t ss = wseg(fs);
                    if (f < WSEG * G::HSTR && ss < nsw) {
                        const EsSeg sq = SEG[ss];
                        const uint32_t da = ((sq.r0 * D * HB) >> 5) + qd;
                        if (da < ((sq.r * D * HB) >> 5)) {
                            uint32_t *const hw = HST + ss * HR + (da & (HR - 1));
                            buf_st32(out, ss * sstride + 4 + 4 * da, *hw);
                            *hw = 0;
                        }
                    }
                }
                wave_sync();
            }
            if (t + 1 < nchunks) stage_commit(t + 1);
        }
        __syncthreads();
    }

    // ---- segment ends: trailing runs, raw tail rows, last units, sizes ----------
    if (!alpha_wave) {
        for (uint32_t k = 0; k < WSEG; ++k) {
            const uint32_t ss = wseg(k);
            if (ss >= nsw) continue;
            const EsSeg q = SEG[ss];
            const uint32_t nrle = (q.run + kRleMax - 1) / kRleMax;
            if (lane < nrle) put_count(ss, q.cursor + 2 * lane, lane + 1 < nrle ? kRleMax : q.run - kRleMax * (nrle - 1));
            const uint32_t tb = q.tail * D * WB;
            const uint32_t tpos = q.cursor + 2 * nrle;
            const uint32_t trow = (ss * jb.S + q.nblk * 8) * D * WB;   // in the workgroup's input
            uint8_t *const pb = PSTB + ss * PR * 16;
            for (uint32_t i = lane; i < tb; i += 64) pb[(tpos + i) & (PR * 16 - 1)] = (uint8_t)buf_ld8(in, trow + i);
            wave_sync();
            const uint32_t paytail = tpos + tb;
            const uint32_t ufirst = q.cursor >> 4, uend = (paytail + 15) >> 4;
            for (uint32_t ua = ufirst + lane; ua < uend; ua += 64)
                buf_st128(out, ss * sstride + p0 + 16 * ua, PST4[ss * PR + (ua & (PR - 1))]);
            const uint32_t nrec = q.r + nrle;
            const uint32_t hbits = nrec * D * HB;
            const uint32_t dfirst = (q.r * D * HB) >> 5, dend = (hbits + 31) >> 5;
            for (uint32_t da = dfirst + lane; da < dend; da += 64)
                buf_st32(out, ss * sstride + 4 + 4 * da, HST[ss * HR + (da & (HR - 1))]);
            if (lane == 0) {
                buf_st32(out, ss * sstride, nrec);
                const uint32_t hdr = (hbits + 7) >> 3;
                u32x4 v;
                v.x = (4 + hdr + paytail + 15) & ~15u;   // segment bytes
                v.y = nrec;
                v.z = paytail;                           // payload and tail bytes
                v.w = 0;
                info[seg0 + ss] = v;
            }
        }
    }
}

template <int W, bool FIRE, int D>
__global__ __launch_bounds__(es_threads(D)) void k_encode_sp(const uint8_t *__restrict__ src, Geom g,
                                                              uint8_t *__restrict__ slots, uint64_t slot_stride,
                                                              u32x4 *__restrict__ info) {
    const EsJob jb{src, slots, info, g.rows, slot_stride, g.S, g.nseg, blockIdx.x * EsGeom<W, D>::SPW, g.sh,
                   g.acc_lo, g.acc_hi};
    es_encode_group<W, FIRE, D>(jb);
}

// One series of a compression batch, as the batched kernels see it.
struct EsStream {
    const uint8_t *src;
    uint8_t *dst;         // container
    uint8_t *slots;
    u32x4 *info;
    uint64_t *out_size;
    uint64_t rows, cap, data_start, slot_stride;
    uint32_t D, S, nseg, w, dtype, forecaster, learn_shift, sh;
    int32_t acc_lo, acc_hi;
    uint32_t status, pad;   // index of the series' status word
};

// Many series of one class (w, forecaster, D): a persistent grid pulls
// groups (series, first segment) from a device queue.
template <int W, bool FIRE, int D>
__global__ __launch_bounds__(es_threads(D)) void k_encode_sp_batch(const EsStream *__restrict__ streams,
                                                                    const uint2 *__restrict__ groups, uint32_t ngroups,
                                                                    uint32_t *__restrict__ queue) {
    __shared__ uint32_t grp_sh;
    for (;;) {
        if (threadIdx.x == 0) grp_sh = atomicAdd(queue, 1u);
        __syncthreads();
        const uint32_t grp = grp_sh;
        __syncthreads();
        if (grp >= ngroups) break;
        const uint2 gr = groups[grp];
        const EsStream &st = streams[gr.x];
        const EsJob jb{st.src, st.slots, st.info, st.rows, st.slot_stride, st.S, st.nseg, gr.y, st.sh, st.acc_lo,
                       st.acc_hi};
        es_encode_group<W, FIRE, D>(jb);
        __syncthreads();
    }
}

// Offset table and container header from the segment sizes (one workgroup),
// in rounds of R sizes per thread: a thread loads a contiguous run of R sizes
// at once (one memory latency per round, not one per size), one block scan,
// then the table entries of its run; a carry links the rounds.
__device__ __forceinline__ void es_scan_body(const u32x4 *__restrict__ info, uint32_t n, uint64_t rows, uint32_t D,
                                             uint32_t S, uint32_t G, uint64_t data_start, uint64_t cap, uint32_t w,
                                             uint32_t dtype, uint32_t forecaster, uint32_t learn_shift,
                                             uint8_t *__restrict__ dst, uint64_t *__restrict__ out_size,
                                             int32_t *__restrict__ status) {
    constexpr uint32_t R = 8;
    __shared__ uint64_t wsum[16];
    const uint32_t t = threadIdx.x, lane = t & 63, wv = t >> 6, nt = blockDim.x, nw = nt >> 6;
    uint64_t *tab = reinterpret_cast<uint64_t *>(dst + 64);
    uint64_t total = 0;   // sizes of the rounds before
    for (uint32_t base = 0; base < n; base += nt * R) {
        const uint32_t k0 = base + t * R;
        uint32_t v[R];
#pragma unroll
        for (uint32_t r = 0; r < R; ++r) v[r] = k0 + r < n ? info[k0 + r].x : 0u;
        uint64_t mine = 0;
#pragma unroll
        for (uint32_t r = 0; r < R; ++r) mine += v[r];
        uint64_t incl = mine;
        for (uint32_t d = 1; d < 64; d <<= 1) {
            const uint64_t o = (uint64_t)__shfl_up((unsigned long long)incl, d, 64);
            if (lane >= d) incl += o;
        }
        if (lane == 63) wsum[wv] = incl;
        __syncthreads();
        uint64_t before = 0, round = 0;
        for (uint32_t q = 0; q < nw; ++q) {
            const uint64_t x = wsum[q];
            if (q < wv) before += x;
            round += x;
        }
        __syncthreads();   // wsum is rewritten by the next round
        uint64_t run = total + before + incl - mine;
#pragma unroll
        for (uint32_t r = 0; r < R; ++r) {
            if (k0 + r < n) tab[k0 + r] = run;
            run += v[r];
        }
        total += round;
    }
    if (t == 0) tab[n] = total;
    if (t < 16) {
        // 64-byte header as 16 dwords (reading R18: the container layout)
        uint32_t word = 0;
        switch (t) {
            case 0: word = 0x315A5053u; break;                                            // "SPZ1"
            case 1: word = 1u | (w << 16) | (dtype << 24); break;                          // version, w, dtype
            case 2: word = forecaster | (learn_shift << 8) | (G << 16); break;             // entropy 0
            case 3: word = D; break;
            case 4: word = (uint32_t)rows; break;
            case 5: word = (uint32_t)(rows >> 32); break;
            case 6: word = S; break;
            case 7: word = n; break;
            case 8: word = (uint32_t)total; break;
            case 9: word = (uint32_t)(total >> 32); break;
            default: word = 0; break;
        }
        reinterpret_cast<uint32_t *>(dst)[t] = word;
    }
    // zero padding between the offset table and the data
    const uint64_t pad0 = 64 + 8ull * (n + 1);
    if (t < data_start - pad0) dst[pad0 + t] = 0;
    if (t == 0) {
        *out_size = data_start + total;
        if (data_start + total > cap && status) atomicOr(status, 2);
    }
}

__global__ __launch_bounds__(1024) void k_enc_scan(const u32x4 *__restrict__ info, Geom g, uint32_t w, uint32_t dtype,
                                                   uint32_t forecaster, uint32_t learn_shift, uint8_t *__restrict__ dst,
                                                   uint64_t *__restrict__ out_size, int32_t *__restrict__ status) {
    es_scan_body(info, g.nseg, g.rows, g.D, g.S, g.G, g.data_start, g.cap, w, dtype, forecaster, learn_shift, dst,
                 out_size, status);
}

// One workgroup per series of a compression batch.
__global__ __launch_bounds__(256) void k_enc_scan_batch(const EsStream *__restrict__ streams, const uint32_t *__restrict__ list,
                                                        int32_t *__restrict__ status) {
    const EsStream &st = streams[list[blockIdx.x]];
    es_scan_body(st.info, st.nseg, st.rows, st.D, st.S, 0, st.data_start, st.cap, st.w, st.dtype, st.forecaster,
                 st.learn_shift, st.dst, st.out_size, status ? status + st.status : nullptr);
}

// Copies K segments per workgroup from their workspace slots to the
// container: destination units of 16 bytes, bytes [0, 4 + header) from the
// slot's start and the rest from its payload at P0, zero padding at the end.
__device__ __forceinline__ void es_compact_body(const uint8_t *__restrict__ slots, uint64_t slot_stride,
                                                const u32x4 *__restrict__ info, uint32_t nseg, uint64_t data_start,
                                                uint64_t cap, uint32_t D, uint32_t S, uint32_t w, uint32_t first,
                                                uint32_t K, uint8_t *__restrict__ dst, int32_t *__restrict__ status) {
    if (first >= nseg) return;
    const uint32_t last = min(nseg, first + K);
    const uint64_t *tab = reinterpret_cast<const uint64_t *>(dst + 64);
    const uint64_t o0 = tab[first], o1 = tab[last];
    if (data_start + o1 > cap || o1 < o0 || o1 - o0 > 0xFFFFFFF0ull) {
        if (threadIdx.x == 0 && status) atomicOr(status, 2);
        return;
    }
    const Buf sb = make_buf(slots + (uint64_t)first * slot_stride, (uint32_t)((last - first) * slot_stride));
    const Buf db = make_buf(dst + data_start + o0, (uint32_t)(o1 - o0));
    const uint32_t hb = w == 8 ? 3u : 4u;
    const uint32_t p0 = (uint32_t)es_p0(S >> 3, D, w);
    for (uint32_t s = first; s < last; ++s) {
        const u32x4 in = info[s];
        const uint32_t size = in.x, A = 4 + (uint32_t)(((uint64_t)in.y * D * hb + 7) >> 3), PT = in.z;
        const uint32_t sbase = (s - first) * (uint32_t)slot_stride;
        const uint32_t dbase = (uint32_t)(tab[s] - o0);
        if (size % 16 || size > slot_stride || A + PT > size || tab[s + 1] - tab[s] != size) {
            if (threadIdx.x == 0 && status) atomicOr(status, 2);   // sizes that the encoder did not write
            continue;
        }
        const uint32_t shift = 8 * ((p0 - A) & 3u);
        for (uint32_t u = threadIdx.x; u < size / 16; u += blockDim.x) {
            const uint32_t k0 = 16 * u;
            u32x4 a = {0u, 0u, 0u, 0u};
            if (k0 < A) a = buf_ld128(sb, sbase + k0);
            uint32_t bw[5] = {0u, 0u, 0u, 0u, 0u};
            if (k0 + 16 > A) {
                // payload bytes for this unit start at slot byte P0 + k0 - A
                // (below P0 for the unit that holds the header's end; those
                // bytes are masked)
                const uint32_t sbyte = p0 + k0 - A;
                const uint32_t d0 = sbase + (sbyte & ~3u);
#pragma unroll
                for (int q = 0; q < 5; ++q) bw[q] = buf_ld32(sb, d0 + 4 * q);
            }
            uint32_t v[4];
            const uint32_t aw[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t kq = k0 + 4 * q;
                const uint32_t bq = __builtin_amdgcn_alignbit(bw[q + 1], bw[q], shift);
                const uint32_t na = A > kq ? min(A - kq, 4u) : 0u;         // bytes from the header part
                const uint32_t nk = A + PT > kq ? min(A + PT - kq, 4u) : 0u;   // bytes that are not padding
                const uint32_t ma = na >= 4 ? ~0u : (1u << (8 * na)) - 1u;
                const uint32_t mk = nk >= 4 ? ~0u : (1u << (8 * nk)) - 1u;
                v[q] = ((aw[q] & ma) | (bq & ~ma)) & mk;
            }
            u32x4 o;
            o.x = v[0]; o.y = v[1]; o.z = v[2]; o.w = v[3];
            buf_st128(db, dbase + k0, o);
        }
    }
}

__global__ __launch_bounds__(256) void k_enc_compact(const uint8_t *__restrict__ slots, uint64_t slot_stride,
                                                     const u32x4 *__restrict__ info, Geom g, uint32_t w, uint32_t K,
                                                     uint8_t *__restrict__ dst, int32_t *__restrict__ status) {
    es_compact_body(slots, slot_stride, info, g.nseg, g.data_start, g.cap, g.D, g.S, w, blockIdx.x * K, K, dst, status);
}

// Compaction groups of a compression batch: (series, first segment, count).
__global__ __launch_bounds__(256) void k_enc_compact_batch(const EsStream *__restrict__ streams,
                                                           const uint4 *__restrict__ groups,
                                                           int32_t *__restrict__ status) {
    const uint4 gr = groups[blockIdx.x];
    const EsStream &st = streams[gr.x];
    es_compact_body(st.slots, st.slot_stride, st.info, st.nseg, st.data_start, st.cap, st.D, st.S, st.w, gr.y, gr.z,
                    st.dst, status ? status + st.status : nullptr);
}

}  // namespace spz

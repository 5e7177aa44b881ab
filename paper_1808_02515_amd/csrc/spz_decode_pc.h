// Pipelined Sprintz decoder for gfx950 (header group = whole segment, D up
// to 16).
//
// Paper: Algorithm 2 (decodeBlock) with the forecasters of Section 4.2. Of
// the decoding work only the forecaster recurrence is serial (Section 5.4
// names the dependence of each prediction on the previous sample as the
// limit). A workgroup holds the segments of 64 column chains and splits into
// a four-stage pipeline of wavefronts over chunks of 8 blocks, one barrier
// per step:
//
//   parser (chunk t)       stage   the loads of chunk t, issued a step
//                                  earlier, go from registers to LDS
//                          parse   lanes = (segment, candidate record k of
//                                  the chunk): the record's header codes give
//                                  its width sum and byte size; scans over k
//                                  give payload offsets, run counts and the
//                                  blocks each record covers
//                          issue   16-byte loads of chunk t+1's header and
//                                  payload windows (their bases come from the
//                                  parse), in flight over the rest of the step
//   NP unpackers (t-3)     rows of chunk t-3 (the consumer's image) to
//                          global memory, 16-byte stores
//                (t-1)     an aligned two-dword LDS read and a funnel shift
//                          give 32 bits = 32/w fields: lanes = (segment,
//                          block, 32/w adjacent columns) for row-major
//                          payloads, one read per row; (segment, block,
//                          column) for column-major ones, one read per 32/w
//                          rows; unzigzag; the errors e go to an LDS buffer
//                          per column chain
//   consumer (chunk t-2)   lane = column chain. For FIRE
//                              delta = e + floor(alpha * delta_prev / 2^w)   (mod 2^w)
//                              x    += delta
//                          with e and the product's high bits as sign-extended
//                          SDWA operands (one multiply and one add on the
//                          serial chain); sgn(e) * delta_prev is summed on odd
//                          rows and the accumulator saturates once per block
//                          (practical FIRE, Section 4.2.2). Samples go to an
//                          LDS image of the chunk's rows, written over the
//                          error buffers the consumer has just read.
//
// Staging windows, records and error buffers (with the row images) are
// double buffered by chunk parity, so each stage reads what the one before
// wrote a step earlier. This pipelined form serves single containers with
// D >= 7; the producer/consumer form below (producers that parse, stage and
// unpack their own segments, a consumer that also stores the rows) serves
// smaller D and every batched decode.
//
// A block inside a run of zero blocks decodes as a block whose errors are
// all 0 (reading R9: the prediction alone; sgn(0) = 0 leaves the FIRE
// accumulator as it is), so runs need no separate path. Every LDS access is
// aligned.
//
// Global accesses are plain loads and stores, each behind an explicit range
// check:
//   - offset-table reads: entries seg and seg + 1 with seg < nseg, inside the
//     table, which ends before the data start;
//   - segment reads (record count, staged 16-byte windows, raw tail): only
//     when the segment's offsets a <= b <= data_bytes are 16-aligned, and
//     only whole units with off + 16 <= b - a (tail: cursor + tail bytes <=
//     b - a). The host bounds data_start + data_bytes by the container size;
//   - output stores: rows of the segment's own whole blocks (tail: its own
//     tail rows), so below rows * D * w/8 <= the destination capacity.
#pragma once

#include "spz_device.h"

namespace spz {

constexpr int kPcChunkBlocks = 8;
constexpr int kPcProducers = 2;      // unpacking wavefronts per workgroup
constexpr int kPcConsumers = 1;      // consumer wavefronts per workgroup
__host__ __device__ constexpr uint32_t pc_threads(uint32_t NP, uint32_t NC) { return 64 * (NP + NC); }
__host__ __device__ constexpr uint32_t pc_spw(uint32_t D, uint32_t NP, uint32_t NC);
// The single-container kernel takes the pipelined form (a parser wavefront
// besides NP unpacking and NC consumer wavefronts) when one parser pass covers
// the workgroup's (segment, candidate record) pairs (D >= 7); with more passes
// the parser becomes the longest stage (measured: D = 1, 2, 3, 6 decode
// slower, D = 4 level). The batched kernel keeps the producer/consumer form
// (NP producers, NC consumers) at every D: batched throughput follows the
// VALU work per sample, which the separate parser wave raises (measured on a
// 10,000-stream batch: 2.12 against 2.23 TB/s with the pipelined form).
__host__ __device__ constexpr bool pc_pipe(uint32_t D) {
    return pc_spw(D, kPcProducers, kPcConsumers) * kPcChunkBlocks <= 64;
}
__host__ __device__ constexpr uint32_t pc_single_threads(uint32_t D, uint32_t NP, uint32_t NC) {
    return pc_pipe(D) ? 64 * (1 + NP + NC) : 64 * (NP + NC);
}
constexpr uint32_t kPcZero = 0xFFu;  // block map entry of a zero (run) block

template <int CTRL> __device__ __forceinline__ uint32_t pc_dpp(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, true);
}

// Inclusive sum over an aligned group of N <= 16 lanes (one DPP row).
template <int N> __device__ __forceinline__ uint32_t pc_incl(uint32_t v, uint32_t i) {
    if constexpr (N >= 2) { const uint32_t t = pc_dpp<0x111>(v); v += i >= 1 ? t : 0u; }
    if constexpr (N >= 4) { const uint32_t t = pc_dpp<0x112>(v); v += i >= 2 ? t : 0u; }
    if constexpr (N >= 8) { const uint32_t t = pc_dpp<0x114>(v); v += i >= 4 ? t : 0u; }
    if constexpr (N >= 16) { const uint32_t t = pc_dpp<0x118>(v); v += i >= 8 ? t : 0u; }
    return v;
}

// Sum over an aligned group of N <= 16 lanes, in every lane of the group.
template <int N> __device__ __forceinline__ uint32_t pc_total(uint32_t v) {
    if constexpr (N >= 2) v += pc_dpp<0xB1>(v);   // quad_perm [1,0,3,2]
    if constexpr (N >= 4) v += pc_dpp<0x4E>(v);   // quad_perm [2,3,0,1]
    if constexpr (N >= 8) v += pc_dpp<0x141>(v);  // row_half_mirror
    if constexpr (N >= 16) v += pc_dpp<0x140>(v); // row_mirror
    return v;
}

// Sum of the widths that D header codes of HB bits (LSB first in hi:lo)
// stand for: code c is width c, except the largest code 2^HB - 1, which is
// width w = c + 1 (Section 4.3: a width of w - 1 never occurs). Summed with
// byte sums (HB = 4) or bit-plane popcounts (HB = 3) instead of one code at
// a time.
__host__ __device__ constexpr uint64_t pc_plane(int D, int HB, int k) {
    uint64_t m = 0;
    for (int j = 0; j < D; ++j) m |= 1ull << (HB * j + k);
    return m;
}
template <int D, int HB> __device__ __forceinline__ uint32_t pc_width_sum(uint32_t lo, uint32_t hi) {
    static_assert(D * HB <= 64 && (HB == 3 || HB == 4), "header codes");
    if constexpr (HB == 4) {
        auto part = [](uint32_t x) -> uint32_t {
            const uint32_t s = (x & 0x0F0F0F0Fu) + ((x >> 4) & 0x0F0F0F0Fu);   // nibble pairs, per byte
            const uint32_t top = x & (x >> 1) & (x >> 2) & (x >> 3) & 0x11111111u;   // codes 15
            return __builtin_amdgcn_sad_u8(s, 0u, 0u) + (uint32_t)__builtin_popcount(top);
        };
        constexpr uint64_t M = pc_plane(D, 4, 0) * 15u;
        uint32_t t = part(lo & (uint32_t)M);
        if constexpr (D > 8) t += part(hi & (uint32_t)(M >> 32));
        return t;
    } else {
        constexpr uint64_t M0 = pc_plane(D, 3, 0), M1 = pc_plane(D, 3, 1), M2 = pc_plane(D, 3, 2);
        auto pc2 = [&](uint64_t m) -> uint32_t {
            return (uint32_t)__builtin_popcount(lo & (uint32_t)m) +
                   (D * 3 > 32 ? (uint32_t)__builtin_popcount(hi & (uint32_t)(m >> 32)) : 0u);
        };
        uint32_t t = pc2(M0) + 2 * pc2(M1) + 4 * pc2(M2);
        // codes 7: all three bits set
        const uint32_t lo1 = __builtin_amdgcn_alignbit(hi, lo, 1), lo2 = __builtin_amdgcn_alignbit(hi, lo, 2);
        t += (uint32_t)__builtin_popcount(lo & lo1 & lo2 & (uint32_t)M0);
        if constexpr (D * 3 > 32) t += (uint32_t)__builtin_popcount(hi & (hi >> 1) & (hi >> 2) & (uint32_t)(M0 >> 32));
        return t;
    }
}

// a * (low w bits of d, sign-extended), one v_mul_i32_i24 with an SDWA
// operand (a within 24 bits).
template <int W> __device__ __forceinline__ int32_t pc_mul_sext(int32_t a, int32_t d) {
    if constexpr (W == 16) return __mul24(a, (int32_t)(int16_t)d);
    else return mul24_sext8(a, d);
}

// Unzigzag of two 16-bit (four 8-bit) fields of a dword at once.
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t unzigzag16x2(uint32_t zz) {
    const u16x2 v = __builtin_bit_cast(u16x2, zz);
    const u16x2 one = {1, 1}, zero = {0, 0};
    return __builtin_bit_cast(uint32_t, (u16x2)((v >> one) ^ (zero - (v & one))));
}
__device__ __forceinline__ uint32_t unzigzag8x4(uint32_t zz) {
    const uint32_t low = zz & 0x01010101u;
    return ((zz >> 1) & 0x7F7F7F7Fu) ^ ((low << 8) - low);
}

// The 32 bits starting at bit p of an LDS word array (two aligned reads).
__device__ __forceinline__ uint32_t lds_bits32(const uint32_t *w, uint32_t p) {
    const uint32_t *q = w + (p >> 5);
    return __builtin_amdgcn_alignbit(q[1], q[0], p);
}

// Segments per workgroup: the whole column groups that NC consumer
// wavefronts hold, rounded down to a multiple of the producer count.
__host__ __device__ constexpr uint32_t pc_spw(uint32_t D, uint32_t NP, uint32_t NC) {
    return (64 * NC / D) / NP * NP;
}
__host__ __device__ constexpr uint32_t pc_pow2(uint32_t D) { return D <= 1 ? 1u : 2 * pc_pow2((D + 1) / 2); }

template <int W, int D, int CB, int NP, int NC> struct PcGeom {
    static constexpr uint32_t HB = W == 8 ? 3 : 4;
    static constexpr uint32_t WB = W / 8;
    static constexpr uint32_t DP = pc_pow2(D);                     // unpack lanes per (segment, block)
    static constexpr uint32_t CHAINS = 64 * NC;                    // consumer lanes per workgroup
    static constexpr uint32_t SPW = pc_spw(D, NP, NC);             // segments per workgroup
    static constexpr uint32_t USED = SPW * D;                      // consumer lanes with a column chain
    static constexpr uint32_t SPP = SPW / NP;                      // segments per producer wave
    static constexpr uint32_t MAXREC = 8 * D * WB;                 // largest record payload
    static constexpr uint32_t HU = (CB * D * HB / 8 + 28 + 15) / 16;   // header window units
    static constexpr uint32_t PU = (CB * MAXREC + 24 + 15) / 16;       // payload window units
    static constexpr uint32_t NU = HU + PU;
    // producer/consumer form: each producer parses and stages its own segments
    static constexpr uint32_t PAIRS = SPP * CB;                    // (segment, candidate) per producer
    static constexpr uint32_t PPASS = (PAIRS + 63) / 64;           // parse passes
    // pipelined form: one parser wave for all segments
    static constexpr uint32_t PPAIRS = SPW * CB;                   // (segment, candidate) of the parser
    static constexpr uint32_t PPPASS = (PPAIRS + 63) / 64;         // its parse passes
    static constexpr uint32_t LPS = 64 / SPW;                      // its staging lanes per segment
    static constexpr uint32_t SP2 = (NU + LPS - 1) / LPS;          // its staged units per lane
    static constexpr bool ROW = D * W > 32;                        // row-major payloads (reading R13)
    static constexpr uint32_t GF = 32 / W;                         // fields of one 32-bit read
    static constexpr uint32_t IL = ROW ? DP / GF : DP;             // unpack lanes per (segment, block)
    static constexpr uint32_t ITEMS = SPP * CB * IL;               // unpack items per producer
    static constexpr uint32_t IPASS = (ITEMS + 63) / 64;
    static constexpr uint32_t ZSTR = CB * 8 * WB + 16;             // error buffer bytes per chain
    static constexpr bool WIDE = D * WB >= 16;
    static constexpr uint32_t OSEG = CB * 8 * D * WB + (WIDE ? (D * WB + 15) & ~15u : 4);  // row image stride
    static constexpr uint32_t UPL = CB * 8 * WB / 16;              // 16-byte output units per lane
};

// Per-segment decoding state in LDS. src and dst are the segment's first
// container byte and first output row; everything a chunk needs is here, so
// one workgroup can decode segments of different containers.
struct PcSeg {
    uint32_t r, cursor, rle_rem, nrec;   // parse: next record, its payload byte, run blocks pending, records
    uint32_t nrow, hbase, pbase, ok;     // rows in whole blocks (x8), staged windows (16-aligned), usable
    const uint8_t *src;                  // segment's first container byte
    uint32_t ext, tail;                  // segment bytes, tail rows
    uint8_t *dst;                        // segment's first output row
    uint32_t sh;                         // FIRE shift (learn_shift + 2)
    int32_t acc_lo, acc_hi;              // FIRE accumulator range
    uint32_t bad, status, pad;           // corrupt, index of the status word
};

// One container (stream) of a batch, as the batched decoder sees it.
struct PcStream {
    const uint8_t *src;       // container (16-byte aligned)
    uint8_t *dst;             // output rows (16-byte aligned)
    uint64_t data_start, data_bytes, rows;
    uint32_t nseg, S, sh;
    int32_t acc_lo, acc_hi;
    uint32_t pad;
};

// Validate segment `seg` of a container and fill its state: offsets from the
// container's table, extents checked against its data bytes, the record
// count read from the segment itself.
__device__ __forceinline__ void pc_seg_init(PcSeg &sg, const uint8_t *src, uint64_t data_start, uint64_t data_bytes,
                                            uint32_t nseg, uint64_t rows, uint32_t S, uint32_t seg, uint32_t D,
                                            uint32_t HB, uint32_t WB, uint8_t *dst) {
    sg.src = src; sg.dst = dst; sg.ext = 0; sg.nrec = 0; sg.nrow = 0; sg.tail = 0;
    sg.r = 0; sg.cursor = 4; sg.rle_rem = 0; sg.hbase = 0; sg.pbase = 0; sg.ok = 0; sg.bad = 0;
    if (seg >= nseg) { sg.bad = 1; return; }
    const uint64_t a = gld64(src + 64 + 8ull * seg), b = gld64(src + 64 + 8ull * (seg + 1));
    const uint32_t nr = (uint32_t)min((uint64_t)S, rows - (uint64_t)seg * S);
    sg.tail = nr & 7u;
    sg.dst = dst + (uint64_t)seg * S * D * WB;
    if (a <= b && b <= data_bytes && !((a | b) & 15u) && b - a >= 16 && b - a <= 0x7FFFFFF0ull) {
        sg.src = src + data_start + a;
        sg.ext = (uint32_t)(b - a);
        sg.nrec = gld32(sg.src);
        sg.ok = sg.nrec <= (nr >> 3) ? 1u : 0u;
    }
    if (sg.ok) {
        sg.nrow = nr & ~7u;
        sg.cursor = 4 + (uint32_t)(((uint64_t)sg.nrec * D * HB + 7) >> 3);
    } else {
        sg.bad = 1;
    }
    sg.pbase = sg.cursor & ~15u;
}

// Producer/consumer form: NP producer wavefronts parse, stage and unpack
// their own segments' chunk t while the consumer runs the recurrence of
// chunk t-1; one barrier per chunk. Decodes the segments whose state the
// producers put in SEG (nchunks chunks of kPcChunkBlocks blocks). Called by
// all threads of the workgroup.
template <int W, bool FIRE, int D, int NP, int NC, typename Init>
__device__ __forceinline__ void pc_decode_group(uint32_t nchunks, Init init, int32_t *__restrict__ status) {
    constexpr int CB = kPcChunkBlocks;
    using G = PcGeom<W, D, CB, NP, NC>;
    constexpr uint32_t HB = G::HB, WB = G::WB, SPW = G::SPW, SPP = G::SPP, HU = G::HU, NU = G::NU;
    constexpr uint32_t ZSTR = G::ZSTR, OSEG = G::OSEG;
    constexpr bool ROW = D * W > 32;   // row-major payloads (reading R13)
    static_assert(SPP * NP == SPW && SPP >= 1 && SPP <= 64 && CB <= 16 && G::DP <= 16, "geometry");
    static_assert(!G::ROW || G::IL >= 2, "row-major items hold whole column groups");

    // One LDS arena, staging windows first: field addresses then need no base.
    constexpr uint32_t O_ZB = SPW * NU * 16;                       // [segment][header window | payload window]
    constexpr uint32_t O_OUT = O_ZB + 2 * G::CHAINS * ZSTR;        // [buffer][chain] errors of a chunk
    // Output rows of a chunk. With at most D + 1 segments per workgroup
    // (D >= 7), the consumer writes them over the errors it has just read:
    // the row image of segment s lies inside the error buffers of its own D
    // chains (16 * D bytes more than its rows), shifted by OST * s bytes so
    // that the images start in different LDS banks. Otherwise a row image
    // [segment] of its own. Consumer lanes without a column chain (D not
    // dividing the wavefront) write a discard image.
    constexpr uint32_t ZPAR = G::CHAINS * ZSTR, ROWB = CB * 8 * D * WB;
    constexpr bool REUSE = SPW <= D + 1;
    constexpr uint32_t OST = (SPW - 1) * ((D * WB + 15) & ~15u) <= 16 * D ? (D * WB + 15) & ~15u : 16u;
    static_assert(!REUSE || (ZSTR == CB * 8 * WB + 16 && (SPW - 1) * OST <= 16 * D && (D * ZSTR) % 16 == 0),
                  "a segment's row image fits its chains' error buffers");
    constexpr uint32_t NOUT = REUSE ? 0u : G::USED < G::CHAINS ? SPW + 1 : SPW;
    constexpr uint32_t O_DIS = O_OUT + NOUT * OSEG;                   // discard image (REUSE)
    constexpr uint32_t O_REC = (O_DIS + (REUSE && G::USED < G::CHAINS ? ROWB : 0u) + 15) & ~15u;
    constexpr uint32_t O_BM = O_REC + SPW * CB * 16;               // [segment][candidate]: codes lo, hi, payload bit, bits per row
    constexpr uint32_t O_SEG = (O_BM + SPW * CB * 4 + 15) & ~15u;  // [segment][block]: candidate or kPcZero
    constexpr uint32_t O_END = O_SEG + SPW * (uint32_t)sizeof(PcSeg);
    __shared__ u32x4 ARENA[O_END / 16];
    u32x4 *const STG = ARENA;
    u32x4 *const ZB4 = reinterpret_cast<u32x4 *>(reinterpret_cast<uint8_t *>(ARENA) + O_ZB);
    u32x4 *const REC = reinterpret_cast<u32x4 *>(reinterpret_cast<uint8_t *>(ARENA) + O_REC);
    uint32_t *const BM = reinterpret_cast<uint32_t *>(reinterpret_cast<uint8_t *>(ARENA) + O_BM);
    PcSeg *const SEG = reinterpret_cast<PcSeg *>(reinterpret_cast<uint8_t *>(ARENA) + O_SEG);
    static_assert(O_END % 16 == 0 && sizeof(PcSeg) % 16 == 0, "arena layout");
    const uint32_t *const stgw = reinterpret_cast<const uint32_t *>(STG);
    uint8_t *const zb = reinterpret_cast<uint8_t *>(ZB4);
    uint8_t *const arena = reinterpret_cast<uint8_t *>(ARENA);

    const uint32_t tid = threadIdx.x;
    const uint32_t wave = tid >> 6, lane = tid & 63;
    const bool consumer = wave >= NP;
    const uint32_t ps0 = (consumer ? 0u : wave) * SPP;   // a producer's first segment

    // ---- producers: segment state and the first chunk's windows --------------
    // staging: each lane moves units of one segment (64 / SPP lanes per segment),
    // so it reads that segment's state once per chunk
    constexpr uint32_t LPS = 64 / SPP;                  // lanes per segment
    constexpr uint32_t SP2 = (NU + LPS - 1) / LPS;      // units per lane
    const bool st_on = lane < LPS * SPP;
    const uint32_t st_s = ps0 + min(lane / LPS, SPP - 1), st_k = lane % LPS;
    u32x4 reg[SP2];
    auto stage_issue = [&]() {
        const PcSeg &sg = SEG[st_s];
        const uint8_t *const src = sg.src;
        const uint32_t ext = sg.ok ? sg.ext : 0u, hbase = sg.hbase, pbase = sg.pbase;
#pragma unroll
        for (uint32_t t = 0; t < SP2; ++t) {
            const uint32_t k = st_k + LPS * t;
            const uint32_t off = k < HU ? hbase + 16 * k : pbase + 16 * (k - HU);
            u32x4 v = {0u, 0u, 0u, 0u};
            // only whole 16-byte units inside the segment (its extent is a multiple of 16)
            if (st_on && k < NU && off + 16 <= ext) v = gld128(src + off);
            reg[t] = v;
        }
    };
    auto stage_commit = [&]() {
#pragma unroll
        for (uint32_t t = 0; t < SP2; ++t) {
            const uint32_t k = st_k + LPS * t;
            if (st_on && k < NU) STG[st_s * NU + k] = reg[t];
        }
    };
    if (!consumer) {
        if (lane < SPP) init(SEG[ps0 + lane], ps0 + lane);
        wave_sync();
        stage_issue();
        stage_commit();
    }
    __syncthreads();

    // ---- consumer state: one column chain per lane ----------------------------
    const uint32_t chain = (wave - NP) * 64 + lane;   // consumers only
    const bool c_on = chain < G::USED;
    const uint32_t cs = c_on ? chain / D : SPW, cj = c_on ? chain % D : 0u;
    uint32_t x = 0;
    int32_t delta = 0, acc = 0;
    uint32_t c_sh = 0, c_nb = 0;
    int32_t c_lo = 0, c_hi = 0;
    uint8_t *c_dst = nullptr;
    if (consumer && c_on) {
        const PcSeg &q = SEG[cs];
        c_sh = q.sh; c_lo = q.acc_lo; c_hi = q.acc_hi; c_dst = q.dst; c_nb = q.nrow >> 3;
    }

    for (uint32_t t = 0; t <= nchunks; ++t) {
        if (!consumer && t < nchunks) {
            const uint32_t c = t;
            // ---- parse: lanes = (segment, candidate record) -----------------
#pragma unroll
            for (uint32_t pp = 0; pp < G::PPASS; ++pp) {
                const uint32_t pr = lane + 64 * pp;
                const uint32_t sl = pr / CB, k = pr % CB;
                const uint32_t s = ps0 + min(sl, SPP - 1);
                const bool here = pr < G::PAIRS;
                const PcSeg sg = SEG[s];   // one read of the chunk's state
                const uint32_t nbk = sg.nrow >> 3;
                const uint32_t bic = c * CB < nbk ? min((uint32_t)CB, nbk - c * CB) : 0u;
                const uint32_t rr = sg.r + k;
                const bool valid = here && sg.ok && rr < sg.nrec;
                // header codes of record rr (D * HB <= 64 bits)
                const uint32_t hp = 32 + rr * D * HB - 8 * sg.hbase;   // bit in the header window
                const uint32_t *hw = stgw + s * NU * 4;
                const uint32_t cw_lo = lds_bits32(hw, hp);
                const uint32_t cw_hi = D * HB > 32 ? lds_bits32(hw, hp + 32) : 0u;
                const uint32_t total = pc_width_sum<D, HB>(cw_lo, cw_hi);
                const bool zero = total == 0;
                const uint32_t size = !valid ? 0u : zero ? 2u : (ROW ? 8 * ((total + 7) >> 3) : total);
                const uint32_t poff = sg.cursor + pc_incl<CB>(size, k) - size;   // payload byte of candidate k
                const uint32_t pb = poff - sg.pbase;                               // byte in the payload window
                const uint32_t *pw = hw + HU * 4;
                const uint32_t cnt = lds_bits32(pw, 8 * pb) & 0xFFFFu;
                const uint32_t nb = !valid ? 0u : zero ? cnt : 1u;
                const bool badk = valid && zero && cnt == 0;
                const uint32_t start = sg.rle_rem + pc_incl<CB>(nb, k) - nb;     // first block it covers
                const bool used = valid && start < bic;
                if (here) BM[s * CB + k] = kPcZero;
                wave_sync();
                if (used && !zero) {
                    u32x4 rec;
                    rec.x = cw_lo;
                    rec.y = cw_hi;
                    rec.z = 8 * ((s * NU + HU) * 16 + pb);   // payload bit in the staging array
                    rec.w = ROW ? 8 * ((total + 7) >> 3) : 0u;
                    REC[s * CB + k] = rec;
                    BM[s * CB + start] = k;
                }
                const uint32_t n_used = pc_total<CB>(used ? 1u : 0u);
                const uint32_t adv = pc_total<CB>(used ? size : 0u);
                const uint32_t cov = sg.rle_rem + pc_total<CB>(used ? nb : 0u);
                const uint32_t nbad = pc_total<CB>(badk ? 1u : 0u);
                const uint32_t r1 = sg.r + n_used, cur1 = sg.cursor + adv;
                wave_sync();
                if (here && k == 0) {
                    PcSeg &ns = SEG[s];
                    if (nbad > 0 || (bic > 0 && cov < bic)) ns.bad = 1;
                    ns.r = r1;
                    ns.cursor = cur1;
                    ns.rle_rem = cov > bic ? cov - bic : 0u;
                    ns.hbase = (4 + ((r1 * D * HB) >> 3)) & ~15u;
                    ns.pbase = cur1 & ~15u;
                }
            }
            wave_sync();
            // ---- stage the next chunk's windows -----------------------------
            if (c + 1 < nchunks) stage_issue();
            // ---- unpack ------------------------------------------------------
            // One aligned two-dword LDS read and a funnel shift give 32
            // payload bits: GF = 32 / W fields at once. Row-major payloads
            // (fields of one row side by side): lanes = (segment, block, GF
            // adjacent columns), one read per row. Column-major payloads (a
            // column's 8 fields side by side): lanes = (segment, block,
            // column), one read per GF rows. All LDS reads of the chunk's
            // items are issued in three batches (block map, records, fields)
            // so that their latency is paid three times per chunk rather than
            // three times per item.
            uint8_t *const zbuf = zb + (c & 1) * G::CHAINS * ZSTR;
            constexpr uint32_t IP = G::IPASS, IL = G::IL, GF = G::GF;
            constexpr uint32_t NRD = ROW ? 8 : 8 / GF;   // reads per item
            uint32_t kk[IP];
#pragma unroll
            for (uint32_t ip = 0; ip < IP; ++ip) {
                const uint32_t it = lane + 64 * ip;
                const uint32_t b = (it / IL) % CB, s = ps0 + min(it / (IL * CB), SPP - 1);
                kk[ip] = BM[s * CB + b];
            }
            u32x4 rr[IP];
#pragma unroll
            for (uint32_t ip = 0; ip < IP; ++ip) {
                const uint32_t it = lane + 64 * ip;
                const uint32_t s = ps0 + min(it / (IL * CB), SPP - 1);
                rr[ip] = REC[s * CB + (kk[ip] & (CB - 1))];
            }
            // widths of the item's columns (0 past D), the bit offset of each
            // field group and the 32 bits read there
            uint32_t wdt[IP][ROW ? GF : 1], fw[IP][NRD];
#pragma unroll
            for (uint32_t ip = 0; ip < IP; ++ip) {
                const uint32_t it = lane + 64 * ip;
                const uint32_t q = it % IL;                       // column group (ROW) or column
                const bool nz = it < G::ITEMS && kk[ip] != kPcZero;
                const u32x4 rec = rr[ip];
                constexpr uint32_t NCOL = ROW ? GF : 1;          // columns of the item
                constexpr uint32_t CBITS = NCOL * HB;            // their header code bits
                const uint32_t bp = q * CBITS;
                const uint32_t cw = bp >= 32 ? rec.y >> (bp - 32) : __builtin_amdgcn_alignbit(rec.y, rec.x, bp);
                uint32_t sum = 0;
#pragma unroll
                for (uint32_t g = 0; g < NCOL; ++g) {
                    const uint32_t code = __builtin_amdgcn_ubfe(cw, g * HB, HB);
                    const uint32_t width = nz && q * NCOL + g < (uint32_t)D ? code + ((code + 1) >> HB) : 0u;   // code w-1 stands for width w
                    wdt[ip][ROW ? g : 0] = width;
                    sum += width;
                }
                const uint32_t off = pc_incl<IL>(sum, q) - sum;  // bits before the item's first column
                // ROW: field (i, first column) at rec.z + off + i * (row bits);
                // column-major: fields GF*k .. GF*k+GF-1 at rec.z + 8*off + GF*k*width
                const uint32_t p0 = nz ? rec.z + (ROW ? off : 8 * off) : 0u;
                const uint32_t step = !nz ? 0u : ROW ? rec.w : GF * sum;
#pragma unroll
                for (uint32_t r = 0; r < NRD; ++r) {
                    const uint32_t p = p0 + r * step;
                    const uint32_t *qd = stgw + (p >> 5);
                    fw[ip][r] = __builtin_amdgcn_alignbit(qd[1], qd[0], p);
                }
            }
#pragma unroll
            for (uint32_t ip = 0; ip < IP; ++ip) {
                const uint32_t it = lane + 64 * ip;
                const uint32_t q = it % IL, b = (it / IL) % CB, s = ps0 + min(it / (IL * CB), SPP - 1);
                constexpr uint32_t NCOL = ROW ? GF : 1;
                uint32_t o = 0;
#pragma unroll
                for (uint32_t g = 0; g < NCOL; ++g) {
                    const uint32_t j = q * NCOL + g;
                    const uint32_t w = wdt[ip][ROW ? g : 0];
                    // the column's 8 zigzag codes
                    uint32_t z[8];
#pragma unroll
                    for (int i = 0; i < 8; ++i)
                        z[i] = ROW ? __builtin_amdgcn_ubfe(fw[ip][i], o, w)
                                   : __builtin_amdgcn_ubfe(fw[ip][i / GF], (i % GF) * w, w);
                    o += w;
                    if (it < G::ITEMS && j < (uint32_t)D) {
                        uint8_t *zp = zbuf + (s * D + j) * ZSTR + b * 8 * WB;
                        // zigzag codes packed 2 (or 4) per dword, then unzigzagged
                        // lane-wise: e = (z >> 1) ^ -(z & 1) in every 16-bit (8-bit) lane
                        if (WB == 2) {
                            u32x4 v;
                            v.x = unzigzag16x2(z[0] | (z[1] << 16));
                            v.y = unzigzag16x2(z[2] | (z[3] << 16));
                            v.z = unzigzag16x2(z[4] | (z[5] << 16));
                            v.w = unzigzag16x2(z[6] | (z[7] << 16));
                            *reinterpret_cast<u32x4 *>(zp) = v;
                        } else {
                            uint2 v;
                            v.x = unzigzag8x4(z[0] | (z[1] << 8) | (z[2] << 16) | (z[3] << 24));
                            v.y = unzigzag8x4(z[4] | (z[5] << 8) | (z[6] << 16) | (z[7] << 24));
                            *reinterpret_cast<uint2 *>(zp) = v;
                        }
                    }
                }
            }
            wave_sync();
            if (c + 1 < nchunks) stage_commit();
        } else if (consumer && t > 0) {
            const uint32_t c = t - 1;
            // ---- recurrence: lane = column chain ------------------------------
            const uint8_t *const zc = zb + (c & 1) * G::CHAINS * ZSTR + chain * ZSTR;
            // row image of segment cs (byte offset in the arena)
            const uint32_t ibase = REUSE ? O_ZB + (c & 1) * ZPAR + cs * (D * ZSTR + OST) : O_OUT + cs * OSEG;
            const uint32_t obase = (REUSE && !c_on ? O_DIS : ibase) + cj * WB;
            const uint32_t sh = c_sh;
            const int32_t acc_lo = c_lo, acc_hi = c_hi;
            // the whole chunk's errors first: one LDS wait per chunk
            uint32_t evs[CB][4];
#pragma unroll
            for (int b = 0; b < CB; ++b) {
                if (WB == 2) {
                    const u32x4 v = *reinterpret_cast<const u32x4 *>(zc + 16 * b);
                    evs[b][0] = v.x; evs[b][1] = v.y; evs[b][2] = v.z; evs[b][3] = v.w;
                } else {
                    const uint2 v = *reinterpret_cast<const uint2 *>(zc + 8 * b);
                    evs[b][0] = v.x; evs[b][1] = v.y; evs[b][2] = 0; evs[b][3] = 0;
                }
            }
            __builtin_amdgcn_sched_barrier(0);
            if (REUSE) wave_sync();   // every lane holds its errors before any writes rows over them
#pragma unroll
            for (int b = 0; b < CB; ++b) {
                const uint32_t *const ev = evs[b];
                const int32_t alpha = acc >> sh;
                int32_t grad = 0;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    // e: the packed field read as a signed w-bit word (the
                    // compiler takes it as a sign-extended SDWA operand)
                    const uint32_t word = ev[WB == 2 ? i >> 1 : i >> 2];
                    const int32_t e = WB == 2 ? ((i & 1) ? (int32_t)(int16_t)(word >> 16) : (int32_t)(int16_t)word)
                                              : (int32_t)(int8_t)(word >> (8 * (i & 3)));
                    if (FIRE) {
                        // delta = e + floor(alpha * delta_prev / 2^w) modulo 2^w.
                        // delta is kept unreduced: only its low w bits are
                        // read, sign-extended, and |alpha * delta_prev| < 2^31
                        // (2^15 for w = 8), so bits [w, 32) of the product
                        // are the floor (wrapping add of e * 2^w gives the same
                        // bits [w, 2w)).
                        const int32_t p = pc_mul_sext<W>(alpha, delta);
                        if (i & 1) grad += pc_mul_sext<W>(sgn_med3(e), delta);
                        delta = (W == 16 ? (p >> 16) : (int32_t)(int8_t)(p >> 8)) + e;
                        x += (uint32_t)delta;
                    } else {
                        x += (uint32_t)e;
                    }
                    const uint32_t o = obase + (uint32_t)((8 * b + i) * D * WB);
                    if (WB == 1) arena[o] = (uint8_t)x;
                    else *reinterpret_cast<uint16_t *>(arena + o) = (uint16_t)x;
                }
                if (FIRE) acc = min(max(acc + grad, acc_lo), acc_hi);
            }
            wave_sync();
            // ---- output: each segment's rows of this chunk ---------------------
            const uint32_t bic = c * CB < c_nb ? min((uint32_t)CB, c_nb - c * CB) : 0u;
            const uint32_t valid = bic * 8 * D * WB;
            // (lanes without a column chain, and segments without rows such as
            // a batch's empty work-list entries, whose dst is null, have valid
            // 0 and store nothing)
            uint8_t *const gp = valid ? c_dst + (size_t)c * CB * 8 * D * WB : c_dst;
#pragma unroll
            for (uint32_t u = 0; u < G::UPL; ++u) {
                const uint32_t lo = 16 * (cj + u * D);
                if (lo + 16 <= valid) {
                    u32x4 v;
                    if (REUSE || G::WIDE) {
                        v = *reinterpret_cast<const u32x4 *>(arena + ibase + lo);
                    } else {
                        const uint32_t *p = reinterpret_cast<const uint32_t *>(arena + ibase + lo);
                        v.x = p[0]; v.y = p[1]; v.z = p[2]; v.w = p[3];
                    }
                    gst128(gp + lo, v);
                } else if (lo + 8 == valid) {
                    const uint32_t *p = reinterpret_cast<const uint32_t *>(arena + ibase + lo);
                    gst32(gp + lo, p[0]);
                    gst32(gp + lo + 4, p[1]);
                }
            }
        }
        __syncthreads();
    }

    // ---- producers: final checks and raw tail rows (a stream's last segment) ----
    if (!consumer) {
        for (uint32_t s = ps0; s < ps0 + SPP; ++s) {
            PcSeg &sg = SEG[s];
            const uint32_t tb = sg.tail * D * WB;
            if (sg.ok && (sg.r != sg.nrec || sg.rle_rem != 0 || sg.cursor + tb > sg.ext)) {
                if (lane == 0) sg.bad = 1;
            } else if (sg.ok) {
                uint8_t *const tp = sg.dst + (size_t)sg.nrow * D * WB;
                for (uint32_t q = lane; q < tb; q += 64) gst8(tp + q, gld8(sg.src + sg.cursor + q));
            }
        }
        wave_sync();
        if (lane < SPP && SEG[ps0 + lane].bad && status) atomicOr(status + SEG[ps0 + lane].status, 1);
    }
}

// Pipelined form: decodes the segments whose state the parser puts in SEG
// (nchunks chunks of kPcChunkBlocks blocks). Called by all threads of the
// workgroup. The wavefronts form a four-stage pipeline over the chunks, one
// barrier per step: at step t the parser (wave 0) stores chunk t's staged
// windows, parses chunk t and issues the loads of chunk t+1's windows; the NP
// unpacking waves store chunk t-3's rows to global memory and unpack chunk
// t-1; the consumer runs the recurrence of chunk t-2 into a row image.
// Staging windows, records, error buffers and row images are double buffered
// by chunk parity. The consumer's recurrence is the longest stage, so it does
// nothing else.
template <int W, bool FIRE, int D, int NP, int NC, typename Init>
__device__ __forceinline__ void pc_decode_group_pipe(uint32_t nchunks, Init init, int32_t *__restrict__ status) {
    constexpr int CB = kPcChunkBlocks;
    using G = PcGeom<W, D, CB, NP, NC>;
    constexpr uint32_t HB = G::HB, WB = G::WB, SPW = G::SPW, SPP = G::SPP, HU = G::HU, NU = G::NU;
    constexpr uint32_t ZSTR = G::ZSTR;
    constexpr bool ROW = D * W > 32;   // row-major payloads (reading R13)
    static_assert(SPP * NP == SPW && SPP >= 1 && SPP <= 64 && SPW <= 64 && CB <= 16 && G::DP <= 16, "geometry");
    static_assert(!G::ROW || G::IL >= 2, "row-major items hold whole column groups");

    // One LDS arena, staging windows first: field addresses then need no base.
    constexpr uint32_t SLOT = SPW * NU * 16;                       // one chunk's windows
    constexpr uint32_t O_ZB = 2 * SLOT;                            // [parity][segment][header | payload window]
    // [parity][chain] errors of a chunk. Once the consumer holds a chunk's
    // errors in registers, it writes the chunk's output rows over them: the
    // row image of segment s lies inside the error buffers of s's own D
    // chains (which hold 16 * D bytes more than its rows), shifted by OST * s
    // bytes so that the images of different segments start in different LDS
    // banks. The unpacking wave that owns s stores that image in the next
    // step, before it unpacks its next chunk into the same buffers.
    constexpr uint32_t ZPAR = G::CHAINS * ZSTR;                     // one parity's error buffers
    constexpr uint32_t ROWB = CB * 8 * D * WB;                       // one segment's rows of a chunk
    constexpr uint32_t OST = (SPW - 1) * ((D * WB + 15) & ~15u) <= 16 * D ? (D * WB + 15) & ~15u : 16u;
    static_assert(ZSTR == CB * 8 * WB + 16 && (SPW - 1) * OST <= 16 * D && (D * ZSTR) % 16 == 0,
                  "a segment's row image fits its chains' error buffers");
    constexpr uint32_t O_DIS = O_ZB + 2 * ZPAR;                     // rows of consumer lanes without a chain
    constexpr uint32_t O_REC = O_DIS + (G::USED < G::CHAINS ? ROWB : 0u);
    constexpr uint32_t O_BM = O_REC + 2 * SPW * CB * 16;           // [parity][segment][candidate]: codes lo, hi, payload bit, bits per row
    constexpr uint32_t O_SEG = (O_BM + 2 * SPW * CB * 4 + 15) & ~15u;  // [parity][segment][block]: candidate or kPcZero
    constexpr uint32_t O_END = O_SEG + SPW * (uint32_t)sizeof(PcSeg);
    __shared__ u32x4 ARENA[O_END / 16];
    u32x4 *const STG = ARENA;
    u32x4 *const ZB4 = reinterpret_cast<u32x4 *>(reinterpret_cast<uint8_t *>(ARENA) + O_ZB);
    u32x4 *const REC = reinterpret_cast<u32x4 *>(reinterpret_cast<uint8_t *>(ARENA) + O_REC);
    uint32_t *const BM = reinterpret_cast<uint32_t *>(reinterpret_cast<uint8_t *>(ARENA) + O_BM);
    PcSeg *const SEG = reinterpret_cast<PcSeg *>(reinterpret_cast<uint8_t *>(ARENA) + O_SEG);
    static_assert(O_END % 16 == 0 && sizeof(PcSeg) % 16 == 0, "arena layout");
    const uint32_t *const stgw = reinterpret_cast<const uint32_t *>(STG);
    uint8_t *const zb = reinterpret_cast<uint8_t *>(ZB4);
    uint8_t *const arena = reinterpret_cast<uint8_t *>(ARENA);

    const uint32_t tid = threadIdx.x;
    const uint32_t wave = tid >> 6, lane = tid & 63;
    const bool parser = wave == 0;
    const bool consumer = wave > NP;
    const bool unpacker = !parser && !consumer;
    const uint32_t ps0 = unpacker ? (wave - 1) * SPP : 0u;   // an unpacking wave's first segment

    // ---- parser: segment state and the first chunk's windows ------------------
    // staging: each lane moves units of one segment (64 / SPW lanes per segment),
    // so it reads that segment's state once per chunk
    constexpr uint32_t LPS = G::LPS, SP2 = G::SP2;
    const bool st_on = lane < LPS * SPW;
    const uint32_t st_s = min(lane / LPS, SPW - 1), st_k = lane % LPS;
    u32x4 reg[SP2];
    // A staging lane's segment: its source and extent are fixed; its window
    // bases change with every chunk. Where the staging lanes of a segment
    // are its parse lanes (one parse pass, 64 / SPW = CB lanes per segment),
    // every such lane keeps the segment's parse state (next record, cursor,
    // pending run blocks, window bases) in registers, since each parse leaves
    // the new state in all of the segment's lanes; otherwise the parse and
    // the staging read it back from the segment state in LDS.
    constexpr bool BASES_IN_REGS = LPS == CB && G::PPPASS == 1;
    const uint8_t *st_src = nullptr;
    uint32_t st_ext = 0, nx_hb = 0, nx_pb = 0;
    uint32_t ps_r = 0, ps_cur = 0, ps_rle = 0, ps_nrow = 0, ps_nrec = 0, ps_ok = 0;
    auto stage_issue = [&]() {
        uint32_t hbase = nx_hb, pbase = nx_pb;
        if (!BASES_IN_REGS) {
            hbase = SEG[st_s].hbase;
            pbase = SEG[st_s].pbase;
        }
        const uint8_t *const src = st_src;
        const uint32_t ext = st_ext;
#pragma unroll
        for (uint32_t t = 0; t < SP2; ++t) {
            const uint32_t k = st_k + LPS * t;
            const uint32_t off = k < HU ? hbase + 16 * k : pbase + 16 * (k - HU);
            u32x4 v = {0u, 0u, 0u, 0u};
            // only whole 16-byte units inside the segment (its extent is a multiple of 16)
            if (st_on && k < NU && off + 16 <= ext) v = gld128(src + off);
            reg[t] = v;
        }
    };
    auto stage_commit = [&](uint32_t c) {
        u32x4 *const slot = STG + (c & 1) * (SLOT / 16);
#pragma unroll
        for (uint32_t t = 0; t < SP2; ++t) {
            const uint32_t k = st_k + LPS * t;
            if (st_on && k < NU) slot[st_s * NU + k] = reg[t];
        }
    };
    if (parser) {
        if (lane < SPW) init(SEG[lane], lane);
        wave_sync();
        const PcSeg &sg = SEG[st_s];
        st_src = sg.src;
        st_ext = sg.ok ? sg.ext : 0u;
        nx_hb = sg.hbase;
        nx_pb = sg.pbase;
        ps_r = sg.r; ps_cur = sg.cursor; ps_rle = sg.rle_rem;
        ps_nrow = sg.nrow; ps_nrec = sg.nrec; ps_ok = sg.ok;
        stage_issue();
    }
    __syncthreads();

    // ---- consumer state: one column chain per lane ----------------------------
    const uint32_t chain = consumer ? (wave - NP - 1) * 64 + lane : 0u;
    const bool c_on = consumer && chain < G::USED;
    const uint32_t cs = c_on ? chain / D : SPW, cj = c_on ? chain % D : 0u;
    uint32_t x = 0;
    int32_t delta = 0, acc = 0;
    uint32_t c_sh = 0;
    int32_t c_lo = 0, c_hi = 0;
    if (c_on) {
        const PcSeg &q = SEG[cs];
        c_sh = q.sh; c_lo = q.acc_lo; c_hi = q.acc_hi;
    }

    for (uint32_t t = 0; t < nchunks + 3; ++t) {
        if (parser && t < nchunks) {
            const uint32_t c = t;
            stage_commit(c);
            wave_sync();
            // ---- parse: lanes = (segment, candidate record) -----------------
            const uint32_t *const slotw = stgw + (c & 1) * (SLOT / 4);
#pragma unroll
            for (uint32_t pp = 0; pp < G::PPPASS; ++pp) {
                const uint32_t pr = lane + 64 * pp;
                const uint32_t sl = pr / CB, k = pr % CB;
                const uint32_t s = min(sl, SPW - 1);
                const bool here = pr < G::PPAIRS;
                // the segment's state at the chunk's start (one LDS read, or
                // none: see BASES_IN_REGS)
                struct { uint32_t r, cursor, rle_rem, nrec, nrow, hbase, pbase, ok; } sg;
                if (BASES_IN_REGS) {
                    sg = {ps_r, ps_cur, ps_rle, ps_nrec, ps_nrow, nx_hb, nx_pb, ps_ok};
                } else {
                    const PcSeg q = SEG[s];
                    sg = {q.r, q.cursor, q.rle_rem, q.nrec, q.nrow, q.hbase, q.pbase, q.ok};
                }
                const uint32_t nbk = sg.nrow >> 3;
                const uint32_t bic = c * CB < nbk ? min((uint32_t)CB, nbk - c * CB) : 0u;
                const uint32_t rr = sg.r + k;
                const bool valid = here && sg.ok && rr < sg.nrec;
                // header codes of record rr (D * HB <= 64 bits)
                const uint32_t hp = 32 + rr * D * HB - 8 * sg.hbase;   // bit in the header window
                const uint32_t *hw = slotw + s * NU * 4;
                const uint32_t cw_lo = lds_bits32(hw, hp);
                const uint32_t cw_hi = D * HB > 32 ? lds_bits32(hw, hp + 32) : 0u;
                const uint32_t total = pc_width_sum<D, HB>(cw_lo, cw_hi);
                const bool zero = total == 0;
                const uint32_t size = !valid ? 0u : zero ? 2u : (ROW ? 8 * ((total + 7) >> 3) : total);
                const uint32_t poff = sg.cursor + pc_incl<CB>(size, k) - size;   // payload byte of candidate k
                const uint32_t pb = poff - sg.pbase;                               // byte in the payload window
                const uint32_t *pw = hw + HU * 4;
                const uint32_t cnt = lds_bits32(pw, 8 * pb) & 0xFFFFu;
                const uint32_t nb = !valid ? 0u : zero ? cnt : 1u;
                const bool badk = valid && zero && cnt == 0;
                const uint32_t start = sg.rle_rem + pc_incl<CB>(nb, k) - nb;     // first block it covers
                const bool used = valid && start < bic;
                uint32_t *const bm = BM + (c & 1) * SPW * CB;
                if (here) bm[s * CB + k] = kPcZero;
                wave_sync();
                if (used && !zero) {
                    u32x4 rec;
                    rec.x = cw_lo;
                    rec.y = cw_hi;
                    // payload bit in the staging array (this chunk's parity slot)
                    rec.z = 8 * ((c & 1) * SLOT + (s * NU + HU) * 16 + pb);
                    rec.w = ROW ? 8 * ((total + 7) >> 3) : 0u;
                    REC[(c & 1) * SPW * CB + s * CB + k] = rec;
                    bm[s * CB + start] = k;
                }
                const uint32_t n_used = pc_total<CB>(used ? 1u : 0u);
                const uint32_t adv = pc_total<CB>(used ? size : 0u);
                const uint32_t cov = sg.rle_rem + pc_total<CB>(used ? nb : 0u);
                const uint32_t nbad = pc_total<CB>(badk ? 1u : 0u);
                const uint32_t r1 = sg.r + n_used, cur1 = sg.cursor + adv;
                if (BASES_IN_REGS) {
                    // this lane's segment is its staging segment (s == st_s)
                    nx_hb = (4 + ((r1 * D * HB) >> 3)) & ~15u;
                    nx_pb = cur1 & ~15u;
                    ps_r = r1;
                    ps_cur = cur1;
                    ps_rle = cov > bic ? cov - bic : 0u;
                }
                wave_sync();
                if (here && k == 0) {
                    PcSeg &ns = SEG[s];
                    if (nbad > 0 || (bic > 0 && cov < bic)) ns.bad = 1;
                    ns.r = r1;
                    ns.cursor = cur1;
                    ns.rle_rem = cov > bic ? cov - bic : 0u;
                    ns.hbase = (4 + ((r1 * D * HB) >> 3)) & ~15u;
                    ns.pbase = cur1 & ~15u;
                }
            }
            wave_sync();
            // ---- the next chunk's windows: loads in flight over the step ------
            if (c + 1 < nchunks) stage_issue();
        } else if (unpacker) {
          if (t >= 3) {
            // ---- output: this wave's segments' rows of chunk t-3 ----------------
            // lanes = 16-byte units of the segments' row images
            const uint32_t c = t - 3;
            constexpr uint32_t NUS = CB * 8 * D * WB / 16;   // units of one segment's chunk
            constexpr uint32_t OPASS = (SPP * NUS + 63) / 64;
            const uint8_t *const img = zb + (c & 1) * ZPAR;
#pragma unroll
            for (uint32_t op = 0; op < OPASS; ++op) {
                const uint32_t u = lane + 64 * op;
                const uint32_t s = ps0 + min(u / NUS, SPP - 1), lo = 16 * (u % NUS);
                const PcSeg &sg = SEG[s];
                const uint32_t nbk = sg.nrow >> 3;
                const uint32_t bic = c * CB < nbk ? min((uint32_t)CB, nbk - c * CB) : 0u;
                // rows of the chunk in whole blocks (none for a segment that
                // failed its checks: nrow is 0 there); units past them, and
                // lanes past the wave's units, store nothing
                const uint32_t valid = u < SPP * NUS ? bic * 8 * D * WB : 0u;
                uint8_t *const gp = sg.dst + (size_t)c * CB * 8 * D * WB;
                const uint8_t *const si = img + s * (D * ZSTR + OST) + lo;
                if (lo + 16 <= valid) {
                    gst128(gp + lo, *reinterpret_cast<const u32x4 *>(si));
                } else if (lo + 8 == valid) {
                    const uint32_t *q = reinterpret_cast<const uint32_t *>(si);
                    gst32(gp + lo, q[0]);
                    gst32(gp + lo + 4, q[1]);
                }
            }
            wave_sync();   // every lane has read the images before any unpacks over them
          }
          if (t >= 1 && t <= nchunks) {
            const uint32_t c = t - 1;
            // ---- unpack ------------------------------------------------------
            // One aligned two-dword LDS read and a funnel shift give 32
            // payload bits: GF = 32 / W fields at once. Row-major payloads
            // (fields of one row side by side): lanes = (segment, block, GF
            // adjacent columns), one read per row. Column-major payloads (a
            // column's 8 fields side by side): lanes = (segment, block,
            // column), one read per GF rows. All LDS reads of the chunk's
            // items are issued in three batches (block map, records, fields)
            // so that their latency is paid three times per chunk rather than
            // three times per item.
            uint8_t *const zbuf = zb + (c & 1) * G::CHAINS * ZSTR;
            const uint32_t *const bm = BM + (c & 1) * SPW * CB;
            const u32x4 *const recs = REC + (c & 1) * SPW * CB;
            constexpr uint32_t IP = G::IPASS, IL = G::IL, GF = G::GF;
            constexpr uint32_t NRD = ROW ? 8 : 8 / GF;   // reads per item
            uint32_t kk[IP];
#pragma unroll
            for (uint32_t ip = 0; ip < IP; ++ip) {
                const uint32_t it = lane + 64 * ip;
                const uint32_t b = (it / IL) % CB, s = ps0 + min(it / (IL * CB), SPP - 1);
                kk[ip] = bm[s * CB + b];
            }
            u32x4 rr[IP];
#pragma unroll
            for (uint32_t ip = 0; ip < IP; ++ip) {
                const uint32_t it = lane + 64 * ip;
                const uint32_t s = ps0 + min(it / (IL * CB), SPP - 1);
                rr[ip] = recs[s * CB + (kk[ip] & (CB - 1))];
            }
            // widths of the item's columns (0 past D), the bit offset of each
            // field group and the 32 bits read there
            uint32_t wdt[IP][ROW ? GF : 1], fw[IP][NRD];
#pragma unroll
            for (uint32_t ip = 0; ip < IP; ++ip) {
                const uint32_t it = lane + 64 * ip;
                const uint32_t q = it % IL;                       // column group (ROW) or column
                const bool nz = it < G::ITEMS && kk[ip] != kPcZero;
                const u32x4 rec = rr[ip];
                constexpr uint32_t NCOL = ROW ? GF : 1;          // columns of the item
                constexpr uint32_t CBITS = NCOL * HB;            // their header code bits
                const uint32_t bp = q * CBITS;
                const uint32_t cw = bp >= 32 ? rec.y >> (bp - 32) : __builtin_amdgcn_alignbit(rec.y, rec.x, bp);
                uint32_t sum = 0;
#pragma unroll
                for (uint32_t g = 0; g < NCOL; ++g) {
                    const uint32_t code = __builtin_amdgcn_ubfe(cw, g * HB, HB);
                    const uint32_t width = nz && q * NCOL + g < (uint32_t)D ? code + ((code + 1) >> HB) : 0u;   // code w-1 stands for width w
                    wdt[ip][ROW ? g : 0] = width;
                    sum += width;
                }
                const uint32_t off = pc_incl<IL>(sum, q) - sum;  // bits before the item's first column
                // ROW: field (i, first column) at rec.z + off + i * (row bits);
                // column-major: fields GF*k .. GF*k+GF-1 at rec.z + 8*off + GF*k*width
                const uint32_t p0 = nz ? rec.z + (ROW ? off : 8 * off) : 0u;
                const uint32_t step = !nz ? 0u : ROW ? rec.w : GF * sum;
#pragma unroll
                for (uint32_t r = 0; r < NRD; ++r) {
                    const uint32_t p = p0 + r * step;
                    const uint32_t *qd = stgw + (p >> 5);
                    fw[ip][r] = __builtin_amdgcn_alignbit(qd[1], qd[0], p);
                }
            }
#pragma unroll
            for (uint32_t ip = 0; ip < IP; ++ip) {
                const uint32_t it = lane + 64 * ip;
                const uint32_t q = it % IL, b = (it / IL) % CB, s = ps0 + min(it / (IL * CB), SPP - 1);
                constexpr uint32_t NCOL = ROW ? GF : 1;
                uint32_t o = 0;
#pragma unroll
                for (uint32_t g = 0; g < NCOL; ++g) {
                    const uint32_t j = q * NCOL + g;
                    const uint32_t w = wdt[ip][ROW ? g : 0];
                    // the column's 8 zigzag codes
                    uint32_t z[8];
#pragma unroll
                    for (int i = 0; i < 8; ++i)
                        z[i] = ROW ? __builtin_amdgcn_ubfe(fw[ip][i], o, w)
                                   : __builtin_amdgcn_ubfe(fw[ip][i / GF], (i % GF) * w, w);
                    o += w;
                    if (it < G::ITEMS && j < (uint32_t)D) {
                        uint8_t *zp = zbuf + (s * D + j) * ZSTR + b * 8 * WB;
                        // zigzag codes packed 2 (or 4) per dword, then unzigzagged
                        // lane-wise: e = (z >> 1) ^ -(z & 1) in every 16-bit (8-bit) lane
                        if (WB == 2) {
                            u32x4 v;
                            v.x = unzigzag16x2(z[0] | (z[1] << 16));
                            v.y = unzigzag16x2(z[2] | (z[3] << 16));
                            v.z = unzigzag16x2(z[4] | (z[5] << 16));
                            v.w = unzigzag16x2(z[6] | (z[7] << 16));
                            *reinterpret_cast<u32x4 *>(zp) = v;
                        } else {
                            uint2 v;
                            v.x = unzigzag8x4(z[0] | (z[1] << 8) | (z[2] << 16) | (z[3] << 24));
                            v.y = unzigzag8x4(z[4] | (z[5] << 8) | (z[6] << 16) | (z[7] << 24));
                            *reinterpret_cast<uint2 *>(zp) = v;
                        }
                    }
                }
            }
          }
        } else if (consumer && t >= 2 && t <= nchunks + 1) {
            const uint32_t c = t - 2;
            // ---- recurrence: lane = column chain ------------------------------
            const uint8_t *const zc = zb + (c & 1) * G::CHAINS * ZSTR + chain * ZSTR;
            const uint32_t obase = c_on ? O_ZB + (c & 1) * ZPAR + cs * (D * ZSTR + OST) + cj * WB : O_DIS;
            const uint32_t sh = c_sh;
            const int32_t acc_lo = c_lo, acc_hi = c_hi;
            // the whole chunk's errors first: one LDS wait per chunk, and every
            // lane holds its errors before any writes rows over them
            uint32_t evs[CB][4];
#pragma unroll
            for (int b = 0; b < CB; ++b) {
                if (WB == 2) {
                    const u32x4 v = *reinterpret_cast<const u32x4 *>(zc + 16 * b);
                    evs[b][0] = v.x; evs[b][1] = v.y; evs[b][2] = v.z; evs[b][3] = v.w;
                } else {
                    const uint2 v = *reinterpret_cast<const uint2 *>(zc + 8 * b);
                    evs[b][0] = v.x; evs[b][1] = v.y; evs[b][2] = 0; evs[b][3] = 0;
                }
            }
            __builtin_amdgcn_sched_barrier(0);
            wave_sync();
#pragma unroll
            for (int b = 0; b < CB; ++b) {
                const uint32_t *const ev = evs[b];
                const int32_t alpha = acc >> sh;
                int32_t grad = 0;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    // e: the packed field read as a signed w-bit word (the
                    // compiler takes it as a sign-extended SDWA operand)
                    const uint32_t word = ev[WB == 2 ? i >> 1 : i >> 2];
                    const int32_t e = WB == 2 ? ((i & 1) ? (int32_t)(int16_t)(word >> 16) : (int32_t)(int16_t)word)
                                              : (int32_t)(int8_t)(word >> (8 * (i & 3)));
                    if (FIRE) {
                        // delta = e + floor(alpha * delta_prev / 2^w) modulo 2^w.
                        // delta is kept unreduced: only its low w bits are
                        // read, sign-extended, and |alpha * delta_prev| < 2^31
                        // (2^15 for w = 8), so bits [w, 32) of the product
                        // are the floor (wrapping add of e * 2^w gives the same
                        // bits [w, 2w)).
                        const int32_t p = pc_mul_sext<W>(alpha, delta);
                        if (i & 1) grad += pc_mul_sext<W>(sgn_med3(e), delta);
                        delta = (W == 16 ? (p >> 16) : (int32_t)(int8_t)(p >> 8)) + e;
                        x += (uint32_t)delta;
                    } else {
                        x += (uint32_t)e;
                    }
                    const uint32_t o = obase + (uint32_t)((8 * b + i) * D * WB);
                    if (WB == 1) arena[o] = (uint8_t)x;
                    else *reinterpret_cast<uint16_t *>(arena + o) = (uint16_t)x;
                }
                if (FIRE) acc = min(max(acc + grad, acc_lo), acc_hi);
            }
        }
        __syncthreads();
    }

    // ---- parser: final checks and raw tail rows (a stream's last segment) ------
    if (parser) {
        for (uint32_t s = 0; s < SPW; ++s) {
            PcSeg &sg = SEG[s];
            const uint32_t tb = sg.tail * D * WB;
            if (sg.ok && (sg.r != sg.nrec || sg.rle_rem != 0 || sg.cursor + tb > sg.ext)) {
                if (lane == 0) sg.bad = 1;
            } else if (sg.ok) {
                uint8_t *const tp = sg.dst + (size_t)sg.nrow * D * WB;
                for (uint32_t q = lane; q < tb; q += 64) gst8(tp + q, gld8(sg.src + sg.cursor + q));
            }
        }
        wave_sync();
        if (lane < SPW && SEG[lane].bad && status) atomicOr(status + SEG[lane].status, 1);
    }
}

// One container: workgroup b decodes segments [b * SPW, b * SPW + SPW).
template <int W, bool FIRE, int D, int NP, int NC>
__global__ __launch_bounds__(pc_single_threads(D, NP, NC)) void k_decode_pc(const uint8_t *__restrict__ src, Geom g,
                                                            typename Elem<W>::T *__restrict__ dst,
                                                            int32_t *__restrict__ status) {
    using G = PcGeom<W, D, kPcChunkBlocks, NP, NC>;
    const uint32_t seg0 = blockIdx.x * G::SPW;
    auto init = [&](PcSeg &sg, uint32_t s) {
        pc_seg_init(sg, src, g.data_start, g.data_bytes, g.nseg, g.rows, g.S, seg0 + s, D, G::HB, G::WB,
                    reinterpret_cast<uint8_t *>(dst));
        if (seg0 + s >= g.nseg) sg.bad = 0;   // past the last segment: nothing to do
        sg.sh = g.sh; sg.acc_lo = g.acc_lo; sg.acc_hi = g.acc_hi; sg.status = 0;
    };
    const uint32_t nchunks = ((g.S >> 3) + kPcChunkBlocks - 1) / kPcChunkBlocks;
    if constexpr (pc_pipe(D)) pc_decode_group_pipe<W, FIRE, D, NP, NC>(nchunks, init, status);
    else pc_decode_group<W, FIRE, D, NP, NC>(nchunks, init, status);
}

// Many containers: a persistent grid pulls groups of SPW work-list entries
// (stream << 32 | segment, ~0 = empty) from a device queue; the segments of a
// group share one seg_rows (group_s). Status bits go to status[stream].
template <int W, bool FIRE, int D, int NP, int NC>
__global__ __launch_bounds__(pc_threads(NP, NC)) void k_decode_pc_batch(const PcStream *__restrict__ streams,
                                                                  const uint64_t *__restrict__ entries,
                                                                  const uint32_t *__restrict__ group_s, uint32_t ngroups,
                                                                  uint32_t *__restrict__ queue,
                                                                  int32_t *__restrict__ status) {
    using G = PcGeom<W, D, kPcChunkBlocks, NP, NC>;
    __shared__ uint32_t grp_sh;
    for (;;) {
        if (threadIdx.x == 0) grp_sh = atomicAdd(queue, 1u);
        __syncthreads();
        const uint32_t grp = grp_sh;
        __syncthreads();
        if (grp >= ngroups) break;
        auto init = [&](PcSeg &sg, uint32_t s) {
            const uint64_t e = entries[(uint64_t)grp * G::SPW + s];
            const uint32_t si = (uint32_t)(e >> 32);
            if (e == ~0ull) {
                sg.ok = 0; sg.bad = 0; sg.nrow = 0; sg.tail = 0; sg.ext = 0; sg.nrec = 0;
                sg.r = 0; sg.cursor = 4; sg.rle_rem = 0; sg.hbase = 0; sg.pbase = 0; sg.status = 0;
                sg.src = nullptr; sg.dst = nullptr; sg.sh = 0; sg.acc_lo = 0; sg.acc_hi = 0;
                return;
            }
            const PcStream st = streams[si];
            pc_seg_init(sg, st.src, st.data_start, st.data_bytes, st.nseg, st.rows, st.S, (uint32_t)e, D, G::HB,
                        G::WB, st.dst);
            sg.sh = st.sh; sg.acc_lo = st.acc_lo; sg.acc_hi = st.acc_hi; sg.status = si;
        };
        const uint32_t nchunks = ((group_s[grp] >> 3) + kPcChunkBlocks - 1) / kPcChunkBlocks;
        pc_decode_group<W, FIRE, D, NP, NC>(nchunks, init, status);
        __syncthreads();
    }
}

__global__ void k_zero_u32(uint32_t *p, uint32_t n) {
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

}  // namespace spz

/*
 * Sprintz CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * This file is the plain, slow reference implementation against which the
 * HIP codec is checked. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load it. It shares no code, header, table or
 * constant with the GPU library, and the GPU library never calls it.
 *
 * It follows Blalock, Madden & Guttag, "Sprintz: Time Series Compression for
 * the Internet of Things" (IMWUT 2(3), 2018):
 *   - Algorithm 1 (encodeBlock) and Algorithm 2 (decodeBlock), Section 4.1;
 *   - delta coding (Section 4.2.1) and the FIRE forecaster, Algorithm 3 with
 *     the three practical changes listed at the end of Section 4.2.2;
 *   - zigzag coding, bit widths, headers and the column-/row-major payload
 *     layouts of Section 4.3 (Bit Packing);
 *   - run-length coding of all-zero blocks (Section 4.1, Algorithm 1/2).
 * Everything is exact integer arithmetic. Bits are handled one at a time.
 *
 * Where the paper leaves a detail open, the reading taken is stated where it
 * is used and marked "reading Rn" (R1-R19), so that the GPU library can take
 * the same one.
 *
 * Byte format (this implementation's own; the paper's layout figure is not
 * available): little-endian fields, LSB-first bit strings, zero padding.
 *   container = 64-byte header | (nseg+1) x u64 segment offsets | pad to 16 |
 *               segments
 *   segment   = u32 nrec | groups of records | raw tail rows | pad to 16
 *   group     = headers of its records (hb bits per column, padded to a byte)
 *               followed by the payloads of its records
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOSPC (-2)
#define OR_ECORRUPT (-3)
#define OR_ENOMEM (-6)

/* ------------------------------------------------------------------------ */
/* Exact integer helpers                                                     */
/* ------------------------------------------------------------------------ */

/* floor(v / 2^s), written as a true floor division (reading R7). */
static int64_t floor_div_pow2(int64_t v, int s) {
    int64_t d = (int64_t)1 << s;
    int64_t q = v / d; /* C division truncates toward zero */
    if ((v % d) != 0 && v < 0) q -= 1;
    return q;
}

/* v mod 2^w in [0, 2^w). */
static int64_t mod_pow2(int64_t v, int w) {
    int64_t m = (int64_t)1 << w;
    int64_t r = v % m;
    if (r < 0) r += m;
    return r;
}

/* Reinterpret the low w bits of v as a w-bit two's complement number
 * (reading R1: all sample arithmetic is modulo 2^w). */
static int64_t sext_w(int64_t v, int w) {
    int64_t r = mod_pow2(v, w);
    if (r >= ((int64_t)1 << (w - 1))) r -= ((int64_t)1 << w);
    return r;
}

static int64_t sign_of(int64_t v) { return (v > 0) - (v < 0); } /* sgn(0)=0, reading R5 */

/* Zigzag code of a signed w-bit value (Section 4.3): 2e for e >= 0 and
 * -2e-1 for e < 0. */
static uint32_t zigzag(int64_t e) { return (uint32_t)(e >= 0 ? 2 * e : -2 * e - 1); }

/* Inverse of zigzag. */
static int64_t unzigzag(uint32_t z) {
    return (z % 2 == 0) ? (int64_t)(z / 2) : -(int64_t)(z / 2) - 1;
}

/* Number of bits needed to write z, i.e. the smallest k with z < 2^k. */
static int required_num_bits(uint32_t z) {
    int k = 0;
    while (k < 32 && (z >> k) != 0) k++;
    return k;
}

/* Section 4.3: a header field has log2(w) bits, so width w-1 is stored as
 * code w-1 and means width w (reading R11). */
static int header_bits(int w) { return w == 8 ? 3 : 4; }
static int code_of_nbits(int nbits, int w) { return nbits < w - 1 ? nbits : w - 1; }
static int width_of_code(int code, int w) { return code < w - 1 ? code : w; }

/* ------------------------------------------------------------------------ */
/* Bit I/O, one bit at a time, LSB first (reading R12)                       */
/* ------------------------------------------------------------------------ */

typedef struct { uint8_t *buf; size_t cap; size_t bitpos; int overflow; } bit_writer;

static void bw_put(bit_writer *bw, uint64_t v, int nbits) {
    for (int k = 0; k < nbits; k++) {
        size_t byte = bw->bitpos / 8;
        int bit = (int)(bw->bitpos % 8);
        if (byte >= bw->cap) { bw->overflow = 1; return; }
        if ((v >> k) & 1u) bw->buf[byte] |= (uint8_t)(1u << bit);
        else bw->buf[byte] &= (uint8_t)~(1u << bit);
        bw->bitpos++;
    }
}

static void bw_align_byte(bit_writer *bw) {
    while (bw->bitpos % 8 != 0) bw_put(bw, 0, 1);
}

typedef struct { const uint8_t *buf; size_t len; size_t bitpos; int overrun; } bit_reader;

static uint64_t br_get(bit_reader *br, int nbits) {
    uint64_t v = 0;
    for (int k = 0; k < nbits; k++) {
        size_t byte = br->bitpos / 8;
        int bit = (int)(br->bitpos % 8);
        if (byte >= br->len) { br->overrun = 1; return 0; }
        if ((br->buf[byte] >> bit) & 1u) v |= (uint64_t)1 << k;
        br->bitpos++;
    }
    return v;
}

static void br_align_byte(bit_reader *br) {
    while (br->bitpos % 8 != 0) br->bitpos++;
}

static void put_le(uint8_t *p, uint64_t v, int nbytes) {
    for (int k = 0; k < nbytes; k++) p[k] = (uint8_t)(v >> (8 * k));
}

static uint64_t get_le(const uint8_t *p, int nbytes) {
    uint64_t v = 0;
    for (int k = 0; k < nbytes; k++) v |= (uint64_t)p[k] << (8 * k);
    return v;
}

/* ------------------------------------------------------------------------ */
/* Forecasters (Section 4.2)                                                 */
/* ------------------------------------------------------------------------ */

/* Per-column state. prev is x_{i-1} (unsigned w-bit pattern); delta is the
 * signed w-bit difference of the two most recent samples; acc is FIRE's
 * accumulator (Algorithm 3, Init). alpha and grad hold the per-block values
 * of the practical variant (end of Section 4.2.2). */
typedef struct {
    int D, w, fire, learn_shift;
    int64_t *prev, *delta, *acc, *alpha, *grad;
    int fixed_alpha_on; /* test hook: hold alpha at fixed_alpha (no training) */
    int64_t fixed_alpha;
} forecaster;

/* alpha = acc >> (learnShift + 2): the learning rate eta = 1/2 gives a shift
 * of 1 (reading R3) and averaging the four gradients of a block adds 2
 * (reading R4). */
static int fire_shift(const forecaster *f) { return f->learn_shift + 2; }

/* Accumulator range, so that alpha/2^w stays in [-1/2, 1] (Section 4.2.2,
 * equation for x_i in terms of alpha; reading R6). */
static int64_t acc_lo(const forecaster *f) { return -(((int64_t)1 << (f->w - 1)) << fire_shift(f)); }
static int64_t acc_hi(const forecaster *f) { return ((int64_t)1 << f->w) << fire_shift(f); }

static int fc_init(forecaster *f, int D, int w, int fire, int learn_shift) {
    memset(f, 0, sizeof(*f));
    f->D = D; f->w = w; f->fire = fire; f->learn_shift = learn_shift;
    f->prev = calloc((size_t)D, sizeof(int64_t));
    f->delta = calloc((size_t)D, sizeof(int64_t));
    f->acc = calloc((size_t)D, sizeof(int64_t));
    f->alpha = calloc((size_t)D, sizeof(int64_t));
    f->grad = calloc((size_t)D, sizeof(int64_t));
    if (!f->prev || !f->delta || !f->acc || !f->alpha || !f->grad) return OR_ENOMEM;
    return OR_OK; /* all state starts at zero: x_0 = 0 (Section 4.2.1), reading R2 */
}

static void fc_free(forecaster *f) {
    free(f->prev); free(f->delta); free(f->acc); free(f->alpha); free(f->grad);
}

/* Practical FIRE: the coefficient is computed once at the start of a block. */
static void fc_block_begin(forecaster *f) {
    for (int j = 0; j < f->D; j++) {
        if (f->fixed_alpha_on) f->alpha[j] = f->fixed_alpha;
        else f->alpha[j] = f->fire ? floor_div_pow2(f->acc[j], fire_shift(f)) : 0;
        f->grad[j] = 0;
    }
}

/* predict(x_{i-1}) for column j. Delta: x_{i-1}. FIRE (Algorithm 3, Predict):
 * x_{i-1} + floor(alpha * delta / 2^w), the product taken exactly. */
static int64_t fc_predict(const forecaster *f, int j) {
    if (!f->fire) return f->prev[j];
    return f->prev[j] + floor_div_pow2(f->alpha[j] * f->delta[j], f->w);
}

/* train(x_{i-1}, x_i, err_i) for column j at row i of the block (0-based).
 * FIRE (Algorithm 3, Train): the gradient is -sign(err) * delta; the
 * accumulator moves against it. Practical variant: gradients only on every
 * other sample (odd rows, reading R4) and summed into one update per block.
 * The delta is refreshed afterwards, so the gradient uses the old delta. */
static void fc_train(forecaster *f, int j, int i, int64_t x, int64_t err) {
    if (f->fire && (i % 2 == 1)) {
        int64_t gradient = -sign_of(err) * f->delta[j];
        f->grad[j] -= gradient;
    }
    f->delta[j] = sext_w(x - f->prev[j], f->w);
    f->prev[j] = x;
}

/* End of block: one accumulator update with the summed gradient, saturated
 * to the accumulator range (reading R6). */
static void fc_block_end(forecaster *f) {
    if (!f->fire || f->fixed_alpha_on) return;
    for (int j = 0; j < f->D; j++) {
        int64_t a = f->acc[j] + f->grad[j];
        if (a < acc_lo(f)) a = acc_lo(f);
        if (a > acc_hi(f)) a = acc_hi(f);
        f->acc[j] = a;
    }
}

/* ------------------------------------------------------------------------ */
/* Records of one segment                                                    */
/* ------------------------------------------------------------------------ */

#define RLE_MAX 65535u /* run counts are u16 (reading R14) */

typedef struct {
    int is_rle;
    uint32_t count;      /* RLE: number of all-zero blocks */
    uint8_t *codes;      /* D header codes (all zero for RLE) */
    uint8_t *payload;    /* payload bytes */
    size_t payload_len;
} record;

typedef struct { record *r; size_t n, cap; } record_list;

static int rl_push(record_list *rl, record rec) {
    if (rl->n == rl->cap) {
        size_t nc = rl->cap ? rl->cap * 2 : 64;
        record *nr = realloc(rl->r, nc * sizeof(record));
        if (!nr) return OR_ENOMEM;
        rl->r = nr; rl->cap = nc;
    }
    rl->r[rl->n++] = rec;
    return OR_OK;
}

static void rl_free(record_list *rl) {
    for (size_t k = 0; k < rl->n; k++) { free(rl->r[k].codes); free(rl->r[k].payload); }
    free(rl->r);
}

static int emit_rle(record_list *rl, int D, uint32_t count) {
    record rec; memset(&rec, 0, sizeof(rec));
    rec.is_rle = 1; rec.count = count;
    rec.codes = calloc((size_t)D, 1);
    rec.payload = calloc(2, 1);
    if (!rec.codes || !rec.payload) return OR_ENOMEM;
    put_le(rec.payload, count, 2); /* number of all-zero blocks as payload */
    rec.payload_len = 2;
    return rl_push(rl, rec);
}

/* Column-major iff a sample is at most 32 bits wide (Section 4.3; reading R13). */
static int is_column_major(int D, int w) { return (int64_t)D * w <= 32; }

/* Bit-pack one block's zigzag values z[i*D + j] with the given widths. */
static int pack_block(const uint32_t *z, const int *width, int D, int w, uint8_t **out, size_t *out_len) {
    size_t bits = 0;
    for (int j = 0; j < D; j++) bits += (size_t)width[j];
    size_t len;
    if (is_column_major(D, w)) len = bits;             /* 8 values x width_j bits = width_j bytes per column */
    else len = 8 * ((bits + 7) / 8);                   /* 8 rows, each padded to a byte */
    uint8_t *buf = calloc(len ? len : 1, 1);
    if (!buf) return OR_ENOMEM;
    bit_writer bw = {buf, len, 0, 0};
    if (is_column_major(D, w)) {
        for (int j = 0; j < D; j++)
            for (int i = 0; i < 8; i++) bw_put(&bw, z[i * D + j], width[j]);
    } else {
        for (int i = 0; i < 8; i++) {
            for (int j = 0; j < D; j++) bw_put(&bw, z[i * D + j], width[j]);
            bw_align_byte(&bw);
        }
    }
    if (bw.overflow || bw.bitpos != 8 * len) { free(buf); return OR_EINVAL; }
    *out = buf; *out_len = len;
    return OR_OK;
}

/* Encode the full 8-row blocks of one segment into a record list
 * (Algorithm 1 applied block after block). x holds rows x D unsigned w-bit
 * values. Also reports the per-block residuals and coefficients when asked
 * (test hook). */
static int encode_records(const uint32_t *x, uint64_t nblk, int D, int w, forecaster *f,
                          record_list *rl, int64_t *resid_out, int64_t *alpha_out) {
    uint32_t *z = malloc((size_t)8 * D * sizeof(uint32_t));
    int *nbits = malloc((size_t)D * sizeof(int));
    int *width = malloc((size_t)D * sizeof(int));
    if (!z || !nbits || !width) { free(z); free(nbits); free(width); return OR_ENOMEM; }
    int rc = OR_OK;
    uint32_t run = 0; /* all-zero blocks seen since the last emitted record */
    for (uint64_t b = 0; b < nblk && rc == OR_OK; b++) {
        const uint32_t *blk = x + (size_t)b * 8 * D;
        fc_block_begin(f);
        if (alpha_out)
            for (int j = 0; j < D; j++) alpha_out[(size_t)b * D + j] = f->alpha[j];
        /* predict, error, train for each sample */
        for (int i = 0; i < 8; i++) {
            for (int j = 0; j < D; j++) {
                int64_t xi = blk[i * D + j];
                int64_t xhat = fc_predict(f, j);
                int64_t err = sext_w(xi - xhat, w); /* reading R1 */
                fc_train(f, j, i, xi, err);
                z[i * D + j] = zigzag(err);
                if (resid_out) resid_out[((size_t)b * 8 + i) * D + j] = err;
            }
        }
        fc_block_end(f);
        /* bits required per column: max over the block's rows */
        int all_zero = 1;
        for (int j = 0; j < D; j++) {
            int m = 0;
            for (int i = 0; i < 8; i++) {
                int k = required_num_bits(z[i * D + j]);
                if (k > m) m = k;
            }
            nbits[j] = m;
            width[j] = width_of_code(code_of_nbits(m, w), w);
            if (m != 0) all_zero = 0;
        }
        if (all_zero) {
            /* Algorithm 1: keep reading blocks until one is nonzero; the run
             * is written as D zero headers plus the count (split at the u16
             * limit, reading R14). */
            run++;
            if (run == RLE_MAX) { rc = emit_rle(rl, D, run); run = 0; }
            continue;
        }
        if (run > 0) { rc = emit_rle(rl, D, run); run = 0; if (rc) break; }
        record rec; memset(&rec, 0, sizeof(rec));
        rec.codes = malloc((size_t)D);
        if (!rec.codes) { rc = OR_ENOMEM; break; }
        for (int j = 0; j < D; j++) rec.codes[j] = (uint8_t)code_of_nbits(nbits[j], w);
        rc = pack_block(z, width, D, w, &rec.payload, &rec.payload_len);
        if (rc) { free(rec.codes); break; }
        rc = rl_push(rl, rec);
    }
    /* a run still open at the end of the segment is flushed (reading R14) */
    if (rc == OR_OK && run > 0) rc = emit_rle(rl, D, run);
    free(z); free(nbits); free(width);
    return rc;
}

/* Serialize a record list: u32 nrec, then groups of G records (G = 0 means
 * a single group), each = packed headers padded to a byte, then payloads
 * (Section 4.3, header grouping; reading R15). */
static size_t serialized_records_size(const record_list *rl, int D, int w, int G) {
    int hb = header_bits(w);
    size_t total = 4;
    size_t g = (G == 0) ? (rl->n ? rl->n : 1) : (size_t)G;
    for (size_t start = 0; start < rl->n; start += g) {
        size_t cnt = rl->n - start < g ? rl->n - start : g;
        total += (cnt * (size_t)D * (size_t)hb + 7) / 8;
        for (size_t k = start; k < start + cnt; k++) total += rl->r[k].payload_len;
    }
    return total;
}

static int serialize_records(const record_list *rl, int D, int w, int G, uint8_t *out, size_t cap) {
    int hb = header_bits(w);
    if (cap < 4) return OR_ENOSPC;
    put_le(out, (uint64_t)rl->n, 4);
    size_t pos = 4;
    size_t g = (G == 0) ? (rl->n ? rl->n : 1) : (size_t)G;
    for (size_t start = 0; start < rl->n; start += g) {
        size_t cnt = rl->n - start < g ? rl->n - start : g;
        size_t hbytes = (cnt * (size_t)D * (size_t)hb + 7) / 8;
        if (pos + hbytes > cap) return OR_ENOSPC;
        bit_writer bw = {out + pos, hbytes, 0, 0};
        memset(out + pos, 0, hbytes);
        for (size_t k = start; k < start + cnt; k++)
            for (int j = 0; j < D; j++) bw_put(&bw, rl->r[k].codes[j], hb);
        bw_align_byte(&bw);
        if (bw.overflow) return OR_ENOSPC;
        pos += hbytes;
        for (size_t k = start; k < start + cnt; k++) {
            if (pos + rl->r[k].payload_len > cap) return OR_ENOSPC;
            memcpy(out + pos, rl->r[k].payload, rl->r[k].payload_len);
            pos += rl->r[k].payload_len;
        }
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Container                                                                 */
/* ------------------------------------------------------------------------ */

#define HDR_BYTES 64
static size_t align16(size_t v) { return (v + 15) & ~(size_t)15; }

static int dtype_bits(int dtype) {
    switch (dtype) { case 1: case 2: return 8; case 3: case 4: return 16; default: return 0; }
}

static uint64_t num_segments(uint64_t rows, uint32_t S) { return rows == 0 ? 0 : (rows + S - 1) / S; }

static int check_params(uint32_t D, int dtype, int forecaster_id, uint32_t S, int G, int learn_shift) {
    if (D == 0 || D > 65535) return OR_EINVAL;
    if (dtype_bits(dtype) == 0) return OR_EINVAL;
    if (forecaster_id != 0 && forecaster_id != 1) return OR_EINVAL;
    if (S < 8 || S % 8 != 0) return OR_EINVAL;
    if (G < 0 || G > 255) return OR_EINVAL;
    if (learn_shift < 0 || learn_shift > 8) return OR_EINVAL;
    return OR_OK;
}

/* Upper bound of the container size: every block at full width, plus the
 * header bits, the per-group padding byte, the tail and the 16-byte pad. */
size_t oracle_compress_bound(uint64_t rows, uint32_t D, int dtype, uint32_t S, int G) {
    int w = dtype_bits(dtype);
    if (w == 0 || S < 8) return 0;
    int hb = header_bits(w);
    uint64_t nseg = num_segments(rows, S);
    size_t total = align16(HDR_BYTES + 8 * (size_t)(nseg + 1));
    for (uint64_t s = 0; s < nseg; s++) {
        uint64_t r = (s + 1 < nseg) ? S : rows - (uint64_t)S * s;
        uint64_t nblk = r / 8, tail = r % 8;
        uint64_t ngroups = (G == 0) ? 1 : (nblk + (uint64_t)G - 1) / (uint64_t)G;
        total += 4 + (size_t)((nblk * D * hb + 7) / 8) + (size_t)ngroups + (size_t)(nblk * D * w) +
                 (size_t)(tail * D * (w / 8)) + 15;
    }
    return total;
}

/* Load rows x D little-endian w-bit values as unsigned patterns. */
static void load_values(const uint8_t *src, uint64_t n, int w, uint32_t *x) {
    for (uint64_t k = 0; k < n; k++) x[k] = (uint32_t)get_le(src + k * (w / 8), w / 8);
}

/* Compress one segment of nrows rows (the tail rows, if any, are stored raw,
 * reading R16). Writes into out (zero padded to a multiple of 16) and
 * returns its length, or 0 on error (rc set). */
static size_t compress_segment(const uint32_t *x, uint64_t nrows, int D, int w, int fire, int learn_shift,
                               int G, uint8_t *out, size_t cap, int *rc,
                               int64_t *resid_out, int64_t *alpha_out, int fixed_alpha_on, int64_t fixed_alpha) {
    forecaster f;
    *rc = fc_init(&f, D, w, fire, learn_shift);
    if (*rc) { fc_free(&f); return 0; }
    f.fixed_alpha_on = fixed_alpha_on; f.fixed_alpha = fixed_alpha;
    record_list rl = {0, 0, 0};
    uint64_t nblk = nrows / 8, tail = nrows % 8;
    *rc = encode_records(x, nblk, D, w, &f, &rl, resid_out, alpha_out);
    size_t len = 0;
    if (*rc == OR_OK) {
        size_t body = serialized_records_size(&rl, D, w, G);
        size_t tail_bytes = (size_t)(tail * D * (w / 8));
        len = align16(body + tail_bytes);
        if (len > cap) *rc = OR_ENOSPC;
        else {
            memset(out, 0, len);
            *rc = serialize_records(&rl, D, w, G, out, body);
            for (uint64_t k = 0; k < tail * D && *rc == OR_OK; k++)
                put_le(out + body + k * (w / 8), x[nblk * 8 * D + k], w / 8);
        }
    }
    rl_free(&rl); fc_free(&f);
    return *rc == OR_OK ? len : 0;
}

int oracle_compress(const void *src, uint64_t rows, uint32_t D, int dtype, int forecaster_id,
                    uint32_t S, int G, int learn_shift, void *dst, size_t cap, size_t *out_size) {
    int rc = check_params(D, dtype, forecaster_id, S, G, learn_shift);
    if (rc) return rc;
    int w = dtype_bits(dtype);
    uint64_t nseg = num_segments(rows, S);
    size_t data_start = align16(HDR_BYTES + 8 * (size_t)(nseg + 1));
    if (cap < data_start) return OR_ENOSPC;
    uint8_t *out = dst;
    memset(out, 0, data_start);
    uint32_t *x = malloc((size_t)((rows * D) != 0 ? rows * D : 1) * sizeof(uint32_t));
    if (!x) return OR_ENOMEM;
    load_values(src, rows * D, w, x);
    size_t pos = data_start;
    for (uint64_t s = 0; s < nseg; s++) {
        uint64_t r = (s + 1 < nseg) ? S : rows - (uint64_t)S * s;
        put_le(out + HDR_BYTES + 8 * s, pos - data_start, 8);
        size_t len = compress_segment(x + (size_t)s * S * D, r, (int)D, w, forecaster_id, learn_shift, G,
                                      out + pos, cap - pos, &rc, NULL, NULL, 0, 0);
        if (rc) { free(x); return rc; }
        pos += len;
    }
    put_le(out + HDR_BYTES + 8 * nseg, pos - data_start, 8);
    free(x);
    memcpy(out, "SPZ1", 4);
    put_le(out + 4, 1, 2);
    out[6] = (uint8_t)w; out[7] = (uint8_t)dtype; out[8] = (uint8_t)forecaster_id;
    out[9] = (uint8_t)learn_shift; out[10] = (uint8_t)G; out[11] = 0;
    put_le(out + 12, D, 4); put_le(out + 16, rows, 8);
    put_le(out + 24, S, 4); put_le(out + 28, nseg, 4);
    put_le(out + 32, pos - data_start, 8);
    *out_size = pos;
    return OR_OK;
}

/* Decode one segment (Algorithm 2 for each record). */
static int decompress_segment(const uint8_t *seg, size_t seg_len, uint64_t nrows, int D, int w, int fire,
                              int learn_shift, int G, uint32_t *x) {
    forecaster f;
    int rc = fc_init(&f, D, w, fire, learn_shift);
    if (rc) { fc_free(&f); return rc; }
    int hb = header_bits(w);
    int colmajor = is_column_major(D, w);
    uint64_t nblk = nrows / 8, tail = nrows % 8;
    int *width = malloc((size_t)D * sizeof(int));
    uint8_t *codes = malloc((size_t)D);
    if (!width || !codes) { free(width); free(codes); fc_free(&f); return OR_ENOMEM; }
    if (seg_len < 4) { rc = OR_ECORRUPT; goto done; }
    uint64_t nrec = get_le(seg, 4);
    size_t pos = 4;
    uint64_t blk = 0;                          /* blocks decoded so far */
    uint64_t g = (G == 0) ? (nrec ? nrec : 1) : (uint64_t)G;
    for (uint64_t start = 0; start < nrec && rc == OR_OK; start += g) {
        uint64_t cnt = nrec - start < g ? nrec - start : g;
        size_t hbytes = (size_t)((cnt * (uint64_t)D * (uint64_t)hb + 7) / 8);
        if (pos + hbytes > seg_len) { rc = OR_ECORRUPT; break; }
        bit_reader hr = {seg + pos, hbytes, 0, 0};
        pos += hbytes;
        for (uint64_t k = 0; k < cnt && rc == OR_OK; k++) {
            /* the header is always first and of fixed size (Section 4.1) */
            int all_zero = 1;
            size_t bits = 0;
            for (int j = 0; j < D; j++) {
                codes[j] = (uint8_t)br_get(&hr, hb);
                width[j] = width_of_code(codes[j], w);
                bits += (size_t)width[j];
                if (codes[j] != 0) all_zero = 0;
            }
            if (all_zero) {
                /* run of zero errors: predict only (Algorithm 2), with the
                 * forecaster state kept in step with the encoder (reading R9) */
                if (pos + 2 > seg_len) { rc = OR_ECORRUPT; break; }
                uint64_t numblocks = get_le(seg + pos, 2);
                pos += 2;
                if (numblocks == 0 || blk + numblocks > nblk) { rc = OR_ECORRUPT; break; }
                for (uint64_t b = 0; b < numblocks; b++, blk++) {
                    fc_block_begin(&f);
                    for (int i = 0; i < 8; i++)
                        for (int j = 0; j < D; j++) {
                            int64_t xi = mod_pow2(fc_predict(&f, j), w);
                            fc_train(&f, j, i, xi, 0);
                            x[(blk * 8 + i) * D + j] = (uint32_t)xi;
                        }
                    fc_block_end(&f);
                }
                continue;
            }
            if (blk + 1 > nblk) { rc = OR_ECORRUPT; break; }
            size_t len = colmajor ? bits : 8 * ((bits + 7) / 8);
            if (pos + len > seg_len) { rc = OR_ECORRUPT; break; }
            /* unpack into z[i*D+j] */
            uint32_t *z = malloc((size_t)8 * D * sizeof(uint32_t));
            if (!z) { rc = OR_ENOMEM; break; }
            bit_reader pr = {seg + pos, len, 0, 0};
            if (colmajor) {
                for (int j = 0; j < D; j++)
                    for (int i = 0; i < 8; i++) z[i * D + j] = (uint32_t)br_get(&pr, width[j]);
            } else {
                for (int i = 0; i < 8; i++) {
                    for (int j = 0; j < D; j++) z[i * D + j] = (uint32_t)br_get(&pr, width[j]);
                    br_align_byte(&pr);
                }
            }
            pos += len;
            fc_block_begin(&f);
            for (int i = 0; i < 8; i++)
                for (int j = 0; j < D; j++) {
                    int64_t xhat = fc_predict(&f, j);
                    int64_t err = unzigzag(z[i * D + j]);
                    int64_t xi = mod_pow2(err + xhat, w);
                    fc_train(&f, j, i, xi, err);
                    x[(blk * 8 + i) * D + j] = (uint32_t)xi;
                }
            fc_block_end(&f);
            blk++;
            free(z);
        }
    }
    if (rc == OR_OK && blk != nblk) rc = OR_ECORRUPT;
    if (rc == OR_OK) {
        size_t tb = (size_t)(tail * D * (w / 8));
        if (pos + tb > seg_len) rc = OR_ECORRUPT;
        else
            for (uint64_t k = 0; k < tail * D; k++)
                x[nblk * 8 * D + k] = (uint32_t)get_le(seg + pos + k * (w / 8), w / 8);
    }
done:
    free(width); free(codes); fc_free(&f);
    return rc;
}

typedef struct {
    uint64_t rows, data_bytes;
    uint32_t D, S, nseg;
    int w, dtype, forecaster_id, learn_shift, G, entropy;
} container_info;

static int parse_header(const uint8_t *src, size_t n, container_info *ci) {
    if (n < HDR_BYTES || memcmp(src, "SPZ1", 4) != 0 || get_le(src + 4, 2) != 1) return OR_ECORRUPT;
    ci->w = src[6]; ci->dtype = src[7]; ci->forecaster_id = src[8];
    ci->learn_shift = src[9]; ci->G = src[10]; ci->entropy = src[11];
    ci->D = (uint32_t)get_le(src + 12, 4); ci->rows = get_le(src + 16, 8);
    ci->S = (uint32_t)get_le(src + 24, 4); ci->nseg = (uint32_t)get_le(src + 28, 4);
    ci->data_bytes = get_le(src + 32, 8);
    if (check_params(ci->D, ci->dtype, ci->forecaster_id, ci->S, ci->G, ci->learn_shift)) return OR_ECORRUPT;
    if (ci->w != dtype_bits(ci->dtype) || (ci->entropy != 0 && ci->entropy != 1)) return OR_ECORRUPT;
    if (num_segments(ci->rows, ci->S) != ci->nseg) return OR_ECORRUPT;
    return OR_OK;
}

int oracle_info(const void *src, size_t n, uint64_t *rows, uint32_t *D, int *dtype, uint64_t *total) {
    container_info ci;
    int rc = parse_header(src, n, &ci);
    if (rc) return rc;
    *rows = ci.rows; *D = ci.D; *dtype = ci.dtype;
    *total = align16(HDR_BYTES + 8 * (size_t)(ci.nseg + 1)) + ci.data_bytes;
    return OR_OK;
}

static int decompress_plain(const uint8_t *src, size_t n, void *dst, size_t cap);
size_t oracle_entropy_plain_size(const void *src_v, size_t n);
int oracle_entropy_decode(const void *src_v, size_t n, void *dst, size_t cap, size_t *out_size);

int oracle_decompress(const void *src_v, size_t n, void *dst, size_t cap) {
    const uint8_t *src = src_v;
    container_info ci;
    int rc = parse_header(src, n, &ci);
    if (rc) return rc;
    if (ci.entropy == 0) return decompress_plain(src, n, dst, cap);
    size_t pn = oracle_entropy_plain_size(src, n);
    if (pn == 0) return OR_ECORRUPT;
    uint8_t *plain = malloc(pn);
    if (!plain) return OR_ENOMEM;
    size_t got = 0;
    rc = oracle_entropy_decode(src, n, plain, pn, &got);
    if (rc == OR_OK) rc = decompress_plain(plain, got, dst, cap);
    free(plain);
    return rc;
}

static int decompress_plain(const uint8_t *src, size_t n, void *dst, size_t cap) {
    container_info ci;
    int rc = parse_header(src, n, &ci);
    if (rc) return rc;
    size_t data_start = align16(HDR_BYTES + 8 * (size_t)(ci.nseg + 1));
    if (data_start + ci.data_bytes > n) return OR_ECORRUPT;
    if (cap < ci.rows * ci.D * (uint64_t)(ci.w / 8)) return OR_ENOSPC;
    const uint8_t *data = src + data_start;
    uint32_t *x = malloc((size_t)((ci.rows * ci.D) != 0 ? ci.rows * ci.D : 1) * sizeof(uint32_t));
    if (!x) return OR_ENOMEM;
    if (get_le(src + HDR_BYTES, 8) != 0 || get_le(src + HDR_BYTES + 8 * (size_t)ci.nseg, 8) != ci.data_bytes) {
        free(x); return OR_ECORRUPT;
    }
    for (uint32_t s = 0; s < ci.nseg && rc == OR_OK; s++) {
        uint64_t a = get_le(src + HDR_BYTES + 8 * (size_t)s, 8);
        uint64_t b = get_le(src + HDR_BYTES + 8 * (size_t)(s + 1), 8);
        if (a > b || b > ci.data_bytes || a % 16 || b % 16) { rc = OR_ECORRUPT; break; }
        uint64_t r = (s + 1 < ci.nseg) ? ci.S : ci.rows - (uint64_t)ci.S * s;
        rc = decompress_segment(data + a, (size_t)(b - a), r, (int)ci.D, ci.w, ci.forecaster_id,
                                ci.learn_shift, ci.G, x + (size_t)s * ci.S * ci.D);
    }
    if (rc == OR_OK) {
        uint8_t *out = dst;
        for (uint64_t k = 0; k < ci.rows * ci.D; k++) put_le(out + k * (ci.w / 8), x[k], ci.w / 8);
    }
    free(x);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Entropy stage: Huffman coding of each segment's packed bytes              */
/* ------------------------------------------------------------------------ */
/*
 * Section 4.4 ends with an entropy stage: the bit-packed bytes are Huffman
 * coded with an off-the-shelf byte-oriented coder, bytes taken as symbols
 * regardless of the data's bit width. The coder and its format are not part
 * of the paper; this implementation uses its own (reading R19):
 *   - one code per segment, built from the byte counts of the whole plain
 *     segment (the segment exactly as the plain container holds it);
 *   - code lengths by the two-queue Huffman construction over the present
 *     byte values sorted by (count, value), a leaf taken before an internal
 *     node of equal weight; lengths above 11 bits are removed by halving the
 *     counts (c -> (c + 1) / 2, so present values stay present) and building
 *     again; a single present value gets length 1;
 *   - canonical codes: values sorted by (length, value), consecutive code
 *     values, one shift left per extra bit of length;
 *   - 16 sub-streams, sub-stream k coding plain bytes [k n/16, (k+1) n/16),
 *     each a byte-aligned LSB-first bit string in which every code is stored
 *     first bit (most significant) first.
 * Entropy-coded segment:
 *   u32 n | u8 len[128] (4 bits per byte value, even values in the low
 *   nibble) | u32 size[16] (bytes of each sub-stream) | sub-streams | pad to 16
 * The container header is the plain one with byte 11 = 1; its offset table
 * and data_bytes describe the entropy-coded segments.
 */
#define HUF_MAXLEN 11
#define HUF_NSUB 16
#define HUF_FIXED (4 + 128 + 4 * HUF_NSUB)

/* Code lengths of the 256 byte values from their counts (0 = absent). */
int oracle_huff_lengths(const uint64_t *count, uint8_t *len) {
    uint64_t f[256];
    int order[256], n = 0;
    for (int v = 0; v < 256; v++) { f[v] = count[v]; len[v] = 0; if (f[v]) n++; }
    if (n == 0) return OR_OK;
    if (n == 1) {
        for (int v = 0; v < 256; v++) if (f[v]) len[v] = 1;
        return OR_OK;
    }
    for (;;) {
        /* present values sorted by (count, value): insertion sort */
        int m = 0;
        for (int v = 0; v < 256; v++) {
            if (!f[v]) continue;
            int k = m++;
            while (k > 0 && (f[order[k - 1]] > f[v])) { order[k] = order[k - 1]; k--; }
            order[k] = v;
        }
        /* nodes 0..m-1 are the leaves in sorted order; internal nodes follow */
        uint64_t weight[511];
        int parent[511];
        for (int k = 0; k < m; k++) weight[k] = f[order[k]];
        int leaf = 0, inner = m, next = m;
        for (int step = 0; step < m - 1; step++) {
            int pick[2];
            for (int t = 0; t < 2; t++) {
                int use_leaf = leaf < m && (inner >= next || weight[leaf] <= weight[inner]);
                pick[t] = use_leaf ? leaf++ : inner++;
            }
            weight[next] = weight[pick[0]] + weight[pick[1]];
            parent[pick[0]] = next;
            parent[pick[1]] = next;
            next++;
        }
        int maxlen = 0;
        for (int k = 0; k < m; k++) {
            int d = 0;
            for (int q = k; q != next - 1; q = parent[q]) d++;
            len[order[k]] = (uint8_t)d;
            if (d > maxlen) maxlen = d;
        }
        if (maxlen <= HUF_MAXLEN) return OR_OK;
        for (int v = 0; v < 256; v++) if (f[v]) f[v] = (f[v] + 1) / 2;
    }
}

/* Canonical code values from the lengths. */
static void huff_codes(const uint8_t *len, uint32_t *code) {
    uint32_t c = 0;
    int prev = -1;
    for (int l = 1; l <= HUF_MAXLEN; l++)
        for (int v = 0; v < 256; v++) {
            if (len[v] != l) continue;
            if (prev >= 0) c = (c + 1) << (l - prev);
            code[v] = c;
            prev = l;
        }
}

static size_t huff_segment_bound(size_t n) { return align16(HUF_FIXED + (n * HUF_MAXLEN + 7) / 8 + HUF_NSUB); }

/* Entropy-code one plain segment of n bytes; returns the coded size. */
static size_t huff_encode_segment(const uint8_t *p, size_t n, uint8_t *out) {
    uint64_t count[256] = {0};
    uint8_t len[256];
    uint32_t code[256] = {0};
    for (size_t i = 0; i < n; i++) count[p[i]]++;
    oracle_huff_lengths(count, len);
    huff_codes(len, code);
    put_le(out, n, 4);
    for (int v = 0; v < 256; v += 2) out[4 + v / 2] = (uint8_t)(len[v] | (len[v + 1] << 4));
    size_t pos = HUF_FIXED;
    for (int k = 0; k < HUF_NSUB; k++) {
        bit_writer bw = {out + pos, huff_segment_bound(n) - pos, 0, 0};
        for (size_t i = k * (n / HUF_NSUB); i < (k + 1) * (n / HUF_NSUB); i++) {
            int l = len[p[i]];
            for (int b = l - 1; b >= 0; b--) bw_put(&bw, (code[p[i]] >> b) & 1u, 1);
        }
        bw_align_byte(&bw);
        put_le(out + 4 + 128 + 4 * k, bw.bitpos / 8, 4);
        pos += bw.bitpos / 8;
    }
    size_t end = align16(pos);
    memset(out + pos, 0, end - pos);
    return end;
}

/* Decode one entropy-coded segment of m bytes into its plain bytes. */
static int huff_decode_segment(const uint8_t *s, size_t m, uint8_t *plain, size_t cap, size_t *n_out) {
    if (m < HUF_FIXED) return OR_ECORRUPT;
    size_t n = get_le(s, 4);
    if (n % 16 || n > cap) return OR_ECORRUPT;
    uint8_t len[256];
    for (int v = 0; v < 256; v += 2) { len[v] = s[4 + v / 2] & 15; len[v + 1] = s[4 + v / 2] >> 4; }
    /* canonical decoding tables: first code and first index of every length */
    int cnt[HUF_MAXLEN + 2] = {0}, sorted[256], ns = 0;
    for (int v = 0; v < 256; v++) {
        if (len[v] > HUF_MAXLEN) return OR_ECORRUPT;
        if (len[v]) cnt[len[v]]++;
    }
    uint32_t first[HUF_MAXLEN + 2];
    int index[HUF_MAXLEN + 2];
    uint32_t c = 0;
    for (int l = 1; l <= HUF_MAXLEN; l++) {
        first[l] = c; index[l] = ns;
        for (int v = 0; v < 256; v++) if (len[v] == l) sorted[ns++] = v;
        c = (c + (uint32_t)cnt[l]) << 1;
    }
    size_t pos = HUF_FIXED;
    for (int k = 0; k < HUF_NSUB; k++) {
        size_t sz = get_le(s + 4 + 128 + 4 * k, 4);
        if (pos + sz > m) return OR_ECORRUPT;
        bit_reader br = {s + pos, sz, 0, 0};
        for (size_t i = k * (n / HUF_NSUB); i < (k + 1) * (n / HUF_NSUB); i++) {
            uint32_t v = 0;
            int l = 0, found = -1;
            while (found < 0) {
                if (++l > HUF_MAXLEN || br.bitpos >= 8 * sz) return OR_ECORRUPT;
                v = (v << 1) | (uint32_t)br_get(&br, 1);
                if (cnt[l] && v >= first[l] && v - first[l] < (uint32_t)cnt[l]) found = sorted[index[l] + (int)(v - first[l])];
            }
            plain[i] = (uint8_t)found;
        }
        pos += sz;
    }
    *n_out = n;
    return OR_OK;
}

/* Test hooks: one segment (n a multiple of 16). */
size_t oracle_huff_encode_segment(const void *plain, size_t n, void *out, size_t cap) {
    if (n % 16 || cap < huff_segment_bound(n)) return 0;
    return huff_encode_segment(plain, n, out);
}
int oracle_huff_decode_segment(const void *seg, size_t m, void *plain, size_t cap, size_t *n_out) {
    return huff_decode_segment(seg, m, plain, cap, n_out);
}

size_t oracle_entropy_bound(const void *plain_v, size_t n) {
    const uint8_t *src = plain_v;
    container_info ci;
    if (parse_header(src, n, &ci) || ci.entropy != 0) return 0;
    size_t data_start = align16(HDR_BYTES + 8 * (size_t)(ci.nseg + 1));
    size_t total = data_start;
    for (uint32_t s = 0; s < ci.nseg; s++) {
        uint64_t a = get_le(src + HDR_BYTES + 8 * (size_t)s, 8), b = get_le(src + HDR_BYTES + 8 * (size_t)(s + 1), 8);
        total += huff_segment_bound((size_t)(b - a));
    }
    return total;
}

/* Plain container -> entropy-coded container. */
int oracle_entropy_encode(const void *plain_v, size_t n, void *dst, size_t cap, size_t *out_size) {
    const uint8_t *src = plain_v;
    uint8_t *out = dst;
    container_info ci;
    int rc = parse_header(src, n, &ci);
    if (rc) return rc;
    if (ci.entropy != 0) return OR_EINVAL;
    size_t data_start = align16(HDR_BYTES + 8 * (size_t)(ci.nseg + 1));
    if (data_start + ci.data_bytes > n) return OR_ECORRUPT;
    if (cap < oracle_entropy_bound(plain_v, n)) return OR_ENOSPC;
    memcpy(out, src, data_start);
    out[11] = 1;
    size_t pos = data_start;
    for (uint32_t s = 0; s < ci.nseg; s++) {
        uint64_t a = get_le(src + HDR_BYTES + 8 * (size_t)s, 8), b = get_le(src + HDR_BYTES + 8 * (size_t)(s + 1), 8);
        if (a > b || b > ci.data_bytes || a % 16 || b % 16) return OR_ECORRUPT;
        put_le(out + HDR_BYTES + 8 * (size_t)s, pos - data_start, 8);
        pos += huff_encode_segment(src + data_start + a, (size_t)(b - a), out + pos);
    }
    put_le(out + HDR_BYTES + 8 * (size_t)ci.nseg, pos - data_start, 8);
    put_le(out + 32, pos - data_start, 8);
    *out_size = pos;
    return OR_OK;
}

/* Entropy-coded container -> plain container (cap >= the plain size). */
int oracle_entropy_decode(const void *src_v, size_t n, void *dst, size_t cap, size_t *out_size) {
    const uint8_t *src = src_v;
    uint8_t *out = dst;
    container_info ci;
    int rc = parse_header(src, n, &ci);
    if (rc) return rc;
    if (ci.entropy != 1) return OR_EINVAL;
    size_t data_start = align16(HDR_BYTES + 8 * (size_t)(ci.nseg + 1));
    if (data_start + ci.data_bytes > n || cap < data_start) return OR_ECORRUPT;
    memcpy(out, src, data_start);
    out[11] = 0;
    size_t pos = data_start;
    for (uint32_t s = 0; s < ci.nseg; s++) {
        uint64_t a = get_le(src + HDR_BYTES + 8 * (size_t)s, 8), b = get_le(src + HDR_BYTES + 8 * (size_t)(s + 1), 8);
        if (a > b || b > ci.data_bytes || a % 16 || b % 16) return OR_ECORRUPT;
        put_le(out + HDR_BYTES + 8 * (size_t)s, pos - data_start, 8);
        size_t m = 0;
        rc = huff_decode_segment(src + data_start + a, (size_t)(b - a), out + pos, cap - pos, &m);
        if (rc) return rc;
        pos += m;
    }
    put_le(out + HDR_BYTES + 8 * (size_t)ci.nseg, pos - data_start, 8);
    put_le(out + 32, pos - data_start, 8);
    *out_size = pos;
    return OR_OK;
}

/* Plain size of an entropy-coded container (from its segments' n fields). */
size_t oracle_entropy_plain_size(const void *src_v, size_t n) {
    const uint8_t *src = src_v;
    container_info ci;
    if (parse_header(src, n, &ci) || ci.entropy != 1) return 0;
    size_t data_start = align16(HDR_BYTES + 8 * (size_t)(ci.nseg + 1));
    if (data_start + ci.data_bytes > n) return 0;
    size_t total = data_start;
    for (uint32_t s = 0; s < ci.nseg; s++) {
        uint64_t a = get_le(src + HDR_BYTES + 8 * (size_t)s, 8);
        if (a + 4 > ci.data_bytes) return 0;
        total += get_le(src + data_start + a, 4);
    }
    return total;
}

/* ------------------------------------------------------------------------ */
/* Test hooks                                                                */
/* ------------------------------------------------------------------------ */

/* Forecaster residuals of one segment of rows x D values (full blocks only):
 * resid[rows*D] (signed w-bit errors) and alpha[(rows/8)*D] (per-block
 * coefficient). With fixed_alpha_on, FIRE runs with alpha held constant. */
int oracle_residuals(const void *src, uint64_t rows, uint32_t D, int dtype, int forecaster_id, int learn_shift,
                     int fixed_alpha_on, int64_t fixed_alpha, int64_t *resid, int64_t *alpha) {
    int rc = check_params(D, dtype, forecaster_id, 8, 0, learn_shift);
    if (rc) return rc;
    int w = dtype_bits(dtype);
    uint64_t nblk = rows / 8;
    uint32_t *x = malloc((size_t)((rows * D) != 0 ? rows * D : 1) * sizeof(uint32_t));
    if (!x) return OR_ENOMEM;
    load_values(src, rows * D, w, x);
    forecaster f;
    rc = fc_init(&f, (int)D, w, forecaster_id, learn_shift);
    f.fixed_alpha_on = fixed_alpha_on; f.fixed_alpha = fixed_alpha;
    record_list rl = {0, 0, 0};
    if (rc == OR_OK) rc = encode_records(x, nblk, (int)D, w, &f, &rl, resid, alpha);
    rl_free(&rl); fc_free(&f); free(x);
    return rc;
}

/* Building blocks exposed for the exhaustive unit tests. */
uint32_t oracle_zigzag(int64_t e) { return zigzag(e); }
int64_t oracle_unzigzag(uint32_t z) { return unzigzag(z); }
int oracle_required_bits(uint32_t z) { return required_num_bits(z); }
int oracle_code_of_nbits(int nbits, int w) { return code_of_nbits(nbits, w); }
int oracle_width_of_code(int code, int w) { return width_of_code(code, w); }

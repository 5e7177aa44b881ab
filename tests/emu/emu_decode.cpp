// CPU harness: decodes a container with the decoder kernels' own source,
// every workgroup of the launch the library would make run by the
// coroutine scheduler of emu_sched.h, with bounds-checked global accesses
// (spz_device_ops.h of this directory) under AddressSanitizer.
//
//   emu_decode <container> <rows out> [batch]
// Prints "status=<device status word> violations=<out-of-bounds accesses>
// blocks=<workgroups>" and writes the decoded rows. The geometry follows the
// library's host code: the producer/consumer or pipelined decoder for
// whole-segment header groups with D <= 16 (16-byte aligned rows), the walker
// otherwise. With "batch", such containers go through the batched kernel
// instead (a one-stream batch: the producer/consumer form at every D).
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "spz_decode.h"
#include "spz_decode_pc.h"

static uint64_t le(const uint8_t *p, int n) {
    uint64_t v = 0;
    for (int k = 0; k < n; ++k) v |= (uint64_t)p[k] << (8 * k);
    return v;
}

template <int W, bool FIRE, int D>
static void run_pc(const uint8_t *src, const spz::Geom &g, uint8_t *dst, int32_t *status, uint32_t *blocks) {
    constexpr uint32_t NP = spz::kPcProducers, NC = spz::kPcConsumers;
    const uint32_t spw = spz::pc_spw(D, NP, NC);
    const uint32_t grid = (g.nseg + spw - 1) / spw;
    for (uint32_t b = 0; b < grid; ++b) {
        emu::dim3e bid, bdim;
        bid.x = b;
        bdim.x = spz::pc_single_threads(D, NP, NC);
        emu::run_block(bid, bdim, [&] {
            spz::k_decode_pc<W, FIRE, D, NP, NC>(src, g, reinterpret_cast<typename spz::Elem<W>::T *>(dst), status);
        });
    }
    *blocks = grid;
}

// The batched kernel on a batch of this one container: work-list groups of
// SPW segments (the last padded with empty entries), one persistent
// workgroup per eight groups.
template <int W, bool FIRE, int D>
static void run_pc_batch(const uint8_t *src, const spz::Geom &g, uint8_t *dst, int32_t *status, uint32_t *blocks) {
    constexpr uint32_t NP = spz::kPcProducers, NC = spz::kPcConsumers;
    const uint32_t spw = spz::pc_spw(D, NP, NC);
    const uint32_t ngroups = (g.nseg + spw - 1) / spw;
    spz::PcStream st;
    memset(&st, 0, sizeof st);
    st.src = src; st.dst = dst; st.data_start = g.data_start; st.data_bytes = g.data_bytes; st.rows = g.rows;
    st.nseg = g.nseg; st.S = g.S; st.sh = g.sh; st.acc_lo = g.acc_lo; st.acc_hi = g.acc_hi;
    std::vector<uint64_t> entries((size_t)ngroups * spw, ~0ull);
    for (uint32_t q = 0; q < g.nseg; ++q) entries[q] = q;   // stream 0
    std::vector<uint32_t> group_s(ngroups, g.S);
    uint32_t queue = 0;
    const uint32_t grid = (ngroups + 7) / 8;
    for (uint32_t b = 0; b < grid; ++b) {
        emu::dim3e bid, bdim;
        bid.x = b;
        bdim.x = spz::pc_threads(NP, NC);
        emu::run_block(bid, bdim, [&] {
            spz::k_decode_pc_batch<W, FIRE, D, NP, NC>(&st, entries.data(), group_s.data(), ngroups, &queue, status);
        });
    }
    *blocks = grid;
}

template <int W, bool FIRE, bool COL>
static void run_walker(const uint8_t *src, const spz::Geom &g, uint8_t *dst, int32_t *status, uint32_t *blocks) {
    const uint32_t lg = g.dp_log2 < 6 ? g.dp_log2 : 6u;
    const uint64_t lanes = (uint64_t)g.nseg << lg;
    const uint32_t grid = (uint32_t)((lanes + spz::kThreads - 1) / spz::kThreads);
    for (uint32_t b = 0; b < grid; ++b) {
        emu::dim3e bid, bdim;
        bid.x = b;
        bdim.x = spz::kThreads;
        emu::run_block(bid, bdim, [&] {
            spz::k_decode<W, FIRE, COL>(src, g, reinterpret_cast<typename spz::Elem<W>::T *>(dst), status);
        });
    }
    *blocks = grid;
}

template <int W, bool FIRE>
static bool dispatch_pc(uint32_t D, const uint8_t *src, const spz::Geom &g, uint8_t *dst, int32_t *st, uint32_t *nb,
                        bool batch) {
#define SPZ_EMU_D(D_)                                                 \
    case D_:                                                          \
        if (batch) run_pc_batch<W, FIRE, D_>(src, g, dst, st, nb);    \
        else run_pc<W, FIRE, D_>(src, g, dst, st, nb);                \
        return true;
    switch (D) {
        SPZ_EMU_D(1) SPZ_EMU_D(2) SPZ_EMU_D(3) SPZ_EMU_D(4) SPZ_EMU_D(5) SPZ_EMU_D(8) SPZ_EMU_D(16)
        default: return false;
    }
#undef SPZ_EMU_D
}

int main(int argc, char **argv) {
    if (argc != 3 && !(argc == 4 && strcmp(argv[3], "batch") == 0)) {
        fprintf(stderr, "usage: %s <container> <rows out> [batch]\n", argv[0]);
        return 2;
    }
    const bool batch = argc == 4;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    std::vector<uint8_t> buf;
    uint8_t tmp[1 << 16];
    size_t k;
    while ((k = fread(tmp, 1, sizeof tmp, f)) > 0) buf.insert(buf.end(), tmp, tmp + k);
    fclose(f);
    if (buf.size() < 64) return 2;
    // exactly the container's bytes in a fresh allocation, so that reads past
    // its end are caught
    uint8_t *src = (uint8_t *)malloc(buf.size());
    memcpy(src, buf.data(), buf.size());
    const uint32_t w = src[6], forecaster = src[8], learn_shift = src[9], G = src[10];
    const uint32_t D = (uint32_t)le(src + 12, 4), S = (uint32_t)le(src + 24, 4), nseg = (uint32_t)le(src + 28, 4);
    const uint64_t rows = le(src + 16, 8), data_bytes = le(src + 32, 8);
    spz::Geom g;
    memset(&g, 0, sizeof g);
    g.rows = rows; g.D = D; g.S = S; g.nseg = nseg; g.G = G;
    uint32_t lg = 0;
    while ((1u << lg) < D) ++lg;
    g.dp_log2 = lg;
    g.sh = learn_shift + 2;
    g.acc_lo = -(int32_t)((1u << (w - 1)) << g.sh);
    g.acc_hi = (int32_t)((1u << w) << g.sh);
    g.data_start = (64 + 8ull * (nseg + 1) + 15) & ~15ull;
    g.cap = buf.size();
    g.data_bytes = data_bytes;
    if (g.data_start + data_bytes > buf.size()) {
        fprintf(stderr, "container shorter than its header says\n");
        return 2;
    }
    const size_t outb = (size_t)rows * D * (w / 8);
    uint8_t *dst = (uint8_t *)aligned_alloc(16, outb ? (outb + 15) & ~size_t(15) : 16);
    memset(dst, 0x5A, outb);
    int32_t status = 0;
    emu::add_region(src, buf.size(), false);
    emu::add_region(dst, outb, true);
    emu::add_region(&status, sizeof status, true);
    uint32_t blocks = 0;
    const bool pc = G == 0 && D <= 16 && ((uint64_t)S * D * (w / 8)) % 16 == 0;
    const bool col = (uint64_t)D * w <= 32;
    bool ran = false;
    if (nseg > 0 && pc) {
        if (w == 8) ran = forecaster ? dispatch_pc<8, true>(D, src, g, dst, &status, &blocks, batch)
                                     : dispatch_pc<8, false>(D, src, g, dst, &status, &blocks, batch);
        else ran = forecaster ? dispatch_pc<16, true>(D, src, g, dst, &status, &blocks, batch)
                              : dispatch_pc<16, false>(D, src, g, dst, &status, &blocks, batch);
    } else if (nseg > 0) {
        ran = true;
        if (w == 8) {
            if (forecaster) col ? run_walker<8, true, true>(src, g, dst, &status, &blocks)
                                : run_walker<8, true, false>(src, g, dst, &status, &blocks);
            else col ? run_walker<8, false, true>(src, g, dst, &status, &blocks)
                     : run_walker<8, false, false>(src, g, dst, &status, &blocks);
        } else {
            if (forecaster) col ? run_walker<16, true, true>(src, g, dst, &status, &blocks)
                                : run_walker<16, true, false>(src, g, dst, &status, &blocks);
            else col ? run_walker<16, false, true>(src, g, dst, &status, &blocks)
                     : run_walker<16, false, false>(src, g, dst, &status, &blocks);
        }
    } else {
        ran = true;
    }
    if (!ran) {
        fprintf(stderr, "D = %u is not built into this harness\n", D);
        return 2;
    }
    FILE *o = fopen(argv[2], "wb");
    if (!o) return 2;
    if (outb) fwrite(dst, 1, outb, o);
    fclose(o);
    printf("status=%d violations=%zu blocks=%u\n", status, emu::violations(), blocks);
    free(src);
    free(dst);
    return 0;
}

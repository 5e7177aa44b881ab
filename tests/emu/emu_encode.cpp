// CPU harness: compresses rows with the single-pass encoder's own source
// (k_encode_sp, k_enc_scan, k_enc_compact, in the geometry the library
// launches them with), every workgroup run by the coroutine scheduler of
// emu_sched.h with bounds-checked buffer resources and global accessors
// under AddressSanitizer.
//
//   emu_encode <rows in> <rows> <D> <dtype 1..4: int8, uint8, int16, uint16> <forecaster 0|1> <seg_rows>
//              <learn_shift> <container out>
// Prints "status=<status word> violations=<out-of-bounds accesses> size=<container bytes>".
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <vector>

#include "spz_encode_sp.h"

template <int W, bool FIRE, int D>
static void run(const uint8_t *src, const spz::Geom &g, uint8_t *ws, uint64_t stride, uint8_t *dst,
                uint64_t *out_size, int32_t *status, uint32_t dtype, uint32_t forecaster, uint32_t ls) {
    using G = spz::EsGeom<W, D>;
    spz::u32x4 *info = reinterpret_cast<spz::u32x4 *>(ws);
    uint8_t *slots = ws + ((16 * (size_t)g.nseg + 255) & ~size_t(255));
    const uint32_t grid = (g.nseg + G::SPW - 1) / G::SPW;
    for (uint32_t b = 0; b < grid; ++b) {
        emu::dim3e bid, bdim;
        bid.x = b;
        bdim.x = G::NT;
        emu::run_block(bid, bdim, [&] { spz::k_encode_sp<W, FIRE, D>(src, g, slots, stride, info); });
    }
    {
        emu::dim3e bid, bdim;
        bdim.x = 1024;
        emu::run_block(bid, bdim, [&] {
            spz::k_enc_scan(info, g, (uint32_t)W, dtype, forecaster, ls, dst, out_size, status);
        });
    }
    const uint64_t units = stride / 16;
    const uint32_t K = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(256, 2048 / units));
    for (uint32_t b = 0; b < (g.nseg + K - 1) / K; ++b) {
        emu::dim3e bid, bdim;
        bid.x = b;
        bdim.x = 256;
        emu::run_block(bid, bdim, [&] { spz::k_enc_compact(slots, stride, info, g, (uint32_t)W, K, dst, status); });
    }
}

template <int W, bool FIRE>
static bool dispatch(uint32_t D, const uint8_t *src, const spz::Geom &g, uint8_t *ws, uint64_t stride, uint8_t *dst,
                     uint64_t *out_size, int32_t *status, uint32_t dtype, uint32_t f, uint32_t ls) {
    switch (D) {
        case 1: run<W, FIRE, 1>(src, g, ws, stride, dst, out_size, status, dtype, f, ls); return true;
        case 2: run<W, FIRE, 2>(src, g, ws, stride, dst, out_size, status, dtype, f, ls); return true;
        case 3: run<W, FIRE, 3>(src, g, ws, stride, dst, out_size, status, dtype, f, ls); return true;
        case 8: run<W, FIRE, 8>(src, g, ws, stride, dst, out_size, status, dtype, f, ls); return true;
        case 16: run<W, FIRE, 16>(src, g, ws, stride, dst, out_size, status, dtype, f, ls); return true;
        default: return false;
    }
}

int main(int argc, char **argv) {
    if (argc != 9) {
        fprintf(stderr, "usage: %s <rows in> <rows> <D> <dtype code 1..4> <forecaster> <seg_rows> <learn_shift> <out>\n", argv[0]);
        return 2;
    }
    const uint64_t rows = strtoull(argv[2], nullptr, 10);
    const uint32_t D = (uint32_t)atoi(argv[3]), dtype = (uint32_t)atoi(argv[4]), f = (uint32_t)atoi(argv[5]);
    if (dtype < 1 || dtype > 4) return 2;
    const uint32_t w = dtype <= 2 ? 8 : 16;   // int8, uint8, int16, uint16
    const uint32_t S = (uint32_t)atoi(argv[6]), ls = (uint32_t)atoi(argv[7]);
    const size_t inb = (size_t)rows * D * (w / 8);
    uint8_t *src = (uint8_t *)aligned_alloc(16, inb ? (inb + 15) & ~size_t(15) : 16);
    FILE *fi = fopen(argv[1], "rb");
    if (!fi || (inb && fread(src, 1, inb, fi) != inb)) return 2;
    fclose(fi);
    spz::Geom g;
    memset(&g, 0, sizeof g);
    g.rows = rows; g.D = D; g.S = S; g.G = 0;
    g.nseg = rows == 0 ? 0 : (uint32_t)((rows + S - 1) / S);
    uint32_t lg = 0;
    while ((1u << lg) < D) ++lg;
    g.dp_log2 = lg;
    g.sh = ls + 2;
    g.acc_lo = -(int32_t)((1u << (w - 1)) << g.sh);
    g.acc_hi = (int32_t)((1u << w) << g.sh);
    g.data_start = (64 + 8ull * (g.nseg + 1) + 15) & ~15ull;
    // container bound (every block at full width) and the single-pass workspace
    const uint32_t hb = w == 8 ? 3 : 4;
    uint64_t cap = g.data_start;
    for (uint32_t s = 0; s < g.nseg; ++s) {
        const uint64_t r = std::min<uint64_t>(S, rows - (uint64_t)s * S), nblk = r / 8, tail = r % 8;
        cap += 4 + (nblk * D * hb + 7) / 8 + 1 + nblk * D * w + tail * D * (w / 8) + 15;
    }
    g.cap = cap;
    const uint64_t stride = spz::es_slot_bytes(S >> 3, D, w);
    const size_t wsz = ((16 * (size_t)g.nseg + 255) & ~size_t(255)) + g.nseg * stride;
    uint8_t *ws = (uint8_t *)aligned_alloc(256, wsz ? (wsz + 255) & ~size_t(255) : 256);
    memset(ws, 0xCD, wsz);   // the workspace holds garbage on entry
    uint8_t *dst = (uint8_t *)aligned_alloc(16, (cap + 15) & ~uint64_t(15));
    memset(dst, 0xA5, cap);
    uint64_t out_size = 0;
    int32_t status = 0;
    emu::add_region(src, inb, false);
    emu::add_region(ws, wsz, true);
    emu::add_region(dst, cap, true);
    emu::add_region(&out_size, sizeof out_size, true);
    emu::add_region(&status, sizeof status, true);
    bool ok;
    if (w == 8) ok = f ? dispatch<8, true>(D, src, g, ws, stride, dst, &out_size, &status, dtype, f, ls)
                       : dispatch<8, false>(D, src, g, ws, stride, dst, &out_size, &status, dtype, f, ls);
    else ok = f ? dispatch<16, true>(D, src, g, ws, stride, dst, &out_size, &status, dtype, f, ls)
                : dispatch<16, false>(D, src, g, ws, stride, dst, &out_size, &status, dtype, f, ls);
    if (!ok) {
        fprintf(stderr, "D = %u is not built into this harness\n", D);
        return 2;
    }
    FILE *o = fopen(argv[8], "wb");
    if (!o) return 2;
    if (out_size <= cap) fwrite(dst, 1, out_size, o);
    fclose(o);
    printf("status=%d violations=%zu size=%llu\n", status, emu::violations(), (unsigned long long)out_size);
    free(src);
    free(ws);
    free(dst);
    return 0;
}

// Host emulation of workgroups for the CPU test harness of the HIP kernels.
//
// Every thread of a workgroup runs as a coroutine (ucontext) on the host.
// A lane runs until it reaches a point where lanes meet: a workgroup
// barrier, a wavefront hand-off point or a cross-lane operation (DPP move,
// shuffle, first-lane read). The scheduler resumes the lanes of a wavefront
// only when all of its unfinished lanes wait at the same kind of point, and
// computes cross-lane results from the values every lane left there; it
// aborts if the lanes of a wavefront disagree (divergent cross-lane code) or
// a workgroup barrier is not reached by all lanes. Lanes between meeting
// points run one after another, which is a valid interleaving of lockstep
// execution for code that hands values between lanes only at those points.
#pragma once

#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <ucontext.h>

#include <functional>
#include <vector>

#if defined(__has_feature)
#if __has_feature(address_sanitizer)
#define EMU_ASAN 1
#endif
#endif
#ifdef EMU_ASAN
extern "C" {
void __sanitizer_start_switch_fiber(void **fake_stack_save, const void *bottom, size_t size);
void __sanitizer_finish_switch_fiber(void *fake_stack_save, const void **bottom_old, size_t *size_old);
}
#endif

namespace emu {

struct dim3e {
    uint32_t x = 0, y = 0, z = 0;
};

enum Wait { RUN = 0, WAVE_OP, WAVE_SYNC, BARRIER, DONE };

// cross-lane operations
enum Op { OP_DPP = 1, OP_SHFL_UP, OP_SHFL, OP_FIRST };

struct Lane {
    ucontext_t ctx;
    std::vector<char> stack;
    dim3e tid;
    int wave = 0, lane = 0;
    Wait wait = RUN;
    int op = 0;
    int param = 0, width = 0;
    uint32_t val = 0, res = 0;
};

struct Block {
    std::vector<Lane> lanes;
    ucontext_t sched;
    int cur = -1;
    std::function<void()> body;
    dim3e bid, bdim;
};

inline Block *&current_block() {
    static Block *b = nullptr;
    return b;
}
inline Lane &me() { return current_block()->lanes[current_block()->cur]; }

[[noreturn]] inline void fail(const char *what) {
    fprintf(stderr, "emulation error: %s (block %u, thread %u)\n", what, current_block() ? current_block()->bid.x : 0u,
            current_block() && current_block()->cur >= 0 ? me().tid.x : 0u);
    exit(3);
}

inline void yield_to_scheduler() {
    Block *b = current_block();
    Lane &l = b->lanes[b->cur];
#ifdef EMU_ASAN
    void *fs = nullptr;
    __sanitizer_start_switch_fiber(&fs, nullptr, 0);
#endif
    swapcontext(&l.ctx, &b->sched);
#ifdef EMU_ASAN
    __sanitizer_finish_switch_fiber(fs, nullptr, nullptr);
#endif
}

inline void lane_entry() {
#ifdef EMU_ASAN
    __sanitizer_finish_switch_fiber(nullptr, nullptr, nullptr);
#endif
    Block *b = current_block();
    b->body();
    b->lanes[b->cur].wait = DONE;
    yield_to_scheduler();
}

// cross-lane values
inline uint32_t dpp_source(int ctrl, int i) {
    const int r = i & ~15, p = i & 15;
    if (ctrl >= 0x111 && ctrl <= 0x11F) {            // row_shr:n
        const int n = ctrl - 0x110;
        return p >= n ? (uint32_t)(i - n) : ~0u;
    }
    if (ctrl <= 0xFF) {                               // quad_perm
        const int sel = (ctrl >> (2 * (i & 3))) & 3;
        return (uint32_t)((i & ~3) + sel);
    }
    if (ctrl == 0x140) return (uint32_t)(r + 15 - p);           // row_mirror
    if (ctrl == 0x141) return (uint32_t)((i & ~7) + 7 - (i & 7));  // row_half_mirror
    fail("DPP control not emulated");
}

inline void resolve_wave(Block &b, int w, int nthreads) {
    const int base = 64 * w, n = nthreads - base < 64 ? nthreads - base : 64;
    int op = -1, param = 0, width = 0;
    for (int i = 0; i < n; ++i) {
        Lane &l = b.lanes[base + i];
        if (l.wait == DONE) continue;
        if (op < 0) { op = l.op; param = l.param; width = l.width; }
        if (l.op != op || l.param != param || l.width != width) fail("lanes of a wavefront at different cross-lane operations");
    }
    auto value = [&](uint32_t src) -> uint32_t {
        if (src >= (uint32_t)n) return 0u;
        const Lane &s = b.lanes[base + src];
        return s.wait == DONE ? 0u : s.val;   // finished lanes read as inactive
    };
    for (int i = 0; i < n; ++i) {
        Lane &l = b.lanes[base + i];
        if (l.wait == DONE) continue;
        switch (op) {
            case OP_DPP: l.res = value(dpp_source(param, i)); break;
            case OP_SHFL_UP: {
                const int wd = width, p = i % wd;
                l.res = p >= param ? value((uint32_t)(i - param)) : l.val;
                break;
            }
            case OP_SHFL: {
                const int wd = width;
                l.res = value((uint32_t)((i & ~(wd - 1)) + (param % wd)));
                break;
            }
            case OP_FIRST: {
                uint32_t v = 0;
                for (int k = 0; k < n; ++k)
                    if (b.lanes[base + k].wait != DONE) { v = b.lanes[base + k].val; break; }
                l.res = v;
                break;
            }
            default: fail("unknown cross-lane operation");
        }
        l.wait = RUN;
    }
}

// Runs `body` for every thread of one workgroup of nthreads threads.
inline void run_block(dim3e bid, dim3e bdim, const std::function<void()> &body, size_t stack_bytes = 256 << 10) {
    Block b;
    b.bid = bid;
    b.bdim = bdim;
    b.body = body;
    const int nt = (int)bdim.x;
    b.lanes.resize(nt);
    current_block() = &b;
    for (int t = 0; t < nt; ++t) {
        Lane &l = b.lanes[t];
        l.tid.x = (uint32_t)t;
        l.wave = t / 64;
        l.lane = t % 64;
        l.stack.resize(stack_bytes);
        getcontext(&l.ctx);
        l.ctx.uc_stack.ss_sp = l.stack.data();
        l.ctx.uc_stack.ss_size = l.stack.size();
        l.ctx.uc_link = nullptr;
        makecontext(&l.ctx, (void (*)())lane_entry, 0);
    }
    const int nw = (nt + 63) / 64;
    for (;;) {
        bool any = false;
        for (int t = 0; t < nt; ++t) {
            Lane &l = b.lanes[t];
            if (l.wait != RUN) continue;
            any = true;
            b.cur = t;
#ifdef EMU_ASAN
            void *fs = nullptr;
            __sanitizer_start_switch_fiber(&fs, l.stack.data(), l.stack.size());
#endif
            swapcontext(&b.sched, &l.ctx);
#ifdef EMU_ASAN
            __sanitizer_finish_switch_fiber(fs, nullptr, nullptr);
#endif
            b.cur = -1;
        }
        if (any) continue;
        // every lane waits or is done: release what can go on
        bool all_done = true, progressed = false;
        for (int t = 0; t < nt; ++t) all_done = all_done && b.lanes[t].wait == DONE;
        if (all_done) break;
        for (int w = 0; w < nw; ++w) {
            const int base = 64 * w, n = nt - base < 64 ? nt - base : 64;
            int waiting = 0, kind = -1;
            bool mixed = false;
            for (int i = 0; i < n; ++i) {
                const Lane &l = b.lanes[base + i];
                if (l.wait == DONE) continue;
                ++waiting;
                if (kind < 0) kind = l.wait;
                else if (kind != l.wait) mixed = true;
            }
            if (!waiting || kind == BARRIER) continue;
            if (mixed) fail("lanes of a wavefront wait at different kinds of points");
            if (kind == WAVE_OP) resolve_wave(b, w, nt);
            else for (int i = 0; i < n; ++i) if (b.lanes[base + i].wait == WAVE_SYNC) b.lanes[base + i].wait = RUN;
            progressed = true;
        }
        if (progressed) continue;
        // only barrier waits left: every unfinished lane must be there
        for (int t = 0; t < nt; ++t)
            if (b.lanes[t].wait != BARRIER && b.lanes[t].wait != DONE) fail("barrier not reached by every lane");
        // (lanes that have left the kernel do not take part, as on the device)
        for (int t = 0; t < nt; ++t)
            if (b.lanes[t].wait == BARRIER) b.lanes[t].wait = RUN;
    }
    current_block() = nullptr;
}

// meeting points, called from lane code
inline void barrier() {
    me().wait = BARRIER;
    yield_to_scheduler();
}
inline void wave_sync() {
    me().wait = WAVE_SYNC;
    yield_to_scheduler();
}
inline uint32_t wave_op(int op, uint32_t v, int param, int width) {
    Lane &l = me();
    l.op = op;
    l.val = v;
    l.param = param;
    l.width = width;
    l.wait = WAVE_OP;
    yield_to_scheduler();
    return me().res;
}

}  // namespace emu

"""Continuous-batching request loop for the Sprintz codec on one GPU.

Requests to compress a (rows, D) series or to decompress a container arrive
over time. The server

* admits a request as soon as its device buffers fit in the HBM budget (one
  preallocated arena, first-fit; nothing is allocated per request);
* launches everything admitted so far as one batch on the next of a few HIP
  streams: all decodes of the batch in one batched call (sprintz_batch_*
  with its plan built in arena memory by an asynchronous copy), all encodes
  in one batched compression call (sprintz_compress_batch_*, its plan in
  arena memory too, every request coding into its own reserved workspace);
  batches on different streams run on the device at the same time, so
  requests that arrive while others are on the GPU start without waiting
  for them;
* polls an event per batch without blocking, reports each request's latency
  (arrival to completion seen by the host) and returns its memory to the
  arena.

The codec itself is unchanged: every request is computed by the same C-ABI
calls as when it runs alone, so results in the mix equal results alone,
byte for byte."""
from __future__ import annotations

import bisect
import time
from dataclasses import dataclass, field

from . import (SPZ_OK, SprintzError, dtype_code, load, make_params, spz_batch_item, spz_compress_item, spz_info,
               sprintz_batch_create_in, sprintz_batch_decompress, sprintz_batch_destroy,
               sprintz_batch_workspace_size, sprintz_compress_batch, sprintz_compress_batch_create_in,
               sprintz_compress_batch_destroy, sprintz_compress_batch_workspace_size, sprintz_compress_bound,
               sprintz_workspace_size)

ALIGN = 256


class DevicePool:
    """First-fit allocator over one device byte arena (the admission budget)."""

    def __init__(self, nbytes: int, device="cuda"):
        import torch
        self.size = nbytes
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.base = self.buf.data_ptr()
        self.free = [(0, nbytes)]   # sorted (offset, size)
        self.used = 0

    def alloc(self, n: int):
        n = max(ALIGN, (n + ALIGN - 1) // ALIGN * ALIGN)
        for i, (off, sz) in enumerate(self.free):
            if sz >= n:
                if sz == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (off + n, sz - n)
                self.used += n
                return off, n
        return None

    def release(self, off: int, n: int) -> None:
        self.used -= n
        i = bisect.bisect_left(self.free, (off, 0))
        self.free.insert(i, (off, n))
        # merge with neighbours
        if i + 1 < len(self.free) and self.free[i][0] + self.free[i][1] == self.free[i + 1][0]:
            self.free[i] = (off, self.free[i][1] + self.free[i + 1][1])
            self.free.pop(i + 1)
        if i > 0 and self.free[i - 1][0] + self.free[i - 1][1] == self.free[i][0]:
            self.free[i - 1] = (self.free[i - 1][0], self.free[i - 1][1] + self.free[i][1])
            self.free.pop(i)

    def view(self, off: int, n: int):
        return self.buf[off:off + n]


@dataclass
class Request:
    """kind 'encode': x is a (rows, D) CUDA tensor; kind 'decode': container is
    a uint8 CUDA tensor and info its parsed header. arrival is in seconds from
    the start of the run."""
    id: int
    kind: str
    arrival: float
    x: object = None
    forecaster: str = "fire"
    seg_rows: int = 1024
    container: object = None
    info: spz_info | None = None
    # filled by the server
    admitted: float = -1.0
    done: float = -1.0
    allocs: list = field(default_factory=list)
    result: object = None   # encode: container bytes (uint8 tensor); decode: (rows, D) tensor
    nbytes: int = 0         # uncompressed bytes of the request
    status: int = 0
    keep: bool = False      # copy the result out (else only its size is reported)

    def need_bytes(self) -> int:
        if self.kind == "encode":
            rows, D = self.x.shape
            p = make_params(self.forecaster, self.seg_rows)
            return (sprintz_compress_bound(rows, D, dtype_code(self.x), p) + ALIGN
                    + sprintz_workspace_size(rows, D, dtype_code(self.x), p) + ALIGN)
        return self.info.rows * self.info.D * (self.info.w // 8) + ALIGN


@dataclass
class _Batch:
    stream: object
    event: object
    reqs: list
    plan: int | None
    cplan: int | None    # compression plan of the batch's encodes
    allocs: tuple        # the batch's region of the metadata arena
    status_off: int      # its offset: status words, output sizes, plan tables


class Server:
    def __init__(self, budget_bytes: int, nstreams: int = 4, max_batch: int = 512, keep_results: bool = False,
                 meta_bytes: int = 64 << 20, device="cuda"):
        import torch
        load()
        self.torch = torch
        self.pool = DevicePool(budget_bytes, device)        # request buffers: the admission budget
        self.meta = DevicePool(meta_bytes, device)          # per-batch status words and plan tables
        self.streams = [torch.cuda.Stream(device=device) for _ in range(nstreams)]
        self.next_stream = 0
        self.max_batch = max_batch
        self.keep = keep_results
        self.pending: list[Request] = []     # arrived, waiting for memory
        self.admitted: list[Request] = []    # memory reserved, not launched
        self.inflight: list[_Batch] = []
        self.completed: list[Request] = []
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    # -- admission -------------------------------------------------------------
    def submit(self, r: Request) -> None:
        self.pending.append(r)

    def _admit(self) -> None:
        keep = []
        for r in self.pending:
            need = r.need_bytes()
            if need > self.pool.size:
                raise SprintzError(-2, f"request {r.id} needs {need} B, more than the whole budget")
            a = self.pool.alloc(need)
            if a is None:
                keep.append(r)     # waits for memory; later requests may still fit
                continue
            r.allocs.append(a)
            r.admitted = self.now()
            self.admitted.append(r)
        self.pending = keep

    # -- launching -------------------------------------------------------------
    def _launch(self) -> None:
        if not self.admitted:
            return
        reqs, self.admitted = self.admitted[: self.max_batch], self.admitted[self.max_batch:]
        reqs.sort(key=lambda r: r.kind != "decode")       # decodes first: item k <-> status word k
        torch = self.torch
        # batch metadata from its own arena: n status words and n output sizes,
        # then the plan tables of the decodes; a batch that does not fit is halved
        while True:
            n = len(reqs)
            decs = [r for r in reqs if r.kind == "decode"]
            items, infos = [], []
            for r in decs:
                off, _ = r.allocs[0]
                nb = r.info.rows * r.info.D * (r.info.w // 8)
                items.append(spz_batch_item(r.container.data_ptr(), r.container.numel(), self.pool.base + off, nb))
                infos.append(r.info)
            wsz = sprintz_batch_workspace_size(items, infos) if decs else 0
            encs = [(i, r) for i, r in enumerate(reqs) if r.kind == "encode"]
            citems = []
            for i, r in encs:
                rows, D = r.x.shape
                dt = dtype_code(r.x)
                p = make_params(r.forecaster, r.seg_rows)
                cap = sprintz_compress_bound(rows, D, dt, p)
                off, _ = r.allocs[0]
                dst = self.pool.base + off
                ws = dst + (cap + ALIGN - 1) // ALIGN * ALIGN
                # d_out_size is set below, once the batch's metadata is placed (8 is a
                # stand-in that only sizes the plan)
                citems.append(spz_compress_item(r.x.data_ptr(), rows, D, dt, p, dst, cap, 8, ws,
                                                sprintz_workspace_size(rows, D, dt, p)))
            cwsz = sprintz_compress_batch_workspace_size(citems) if encs else 0
            meta = self.meta.alloc(16 * n + 16 + (wsz + ALIGN - 1) // ALIGN * ALIGN + ALIGN + cwsz)
            if meta is not None:
                break
            if n == 1:
                if not self.inflight:
                    raise SprintzError(-2, "batch metadata does not fit in the metadata arena")
                self.admitted = reqs + self.admitted     # wait for running batches to free it
                return
            self.admitted = reqs[n // 2:] + self.admitted
            reqs = reqs[: n // 2]
        s = self.streams[self.next_stream]
        self.next_stream = (self.next_stream + 1) % len(self.streams)
        sh = int(s.cuda_stream)
        st_ptr = self.meta.base + meta[0]
        sz_off = meta[0] + (4 * n + 15) // 16 * 16
        ws_off = meta[0] + 16 * n + 16
        with torch.cuda.stream(s):
            self.meta.view(meta[0], 16 * n + 16).zero_()
        plan = cplan = None
        if decs:
            for r in decs:
                r.result = (r.allocs[0][0], r.info.rows * r.info.D * (r.info.w // 8))
            plan = sprintz_batch_create_in(items, infos, self.meta.base + ws_off, max(wsz, 16), sh)
            rc = sprintz_batch_decompress(plan, st_ptr, sh)
            if rc != SPZ_OK:
                raise SprintzError(rc, "sprintz_batch_decompress")
        if encs:
            # the encodes' status words and sizes follow the decodes' (item k of
            # the compression batch is request encs[k][0])
            k0 = encs[0][0]
            for k, (i, r) in enumerate(encs):
                citems[k].d_out_size = self.meta.base + sz_off + 8 * i
                r.result = (r.allocs[0][0], 0)
            cws = self.meta.base + (ws_off + (wsz + ALIGN - 1) // ALIGN * ALIGN + ALIGN - 1) // ALIGN * ALIGN
            cplan = sprintz_compress_batch_create_in(citems, cws, max(cwsz, 16), sh)
            rc = sprintz_compress_batch(cplan, st_ptr + 4 * k0, sh)
            if rc != SPZ_OK:
                raise SprintzError(rc, "sprintz_compress_batch")
        ev = torch.cuda.Event()
        ev.record(s)
        self.inflight.append(_Batch(s, ev, reqs, plan, cplan, meta, meta[0]))

    # -- completion ------------------------------------------------------------
    def _poll(self) -> bool:
        progressed = False
        keep = []
        torch = self.torch
        for b in self.inflight:
            if not b.event.query():
                keep.append(b)
                continue
            progressed = True
            t = self.now()
            n = len(b.reqs)
            meta = self.meta.view(b.status_off, 16 * n + 16).cpu()     # one copy per batch
            status = meta[: 4 * n].view(torch.int32)
            sizes = meta[(4 * n + 15) // 16 * 16:(4 * n + 15) // 16 * 16 + 8 * n].view(torch.int64)
            for i, r in enumerate(b.reqs):
                r.status = int(status[i])
                off, nb = r.result
                if r.kind == "encode":
                    size = int(sizes[i])
                    r.result = self.pool.view(off, size).clone() if (self.keep or r.keep) else size
                    r.nbytes = r.x.numel() * r.x.element_size()
                else:
                    r.nbytes = nb
                    r.result = self.pool.view(off, nb).clone() if (self.keep or r.keep) else None
                r.done = t
                self.completed.append(r)
            if self.keep or any(r.keep for r in b.reqs):
                # the copies above run on this thread's stream: let them finish
                # before another batch may reuse the memory
                torch.cuda.current_stream().synchronize()
            for r in b.reqs:
                for a in r.allocs:
                    self.pool.release(*a)
                r.allocs = []
            if b.plan is not None:
                sprintz_batch_destroy(b.plan)
            if b.cplan is not None:
                sprintz_compress_batch_destroy(b.cplan)
            self.meta.release(*b.allocs)
        self.inflight = keep
        return progressed

    def step(self) -> bool:
        """One round of admission, launching and polling; True if anything moved."""
        before = (len(self.pending), len(self.admitted), len(self.inflight), len(self.completed))
        self._admit()
        if self.admitted and len(self.inflight) < len(self.streams):
            self._launch()
        self._poll()
        return before != (len(self.pending), len(self.admitted), len(self.inflight), len(self.completed))

    def run(self, requests, realtime: bool = True):
        """Feed requests at their arrival times (seconds from now) and serve
        until all have completed; returns them in completion order."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        self.t0 = time.perf_counter()
        k = 0
        while k < len(reqs) or self.pending or self.admitted or self.inflight:
            now = self.now()
            while k < len(reqs) and (not realtime or reqs[k].arrival <= now):
                self.submit(reqs[k])
                k += 1
            moved = self.step()
            if not moved and k < len(reqs) and realtime:
                time.sleep(min(max(reqs[k].arrival - self.now(), 0.0), 50e-6))
        self.torch.cuda.synchronize()
        return self.completed


def latency_stats(done) -> dict:
    import numpy as np
    lat = np.array([r.done - r.arrival for r in done])
    return {"p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
            "mean_ms": round(float(lat.mean()) * 1e3, 3)}

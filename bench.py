"""Benchmark of the gfx950 Sprintz codec on one GPU.

A step is one pass of the whole hot path over one batch: compress the
4,194,304 x 8 uint16 AR(2) stream (FIRE forecaster, 1,024-row segments) and
decompress the container again. Inputs are resident in HBM before timing;
eight buffer sets rotate (> 1 GB touched between reuses) so the 256 MB
Infinity Cache cannot hold a step's data. Phases are timed with HIP events on
the library's stream. Every measured output is checked against the input and
every container against the CPU oracle's bytes.

Prints one JSON line. ``value`` is decode throughput in GB/s of uncompressed
bytes (GB = 1e9); encode throughput, HBM-roofline fractions and the CPU
oracle baseline ride along.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, published


def kernel_source_hash() -> str:
    """sha256 (first 16 hex digits) of the device code: the kernel headers
    csrc/spz_*.h. The host runtime (sprintz.hip: validation, plans, stream
    order) does not change the bytes a kernel launch moves."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1808_02515_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if not (f.startswith("spz_") and f.endswith(".h")):
            continue
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stream_workload_name(rows: int, D: int, forecaster: str, seg_rows: int) -> str:
    """Name of the single-stream workload, as the counter summaries key it."""
    return f"ar2_uint16 {rows}x{D} {forecaster} seg_rows={seg_rows}"


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel sources (else None)."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as fh:
        d = json.load(fh)
    e = d.get(f"{kernel}|{workload}")
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def host_description() -> dict:
    """CPU model (from /proc/cpuinfo, as lscpu reports it), logical CPUs and
    the CPUs this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


def cpu_baseline_all_cores(x, forecaster, seg_rows, threads):
    """The CPU oracle on `threads` threads over independent parts of the
    stream (whole segments each, so the segments are those of the whole
    stream): wall time of compressing all parts, then of decompressing them.
    ctypes releases the interpreter lock during the oracle's calls."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor

    rows = x.shape[0]
    per = -(-rows // threads)
    per = -(-per // seg_rows) * seg_rows
    parts = [x[k:k + per] for k in range(0, rows, per)]
    with ThreadPoolExecutor(max_workers=threads) as pool:
        t0 = time.perf_counter()
        blobs = list(pool.map(lambda p: oracle.compress(p, forecaster, seg_rows), parts))
        enc = time.perf_counter() - t0
        t0 = time.perf_counter()
        ys = list(pool.map(oracle.decompress, blobs))
        dec = time.perf_counter() - t0
    assert all(np.array_equal(y, p) for y, p in zip(ys, parts))
    return dec, enc, len(parts)


def cpu_baseline(x, forecaster, seg_rows, budget_s=20.0):
    """The CPU oracle on this host (1 thread): decode and encode of the same
    stream, best of up to 3 runs within the time budget."""
    import oracle

    t0 = time.perf_counter()
    blob = oracle.compress(x, forecaster, seg_rows)
    enc = [time.perf_counter() - t0]
    dec = []
    while True:
        t0 = time.perf_counter()
        y = oracle.decompress(blob)
        dec.append(time.perf_counter() - t0)
        assert np.array_equal(y, x)
        spent = sum(enc) + sum(dec)
        if len(dec) >= 3 or spent + dec[-1] + enc[-1] > budget_s:
            break
        t0 = time.perf_counter()
        oracle.compress(x, forecaster, seg_rows)
        enc.append(time.perf_counter() - t0)
    return blob, min(dec), min(enc), len(dec), len(enc)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--forecaster", default="fire", choices=["fire", "delta"])
    ap.add_argument("--seg-rows", type=int, default=1024,
                    help="stream workload: rows per segment; 0 = the library's autotuner (sprintz_autotune)")
    ap.add_argument("--rotate", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle-sample", action="store_true",
                    help="batch workload: skip comparing sampled containers with the oracle's bytes")
    ap.add_argument("--workload", default="stream",
                    choices=["stream", "batch", "serve", "dsweep", "huffman", "latency"],
                    help="stream: the 4,194,304 x 8 uint16 stream; batch: the many-stream batch; "
                         "serve: the request-serving loop; dsweep: speed against D on uniform values; "
                         "huffman: the 4 GiB D=4 uint16 walk with and without the entropy stage; "
                         "latency: the 65,536-sample int8 walk, call latency")
    ap.add_argument("--duration", type=float, default=10.0, help="serve: seconds of arrivals")
    ap.add_argument("--rate", type=float, default=2000.0, help="serve: requests per second (Poisson)")
    ap.add_argument("--streams", type=int, default=10000, help="batch workload: number of streams")
    ap.add_argument("--batch-streams", type=int, default=10000,
                    help="stream workload: also run this many streams of the batch workload, batched vs one "
                         "launch per stream (0: skip)")
    ap.add_argument("--huffman-streams", type=int, default=1024,
                    help="huffman workload: streams of the batched-vs-per-stream leg")
    ap.add_argument("--batched-only", action="store_true",
                    help="batch workload: time only the batched calls (skip the one-launch-per-stream legs, "
                         "tens of thousands of dispatches, which counter collection serialises)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run plain device copies of MIB MiB (HBM counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the codec has no multi-GPU path "
              "(segments are independent, so decoding shards across GPUs without communication). Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if args.calibrate_copy:
        n = args.calibrate_copy << 20
        a = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(7)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(max(args.steps, 1)):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n, "copies": max(args.steps, 1)}), flush=True)
        return

    import datagen
    import paper_1808_02515_amd as spz

    spz.load()
    if args.workload == "batch":
        print(json.dumps(run_batch(args)), flush=True)
        return
    if args.workload == "serve":
        run_serve(args)
        return
    if args.workload == "dsweep":
        run_dsweep(args)
        return
    if args.workload == "huffman":
        run_huffman(args)
        return
    if args.workload == "latency":
        run_latency(args)
        return
    dev = torch.device("cuda:0")
    rows, D = 4194304, 8
    print(f"[bench] generating ar2_uint16 {rows}x{D}", file=sys.stderr, flush=True)
    x_np = datagen.ar2_uint16(rows, D, seed=1)
    U = x_np.nbytes
    tune = None
    if args.seg_rows == 0:
        xt = torch.from_numpy(x_np).to(dev)
        args.seg_rows = spz.sprintz_autotune(xt.data_ptr(), rows, D, spz.SPZ_UINT16, spz.make_params(args.forecaster, 0),
                                             torch.cuda.current_stream().cuda_stream)
        tune = "library autotuner (sprintz_autotune)"
        del xt
        print(f"[bench] seg_rows {args.seg_rows} (autotuned)", file=sys.stderr, flush=True)
    workload = stream_workload_name(rows, D, args.forecaster, args.seg_rows)

    base_blob = cpu = None
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        base_blob, cpu_dec_s, cpu_enc_s, ndec, nenc = cpu_baseline(x_np, args.forecaster, args.seg_rows)
        host = host_description()
        threads = max(1, min(host["usable_cpus"], 16))
        all_dec_s, all_enc_s, nparts = cpu_baseline_all_cores(x_np, args.forecaster, args.seg_rows, threads)
        cpu = {"value": round(U / cpu_dec_s / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": f"the full {rows}x{D} uint16 stream ({U} B), decode best of {ndec}; "
                         f"encode {U / cpu_enc_s / 1e9:.4f} GB/s best of {nenc}",
               "encode_GBps": round(U / cpu_enc_s / 1e9, 4),
               "all_cores": {"cores": threads, "decode_GBps": round(U / all_dec_s / 1e9, 4),
                             "encode_GBps": round(U / all_enc_s / 1e9, 4),
                             "sample": f"the same stream in {nparts} parts of whole segments, one thread each"},
               **host}

    p = spz.make_params(args.forecaster, args.seg_rows)
    R = args.rotate
    x0 = torch.from_numpy(x_np).to(dev)
    xs = [x0.clone() for _ in range(R)]
    encs = [spz.Encoder.create(rows, D, spz.SPZ_UINT16, p, device=dev) for _ in range(R)]
    ys = [torch.empty_like(x0) for _ in range(R)]
    dstatus = torch.zeros(R, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)

    # container size is fixed for this input: learn it once (not timed)
    encs[0].run(xs[0], stream)
    torch.cuda.synchronize()
    csize = int(encs[0].out_size.item())
    info = spz.sprintz_get_info(encs[0].dst[:64].cpu().numpy().tobytes())

    def step(k, ev=None):
        r = k % R
        if ev is not None:
            ev[0].record(stream)
        encs[r].run(xs[r], stream)
        if ev is not None:
            ev[1].record(stream)
        rc = spz.sprintz_decompress(encs[r].dst.data_ptr(), csize, info, ys[r].data_ptr(), U,
                                    dstatus[r:r + 1].data_ptr(), sh)
        if rc != spz.SPZ_OK:
            raise spz.SprintzError(rc, "sprintz_decompress")
        if ev is not None:
            ev[2].record(stream)

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(args.warmup + k, evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    enc_ms = [e[0].elapsed_time(e[1]) for e in evs]
    dec_ms = [e[1].elapsed_time(e[2]) for e in evs]

    # parity of every measured buffer
    ok = int(dstatus.sum().item()) == 0 and all(int(e.status.item()) == 0 for e in encs)
    ok = ok and all(torch.equal(y, x0) for y in ys[: min(R, args.warmup + args.steps)])
    if base_blob is not None:
        # container bytes against the oracle's (made in the CPU leg)
        ref = torch.from_numpy(np.frombuffer(base_blob, np.uint8).copy()).to(dev)
        ok = ok and csize == len(base_blob)
        ok = ok and all(torch.equal(e.dst[:csize], ref) for e in encs[: min(R, args.warmup + args.steps)])
        parity = "bit-exact vs CPU oracle (container bytes and decoded samples, every rotated buffer)"
    else:
        ok = ok and all(torch.equal(e.dst[:csize], encs[0].dst[:csize]) for e in encs[: min(R, args.warmup + args.steps)])
        parity = "decoded samples equal to the input on every rotated buffer (oracle leg skipped)"
    if not ok:
        print("[bench] PARITY FAILURE", file=sys.stderr, flush=True)
        sys.exit(1)

    dec_mean = float(np.mean(dec_ms)) * 1e-3
    enc_mean = float(np.mean(enc_ms)) * 1e-3
    algo_bytes = U + csize  # decode reads the container and writes the samples
    dec_gbps = U / dec_mean / 1e9
    enc_gbps = U / enc_mean / 1e9
    achieved = algo_bytes / dec_mean / 1e9
    traffic = measured_traffic("k_decode_pc", workload)
    out = {
        "metric": "decode GB/s and encode GB/s (uncompressed bytes), % HBM peak, batched vs plain",
        "value": round(dec_gbps, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16",
        "data": "synthetic",
        "config": {"workload": workload, "rows": rows, "D": D, "dtype": "uint16", "forecaster": args.forecaster,
                   "seg_rows": args.seg_rows, "hdr_group": 0, "launch": "plain (one stream per call)",
                   "seg_rows_tuning": tune},
        "decode_GBps": round(dec_gbps, 2),
        "encode_GBps": round(enc_gbps, 2),
        "decode_ms": round(dec_mean * 1e3, 4),
        "encode_ms": round(enc_mean * 1e3, 4),
        "decode_best_ms": round(min(dec_ms), 4),
        "compressed_bytes": csize,
        "compression_ratio": round(U / csize, 4),
        "hbm_frac_decode": round(achieved / HBM_PEAK_GBPS, 4),
        "hbm_frac_encode": round((U + csize) / enc_mean / 1e9 / HBM_PEAK_GBPS, 4),
        "parity": parity,
        "roofline": {"bound": "hbm", "kernel": "k_decode_pc", "achieved": round(achieved, 2),
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": traffic, "algorithmic_bytes_per_launch": algo_bytes},
        "roofline_encode": {"bound": "hbm", "kernels": "k_encode_sp + k_enc_scan + k_enc_compact (one call)",
                            "achieved": round(algo_bytes / enc_mean / 1e9, 2), "peak": HBM_PEAK_GBPS,
                            "unit": "GB/s", "frac": round(algo_bytes / enc_mean / 1e9 / HBM_PEAK_GBPS, 4),
                            "traffic": measured_traffic("encode", workload),
                            "algorithmic_bytes_per_call": algo_bytes},
        "cpu_baseline": cpu,
        "paper_context": "paper: >3 GB/s single-thread decompression on an Intel i7-4960HQ (2.6 GHz, AVX2)",
    }
    if args.batch_streams > 0:
        del xs, encs, ys
        torch.cuda.empty_cache()
        bargs = argparse.Namespace(**vars(args))
        bargs.streams, bargs.steps, bargs.warmup, bargs.no_cpu_baseline = args.batch_streams, 5, 2, True
        b = run_batch(bargs)
        out["batched_vs_plain"] = {k: b[k] for k in (
            "batch_decode_GBps", "per_stream_decode_GBps", "batched_vs_per_stream", "per_stream_graph_decode_GBps",
            "batched_vs_per_stream_graph", "graph_decode_GBps", "batch_encode_GBps", "per_stream_encode_GBps",
            "encode_batched_vs_per_stream", "u16_fire_decode_GBps", "u16_fire_hbm_frac", "compression_ratio",
            "parity", "roofline")}
        out["batched_vs_plain"]["workload"] = b["config"]["workload"]
        out["batched_vs_plain"]["seg_rows_per_class"] = b["config"]["seg_rows_per_class"]
    print(json.dumps(out), flush=True)


def _events(n):
    import torch
    return [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]


def _r(v, nd):
    return None if v is None else round(v, nd)


def run_batch(args):
    """The many-stream workload: streams drawn on the GPU; segment sizes from
    the library's autotuner (once per class dtype x D); compression (a) in
    one batched call (sprintz_compress_batch) and (b) one sprintz_compress
    launch per stream; decompression (a) in one batched call per class work
    list, (b) as a captured HIP graph of that call, (c) one
    sprintz_decompress launch per stream, eager and (d) captured as one
    graph of all those launches (no host overhead). Every output is
    compared with its input; a deterministic sample of containers with the
    CPU oracle's bytes."""
    import torch
    import datagen
    import oracle
    import paper_1808_02515_amd as spz

    n = args.streams
    t0 = time.time()
    streams = [datagen.batch_stream_torch(k) for k in range(n)]
    torch.cuda.synchronize()
    print(f"[bench] drew {n} streams in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    U = sum(x.numel() * x.element_size() for x in streams)
    reps = max(args.steps, 1)
    sh = torch.cuda.current_stream().cuda_stream

    # ---- compression: batched vs one call per stream ---------------------------
    t0 = time.time()
    be = spz.BatchEncoder(streams, args.forecaster, 0)
    print(f"[bench] tuned seg_rows per class {be.tuned} and planned in {time.time() - t0:.1f}s", file=sys.stderr,
          flush=True)
    for _ in range(max(args.warmup, 1)):
        be.run()
    torch.cuda.synchronize()
    ev = _events(reps)
    for a, b in ev:
        a.record()
        be.run()
        b.record()
    torch.cuda.synchronize()
    enc_batch_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    conts = be.containers()
    ok_all = int(be.status.abs().sum().item()) == 0
    enc_per_ms = None
    if not args.batched_only:
        encs = [spz.Encoder.create(x.shape[0], x.shape[1], spz.dtype_code(x), p) for x, p in zip(streams, be.params)]

        def enc_per_stream():
            for e, x in zip(encs, streams):
                e.run(x)
        enc_per_stream()
        torch.cuda.synchronize()
        a, b = _events(1)[0]
        a.record()
        enc_per_stream()
        b.record()
        torch.cuda.synchronize()
        enc_per_ms = a.elapsed_time(b)
        for k in range(0, n, max(1, n // 200)):       # the two forms give the same bytes
            ok_all = ok_all and torch.equal(encs[k].dst[: int(encs[k].out_size.item())], conts[k])
        del encs
    C = sum(c.numel() for c in conts)
    print(f"[bench] encode batched {enc_batch_ms:.2f} ms vs per stream {enc_per_ms} ms", file=sys.stderr,
          flush=True)

    def timed_batch(idx, reps):
        bd = spz.BatchDecoder([conts[k] for k in idx])
        for _ in range(max(args.warmup, 1)):
            bd.run()
        torch.cuda.synchronize()
        ev = _events(reps)
        for a, b in ev:
            a.record()
            bd.run()
            b.record()
        torch.cuda.synchronize()
        ms = [a.elapsed_time(b) for a, b in ev]
        good = int(bd.status.abs().sum().item()) == 0 and all(
            torch.equal(o.view(torch.uint8), streams[k].view(torch.uint8)) for o, k in zip(bd.outs, idx))
        return bd, float(np.mean(ms)), min(ms), good

    allk = list(range(n))
    bd, all_ms, all_best, ok = timed_batch(allk, reps)
    ok_all = ok_all and ok
    # the same call captured once as a HIP graph and replayed
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        bd.run(stream=s)
    g.replay()
    torch.cuda.synchronize()
    ev = _events(reps)
    for a, b in ev:
        a.record()
        g.replay()
        b.record()
    torch.cuda.synchronize()
    graph_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    ok_all = ok_all and all(torch.equal(o.view(torch.uint8), streams[k].view(torch.uint8)) for k, o in enumerate(bd.outs))
    # one launch per stream: eager, and all launches captured in one graph
    st = torch.zeros(n, dtype=torch.int32, device="cuda")

    def per_stream(stream_handle):
        for k in range(n):
            o = bd.outs[k]
            rc = spz.sprintz_decompress(conts[k].data_ptr(), conts[k].numel(), bd.infos[k], o.data_ptr(),
                                        o.numel() * o.element_size(), st[k:k + 1].data_ptr(), stream_handle)
            if rc != spz.SPZ_OK:
                raise spz.SprintzError(rc, "sprintz_decompress")
    per_ms = per_graph_ms = None
    if not args.batched_only:
        per_stream(sh)
        torch.cuda.synchronize()
        a, b = _events(1)[0]
        a.record()
        per_stream(sh)
        b.record()
        torch.cuda.synchronize()
        per_ms = a.elapsed_time(b)
        gp = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gp, stream=s):
            per_stream(s.cuda_stream)
        gp.replay()
        torch.cuda.synchronize()
        ev = _events(3)
        for a, b in ev:
            a.record()
            gp.replay()
            b.record()
        torch.cuda.synchronize()
        per_graph_ms = min(a.elapsed_time(b) for a, b in ev)
        del gp
        ok_all = ok_all and int(st.abs().sum().item()) == 0
        ok_all = ok_all and all(torch.equal(o.view(torch.uint8), streams[k].view(torch.uint8))
                                for k, o in enumerate(bd.outs))
    bd.close()
    del bd, g
    # 16-bit FIRE sub-batch
    k16 = [k for k in allk if streams[k].element_size() == 2]
    U16 = sum(streams[k].numel() * 2 for k in k16)
    C16 = sum(conts[k].numel() for k in k16)
    bd16, ms16, best16, ok16 = timed_batch(k16, reps)
    bd16.close()
    if not (ok_all and ok16):
        print("[bench] PARITY FAILURE (round trip or batched/per-stream bytes)", file=sys.stderr, flush=True)
        sys.exit(1)
    # container bytes of a deterministic sample of streams (every n/40-th, at
    # most 2M samples each) against the CPU oracle's
    parity = 0
    if not args.no_oracle_sample:
        for k in range(0, n, max(1, n // 40)):
            x = streams[k]
            if x.numel() > 2_000_000:
                continue
            S = int.from_bytes(conts[k][24:28].cpu().numpy().tobytes(), "little")
            if conts[k].cpu().numpy().tobytes() != oracle.compress(x.cpu().numpy(), args.forecaster, S):
                print(f"[bench] PARITY FAILURE (container bytes) stream {k}", file=sys.stderr, flush=True)
                sys.exit(1)
            parity += 1
    cpu = None
    if not args.no_cpu_baseline:
        done, secs = 0, 0.0
        for k in range(n):
            if secs > 20.0:
                break
            blob = conts[k].cpu().numpy().tobytes()
            t1 = time.perf_counter()
            oracle.decompress(blob)
            secs += time.perf_counter() - t1
            done += streams[k].numel() * streams[k].element_size()
        cpu = {"value": round(done / secs / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": f"the first streams of the batch up to 20 s of decoding ({done} B)"}
    key16 = f"{n} streams u16 fire sub-batch"
    achieved16 = (U16 + C16) / (ms16 * 1e-3) / 1e9
    out = {
        "metric": "decode GB/s and encode GB/s (uncompressed bytes), % HBM peak, batched vs plain",
        "value": round(U / (all_ms * 1e-3) / 1e9, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": reps,
        "warmup": args.warmup,
        "ms_per_step": round(all_ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8/u16",
        "data": "synthetic",
        "config": {"workload": f"batch of {n} streams: rows log-uniform 1e3..1e6, D in {{1,2,4,8,16}}, "
                               f"int8 walks and uint16 AR(2), {args.forecaster}", "streams": n,
                   "uncompressed_bytes": U, "compressed_bytes": C, "launch": "batched (per-class persistent grids)",
                   "seg_rows_per_class": {f"{8 * (2 if k[0] >= 3 else 1)}bit_D{k[1]}": v
                                          for k, v in sorted(be.tuned.items())},
                   "seg_rows_tuning": "library autotuner (sprintz_autotune) on each class's longest stream"},
        "batch_decode_GBps": round(U / (all_ms * 1e-3) / 1e9, 2),
        "batch_decode_best_ms": round(all_best, 4),
        "graph_replay_ms": round(graph_ms, 4),
        "graph_decode_GBps": round(U / (graph_ms * 1e-3) / 1e9, 2),
        "per_stream_launch_ms": _r(per_ms, 4),
        "per_stream_decode_GBps": _r(per_ms and U / (per_ms * 1e-3) / 1e9, 2),
        "per_stream_graph_ms": _r(per_graph_ms, 4),
        "per_stream_graph_decode_GBps": _r(per_graph_ms and U / (per_graph_ms * 1e-3) / 1e9, 2),
        "batched_vs_per_stream": _r(per_ms and per_ms / all_ms, 2),
        "batched_vs_per_stream_graph": _r(per_graph_ms and per_graph_ms / all_ms, 2),
        "batch_encode_GBps": round(U / (enc_batch_ms * 1e-3) / 1e9, 2),
        "per_stream_encode_GBps": _r(enc_per_ms and U / (enc_per_ms * 1e-3) / 1e9, 2),
        "encode_batched_vs_per_stream": _r(enc_per_ms and enc_per_ms / enc_batch_ms, 2),
        "u16_fire_streams": len(k16),
        "u16_fire_decode_GBps": round(U16 / (ms16 * 1e-3) / 1e9, 2),
        "u16_fire_hbm_frac": round(achieved16 / HBM_PEAK_GBPS, 4),
        "compression_ratio": round(U / C, 4),
        "parity": (f"round trip exact on all {n} streams (batched and graph)" if args.batched_only else
                   f"round trip exact on all {n} streams (batched, graph, per-stream and per-stream graph); "
                   "batched and per-stream compression give equal containers on a sample of 200")
                  + "; " + (f"container bytes equal to the CPU oracle on {parity} sampled streams" if parity
                     else "oracle sample not run here"),
        "roofline": {"bound": "hbm", "kernel": "k_decode_pc_batch", "workload": key16,
                     "achieved": round(achieved16, 2), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved16 / HBM_PEAK_GBPS, 4),
                     "traffic": measured_traffic("k_decode_pc_batch", key16),
                     "algorithmic_bytes_per_launch": U16 + C16},
        "cpu_baseline": cpu,
    }
    return out


def run_latency(args, S=1024):
    """The small stream: 65,536 x 1 int8 random walk (15 % constant runs),
    seed 0, both forecasters. Call latency of compress and decompress (HIP
    events around each call, inputs resident); the container must equal the
    oracle's in the CPU leg."""
    import torch
    import datagen
    import paper_1808_02515_amd as spz

    x_np = datagen.walk_int8(seed=0)
    x = torch.from_numpy(x_np).cuda()
    rows, D = x.shape
    U = x_np.nbytes
    sh = torch.cuda.current_stream().cuda_stream
    res = {}
    for f in ("delta", "fire"):
        enc = spz.Encoder.create(rows, D, spz.SPZ_INT8, spz.make_params(f, S))
        enc.run(x)
        torch.cuda.synchronize()
        csize = int(enc.out_size.item())
        info = spz.info_of(enc.dst[:64])
        y = torch.empty_like(x)
        st = torch.zeros(1, dtype=torch.int32, device="cuda")
        te, td = [], []
        for k in range(max(args.steps, 1) + 5):
            a, b, c = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            a.record()
            enc.run(x)
            b.record()
            rc = spz.sprintz_decompress(enc.dst.data_ptr(), csize, info, y.data_ptr(), U, st.data_ptr(), sh)
            c.record()
            if rc != spz.SPZ_OK:
                raise spz.SprintzError(rc, "sprintz_decompress")
            torch.cuda.synchronize()
            if k >= 5:
                te.append(a.elapsed_time(b) * 1e3)
                td.append(b.elapsed_time(c) * 1e3)
        if not torch.equal(x, y) or int(st.item()) != 0 or int(enc.status.item()) != 0:
            print(f"[bench] PARITY FAILURE latency {f}", file=sys.stderr, flush=True)
            sys.exit(1)
        res[f] = {"decode_us_median": round(float(np.median(td)), 2), "decode_us_best": round(min(td), 2),
                  "encode_us_median": round(float(np.median(te)), 2), "encode_us_best": round(min(te), 2),
                  "ratio": round(U / csize, 4), "container": enc.dst[:csize].cpu().numpy().tobytes()}
    cpu = None
    parity = "decoded samples equal to the input (both forecasters)"
    if not args.no_cpu_baseline:
        import oracle
        secs = []
        for f in ("delta", "fire"):
            t1 = time.perf_counter()
            ref = oracle.compress(x_np, f, S)
            oracle.decompress(ref)
            secs.append(time.perf_counter() - t1)
            if ref != res[f]["container"]:
                print(f"[bench] PARITY FAILURE (latency container bytes, {f})", file=sys.stderr, flush=True)
                sys.exit(1)
        cpu = {"value": round(U / (secs[1] / 2) / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": "the whole 65,536-sample stream, FIRE, encode + decode (rate of one of the two)"}
        parity += "; container bytes equal to the CPU oracle's"
    for f in res:
        del res[f]["container"]
    out = {
        "metric": "decode GB/s and encode GB/s (uncompressed bytes), % HBM peak, batched vs plain",
        "value": round(U / (res["fire"]["decode_us_median"] * 1e-6) / 1e9, 4), "unit": "GB/s", "n_gpus": 1,
        "steps": max(args.steps, 1), "warmup": 5, "ms_per_step": res["fire"]["decode_us_median"] / 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": f"walk_int8 {rows}x{D} seg_rows={S}, call latency"},
        "value_note": "a latency configuration: the call is launch-bound, so the µs figures matter, not %HBM",
        "delta": res["delta"], "fire": res["fire"], "parity": parity, "roofline": None, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def run_huffman(args, rows=1 << 29, D=4, S=2048):
    """The entropy workload: a 4 GiB (2^29 x 4) uint16 series of wrapping
    random walks with rint(Laplace(0, 3)) steps, drawn on the GPU, coded with
    FIRE at seg_rows 2048 without and with the Huffman stage; decode and
    encode speed of both forms (inputs resident in HBM). The CPU leg compares
    sampled segments with the oracle's bytes and times the oracle on them."""
    import torch
    import datagen
    import paper_1808_02515_amd as spz

    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(3)
    t0 = time.time()
    x = datagen.laplace_walk_uint16_torch(rows, D, 3.0, g, dev)
    torch.cuda.synchronize()
    U = x.numel() * 2
    print(f"[bench] drew {rows}x{D} uint16 in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    sh = torch.cuda.current_stream().cuda_stream
    res = {}
    conts = {}
    for ent in (0, 1):
        p = spz.make_params("fire", S, entropy=ent)
        enc = spz.Encoder.create(rows, D, spz.SPZ_UINT16, p, device=dev)
        enc.run(x)
        torch.cuda.synchronize()
        csize = int(enc.out_size.item())
        cont = enc.dst[:csize]
        info = spz.info_of(cont)
        wsz = spz.sprintz_decompress_workspace_size(info)
        ws = torch.empty(max(wsz, 16), dtype=torch.uint8, device=dev)
        y = torch.empty_like(x)
        st = torch.zeros(1, dtype=torch.int32, device=dev)

        def dec():
            rc = spz.sprintz_decompress_ws(cont.data_ptr(), csize, info, y.data_ptr(), U, st.data_ptr(),
                                           ws.data_ptr(), wsz, sh)
            if rc != spz.SPZ_OK:
                raise spz.SprintzError(rc, "sprintz_decompress_ws")
        dec()
        torch.cuda.synchronize()
        ev = _events(2 * max(args.steps, 1))
        for k, (a, b) in enumerate(ev):
            a.record()
            (enc.run(x) if k % 2 == 0 else dec())
            b.record()
        torch.cuda.synchronize()
        te = [a.elapsed_time(b) for k, (a, b) in enumerate(ev) if k % 2 == 0]
        td = [a.elapsed_time(b) for k, (a, b) in enumerate(ev) if k % 2 == 1]
        ok = torch.equal(x, y) and int(st.item()) == 0 and int(enc.status.item()) == 0
        if not ok or int(enc.out_size.item()) != csize:
            print(f"[bench] PARITY FAILURE huffman entropy={ent}", file=sys.stderr, flush=True)
            sys.exit(1)
        name = "huffman" if ent else "plain"
        res[name] = {"compressed_bytes": csize, "ratio": round(U / csize, 4),
                     "decode_GBps": round(U / (np.mean(td) * 1e-3) / 1e9, 2),
                     "encode_GBps": round(U / (np.mean(te) * 1e-3) / 1e9, 2),
                     "decode_ms": round(float(np.mean(td)), 3), "encode_ms": round(float(np.mean(te)), 3),
                     "hbm_frac_decode": round((U + csize) / (np.mean(td) * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)}
        print(f"[bench] {name}: {res[name]}", file=sys.stderr, flush=True)
        conts[name] = cont.cpu().numpy().tobytes() if not args.no_cpu_baseline else None
        del enc, ws, y
        torch.cuda.empty_cache()
    # batched vs one call per stream: the same rows as K streams of rows / K
    # rows, each coded with the Huffman stage; decoded (a) by one batched call
    # (every segment of every stream Huffman-decoded in one launch, then the
    # per-class batched decoder) and (b) by one sprintz_decompress_ws call per
    # stream
    K = args.huffman_streams
    per = rows // K
    parts = [x[k * per:(k + 1) * per] for k in range(K)]
    bconts = [spz.compress(pt, "fire", S, entropy=1) for pt in parts]
    torch.cuda.synchronize()
    bd = spz.BatchDecoder(bconts)
    bd.run()
    torch.cuda.synchronize()
    ev = _events(max(args.steps, 1))
    for a, b in ev:
        a.record()
        bd.run()
        b.record()
    torch.cuda.synchronize()
    bms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    bok = int(bd.status.abs().sum().item()) == 0 and all(
        torch.equal(o.view(torch.uint8), pt.view(torch.uint8)) for o, pt in zip(bd.outs, parts))
    binfos = [spz.info_of(c) for c in bconts]
    bws = [torch.empty(max(spz.sprintz_decompress_workspace_size(i), 16), dtype=torch.uint8, device=dev) for i in binfos]
    bst = torch.zeros(K, dtype=torch.int32, device=dev)

    def per_stream():
        for k in range(K):
            rc = spz.sprintz_decompress_ws(bconts[k].data_ptr(), bconts[k].numel(), binfos[k], bd.outs[k].data_ptr(),
                                           per * D * 2, bst[k:k + 1].data_ptr(), bws[k].data_ptr(), bws[k].numel(), sh)
            if rc != spz.SPZ_OK:
                raise spz.SprintzError(rc, "sprintz_decompress_ws")
    per_stream()
    torch.cuda.synchronize()
    a, b = _events(1)[0]
    a.record()
    per_stream()
    b.record()
    torch.cuda.synchronize()
    pms = a.elapsed_time(b)
    bok = bok and int(bst.abs().sum().item()) == 0 and all(
        torch.equal(o.view(torch.uint8), pt.view(torch.uint8)) for o, pt in zip(bd.outs, parts))
    if not bok:
        print("[bench] PARITY FAILURE huffman batch", file=sys.stderr, flush=True)
        sys.exit(1)
    UB = per * K * D * 2
    CB_ = sum(c.numel() for c in bconts)
    res["huffman_batch"] = {"streams": K, "rows_per_stream": per, "compressed_bytes": CB_,
                            "batched_decode_GBps": round(UB / (bms * 1e-3) / 1e9, 2),
                            "batched_decode_ms": round(bms, 3),
                            "per_stream_decode_GBps": round(UB / (pms * 1e-3) / 1e9, 2),
                            "per_stream_decode_ms": round(pms, 3),
                            "batched_vs_per_stream": round(pms / bms, 2),
                            "hbm_frac_batched": round((UB + CB_) / (bms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)}
    print(f"[bench] huffman batch: {res['huffman_batch']}", file=sys.stderr, flush=True)
    bd.close()
    del bd, bconts, bws, parts
    torch.cuda.empty_cache()
    cpu = None
    parity = ("decoded samples equal to the input (both forms, and every stream of the batched and per-stream "
              "decodes); encode repeatable")
    if not args.no_cpu_baseline:
        # oracle leg: segments 0, nseg/3, 2 nseg/3, last coded alone by the
        # oracle must equal the GPU container's segments; timed as the baseline
        import oracle
        blob = conts["huffman"]
        nseg = int.from_bytes(blob[28:32], "little")
        ds = (64 + 8 * (nseg + 1) + 15) & ~15
        secs, done = 0.0, 0
        for s in sorted({0, nseg // 3, 2 * nseg // 3, nseg - 1}):
            xs = x[s * S:(s + 1) * S].cpu().numpy()
            t1 = time.perf_counter()
            one = oracle.compress(xs, "fire", S, entropy=1)
            oracle.decompress(one)
            secs += time.perf_counter() - t1
            done += xs.nbytes
            a = int.from_bytes(blob[64 + 8 * s:72 + 8 * s], "little")
            b = int.from_bytes(blob[72 + 8 * s:80 + 8 * s], "little")
            ods = (64 + 16 + 15) & ~15
            if blob[ds + a:ds + b] != one[ods:]:
                print(f"[bench] PARITY FAILURE (entropy segment {s} bytes)", file=sys.stderr, flush=True)
                sys.exit(1)
        cpu = {"value": round(done / secs / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": f"4 segments of {S} rows coded and decoded with the entropy stage ({done} B)"}
        parity += "; 4 sampled segments byte-equal to the CPU oracle's"
    out = {
        "metric": "decode GB/s and encode GB/s (uncompressed bytes), % HBM peak, batched vs plain",
        "value": res["huffman"]["decode_GBps"], "unit": "GB/s", "n_gpus": 1, "steps": max(args.steps, 1),
        "warmup": 1, "ms_per_step": res["huffman"]["decode_ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u16", "data": "synthetic",
        "config": {"workload": f"laplace_walk_uint16 {rows}x{D} scale 3 fire seg_rows={S}, Huffman vs plain; "
                               f"the same rows as {args.huffman_streams} Huffman-coded streams, batched vs per stream"},
        "value_note": "decode GB/s of the Huffman-coded form",
        "plain": res["plain"], "huffman": res["huffman"], "huffman_batch": res["huffman_batch"], "parity": parity,
        "roofline": None, "cpu_baseline": cpu,
        "paper_context": "paper Section 5.4: with Huffman coding decompression stays above 500 MB/s (one CPU thread)",
    }
    print(json.dumps(out), flush=True)


def run_dsweep(args, values=100_000_000):
    """Encode and decode speed against D on full-range uniform values (the
    paper's speed workload, Section 5.4: every block needs the full width),
    about 100M values per point, 8- and 16-bit, delta and FIRE, FIRE with
    two-record header groups (the paper's layout) and FIRE with the Huffman
    stage (where its coded segment fits the write pass), one stream per call,
    seg_rows 1024 (2048 where 1024 * D * w/8 is not a multiple of 16). At
    every point the first two segments of the GPU container are compared
    with the CPU oracle's segments of the same rows (segments are coded
    independently, so a prefix of whole segments gives the same bytes)."""
    import torch
    import oracle
    import paper_1808_02515_amd as spz

    def segments(blob: bytes, k: int):
        nseg = int.from_bytes(blob[28:32], "little")
        ds = (64 + 8 * (nseg + 1) + 15) & ~15
        offs = [int.from_bytes(blob[64 + 8 * q:72 + 8 * q], "little") for q in range(min(k, nseg) + 1)]
        return [blob[ds + offs[q]:ds + offs[q + 1]] for q in range(min(k, nseg))]

    res = []
    for w in (8, 16):
        for D in (1, 2, 3, 4, 6, 8, 12, 16, 20, 24, 32, 40, 48, 56, 64, 72, 80):
            rows = values // D
            g = torch.Generator(device="cuda")
            g.manual_seed(D * 100 + w)
            dt = torch.int8 if w == 8 else torch.int16
            x = torch.randint(-(1 << (w - 1)), 1 << (w - 1), (rows, D), generator=g, device="cuda",
                              dtype=torch.int32).to(dt)
            U = x.numel() * x.element_size()
            for f, G, ent in (("delta", 0, 0), ("fire", 0, 0), ("fire", 2, 0), ("fire", 0, 1)):
                S = 1024
                while (S * D * (w // 8)) % 16:
                    S *= 2
                p = spz.make_params(f, S, hdr_group=G, entropy=ent)
                try:
                    enc = spz.Encoder.create(rows, D, spz.dtype_code(x), p)
                    enc.run(x)
                except spz.SprintzError as e:
                    if e.status != spz.SPZ_EUNSUPPORTED:
                        raise
                    continue    # the coded segment does not fit the entropy write pass
                torch.cuda.synchronize()
                csize = int(enc.out_size.item())
                cont = enc.dst[:csize]
                info = spz.info_of(cont)
                wsz = spz.sprintz_decompress_workspace_size(info)
                ws = torch.empty(max(wsz, 16), dtype=torch.uint8, device="cuda")
                y = torch.empty_like(x)
                st = torch.zeros(1, dtype=torch.int32, device="cuda")
                sh = torch.cuda.current_stream().cuda_stream
                def dec():
                    rc = spz.sprintz_decompress_ws(cont.data_ptr(), csize, info, y.data_ptr(), U, st.data_ptr(),
                                                   ws.data_ptr(), wsz, sh)
                    if rc != spz.SPZ_OK:
                        raise spz.SprintzError(rc, "sprintz_decompress_ws")
                dec()
                ev = _events(6)
                for k, (a, b) in enumerate(ev):
                    a.record()
                    (enc.run(x) if k % 2 == 0 else dec())
                    b.record()
                torch.cuda.synchronize()
                te = min(a.elapsed_time(b) for k, (a, b) in enumerate(ev) if k % 2 == 0)
                td = min(a.elapsed_time(b) for k, (a, b) in enumerate(ev) if k % 2 == 1)
                ok = torch.equal(x, y) and int(st.item()) == 0 and int(enc.status.item()) == 0
                variant = "huffman" if ent else ("hdr_group2" if G else "plain")
                # the oracle's bytes for the first two segments' rows
                head = x[: 2 * S].cpu().numpy()
                ref = oracle.compress(head, f, S, G, entropy=ent)
                got = cont[: min(csize, 64 + 8 * 1024 + (4 << 20))].cpu().numpy().tobytes()
                ok = ok and segments(got, 2) == segments(ref, 2)
                if not ok:
                    print(f"[bench] PARITY FAILURE dsweep w={w} D={D} {f} {variant}", file=sys.stderr, flush=True)
                    sys.exit(1)
                res.append({"w": w, "D": D, "forecaster": f, "variant": variant, "seg_rows": S,
                            "ratio": round(U / csize, 4),
                            "decode_GBps": round(U / td * 1e-6, 2), "encode_GBps": round(U / te * 1e-6, 2),
                            "oracle_segments_equal": len(segments(ref, 2))})
                print(f"[bench] w={w} D={D:2d} {f:5s} {variant:10s} decode {res[-1]['decode_GBps']:8.1f} GB/s "
                      f"encode {res[-1]['encode_GBps']:8.1f} GB/s", file=sys.stderr, flush=True)
                del enc, y, cont, ws
            del x
            torch.cuda.empty_cache()
    dec16 = [r["decode_GBps"] for r in res if r["w"] == 16 and r["forecaster"] == "fire" and r["variant"] == "plain"]
    out = {
        "metric": "decode GB/s and encode GB/s (uncompressed bytes), % HBM peak, batched vs plain",
        "value": round(float(np.median(dec16)), 2), "unit": "GB/s", "n_gpus": 1, "steps": 3, "warmup": 1,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8/u16",
        "data": "synthetic",
        "config": {"workload": "D sweep on uniform values (~1e8 values per point), one stream per call"},
        "value_note": "median decode GB/s of the 16-bit plain FIRE points",
        "parity": "round trip exact at every point; the first two segments equal to the CPU oracle's at every point",
        "sweep": res, "roofline": None, "cpu_baseline": None,
        "paper_context": "paper Section 5.4: decompression speed against D on uniform values, single-threaded CPU",
    }
    print(json.dumps(out), flush=True)


def run_serve(args):
    """The serving loop: Poisson arrivals of encode and decode requests of
    log-uniform sizes (4 KB to 64 MB), int8 / uint16, D in 1..16, admitted
    under a 64 GB HBM budget; reports p50 / p99 latency and throughput. The
    payloads come from a pool of 256 series (and their containers) drawn on
    the GPU; every 50th request keeps its result, which is compared with the
    same call made alone."""
    import torch
    import datagen
    import paper_1808_02515_amd as spz
    from paper_1808_02515_amd.serving import Request, Server, latency_stats

    rng = np.random.default_rng(4)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(4)
    pay = []
    for k in range(256):
        size = float(np.exp(rng.uniform(np.log(4096), np.log(64 << 20))))
        D = int(rng.integers(1, 17))
        u16 = k % 2 == 1
        rows = max(8, int(size // (D * (2 if u16 else 1))))
        sigma = float(np.exp(rng.uniform(np.log(0.5), np.log(200.0))))
        x = (datagen.ar2_uint16_torch(rows, D, sigma, 0.2, gen, "cuda") if u16
             else datagen.walk_int8_torch(rows, D, sigma, 0.15, gen, "cuda"))
        S = 1024 if (1024 * D * x.element_size()) % 16 == 0 else 2048
        pay.append((x, spz.compress(x, args.forecaster, S), S))
    torch.cuda.synchronize()
    reqs, t = [], 0.0
    while True:
        t += float(rng.exponential(1.0 / args.rate))
        if t > args.duration:
            break
        k = int(rng.integers(0, len(pay)))
        x, c, S = pay[k]
        if rng.random() < 0.5:
            r = Request(len(reqs), "encode", t, x=x, forecaster=args.forecaster, seg_rows=S)
        else:
            r = Request(len(reqs), "decode", t, container=c, info=spz.info_of(c))
        r.keep = len(reqs) % 50 == 0
        r.payload = k
        reqs.append(r)
    print(f"[bench] serving {len(reqs)} requests over {args.duration}s", file=sys.stderr, flush=True)
    srv = Server(64 << 30, nstreams=4)
    t0 = time.perf_counter()
    done = srv.run(reqs)
    wall = time.perf_counter() - t0
    bad = sum(r.status != 0 for r in done)
    checked = 0
    for r in done:
        if not r.keep:
            continue
        x, c, S = pay[r.payload]
        if r.kind == "encode":
            ok = torch.equal(spz.compress(x, args.forecaster, S), r.result)
        else:
            ok = torch.equal(r.result, x.contiguous().view(torch.uint8).reshape(-1))
        bad += 0 if ok else 1
        checked += 1
    if bad:
        print(f"[bench] PARITY FAILURE in serving ({bad})", file=sys.stderr, flush=True)
        sys.exit(1)
    U = sum(r.nbytes for r in done)
    makespan = max(r.done for r in done)
    lat = latency_stats(done)
    out = {
        "metric": "decode GB/s and encode GB/s (uncompressed bytes), % HBM peak, batched vs plain",
        "value": round(U / makespan / 1e9, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": len(done),
        "warmup": 0,
        "ms_per_step": round(wall / max(len(done), 1) * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8/u16",
        "data": "synthetic",
        "config": {"workload": f"serving: Poisson {args.rate:.0f} req/s for {args.duration}s, 4 KB..64 MB, "
                               f"encode/decode 50/50, int8/uint16, D 1..16, HBM budget 64 GB",
                   "requests": len(done), "streams": 4},
        "throughput_GBps": round(U / makespan / 1e9, 3),
        "offered_GBps": round(U / args.duration / 1e9, 3),
        "latency": lat,
        "latency_encode": latency_stats([r for r in done if r.kind == "encode"]),
        "latency_decode": latency_stats([r for r in done if r.kind == "decode"]),
        "parity": f"{checked} kept results equal to the same call made alone; all device statuses 0",
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

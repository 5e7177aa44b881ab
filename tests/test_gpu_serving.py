"""GPU test of the continuous-batching serving loop: requests that overlap on
the device under a tight HBM budget give, each one, exactly the result it
gives alone (tolerance 0: compressed bytes and decoded samples are equal),
and compressed containers equal the CPU oracle's bytes."""
import sys

import numpy as np
import pytest

import datagen
import oracle
import paper_1808_02515_amd as spz
from paper_1808_02515_amd.serving import Request, Server, latency_stats

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _requests(n=80, seed=4):
    rng = np.random.default_rng(seed)
    out, t = [], 0.0
    for k in range(n):
        D = int(rng.integers(1, 17))
        dt = [np.int8, np.uint16][k % 2]
        rows = int(np.exp(rng.uniform(np.log(8), np.log(40000))))
        x = datagen.ar2_uint16(rows, D, sigma=float(rng.uniform(1, 100)), seed=500 + k).astype(dt)
        S = int(rng.choice([64, 256, 1024]))
        if (S * D * np.dtype(dt).itemsize) % 16:
            S = 1024
        t += float(rng.exponential(1 / 5000.0))           # 5,000 requests per second
        xd = torch.from_numpy(x).cuda()
        if k % 2 == 0:
            out.append(Request(k, "encode", t, x=xd, forecaster=["fire", "delta"][k % 3 == 0], seg_rows=S))
        else:
            c = torch.from_numpy(np.frombuffer(oracle.compress(x, "fire", S), np.uint8).copy()).cuda()
            out.append(Request(k, "decode", t, container=c, info=spz.info_of(c)))
        out[-1].x_np = x
    return out


def test_serving_results_equal_alone_results():
    reqs = _requests()
    need = sorted(r.need_bytes() for r in reqs)
    budget = max(need[-1] * 2, sum(need) // 4)             # not everything fits at once
    _say(f"{len(reqs)} requests, budget {budget} B of {sum(need)} B requested")
    srv = Server(budget, nstreams=4, keep_results=True)
    done = srv.run(reqs)
    assert len(done) == len(reqs)
    assert all(r.status == 0 for r in done)
    _say("latency", latency_stats(done))
    for r in done:
        if r.kind == "encode":
            alone = spz.compress(r.x, r.forecaster, r.seg_rows)
            assert torch.equal(alone, r.result), r.id
            ref = oracle.compress(r.x_np, r.forecaster, r.seg_rows)
            assert r.result.cpu().numpy().tobytes() == ref, r.id
        else:
            alone = spz.decompress(r.container)
            assert torch.equal(alone.view(torch.uint8).reshape(-1), r.result), r.id
            assert np.array_equal(r.result.cpu().numpy().view(r.x_np.dtype).reshape(r.x_np.shape), r.x_np), r.id
    assert srv.pool.used == 0


def test_serving_waits_for_memory():
    # a budget that holds only the largest request: requests run one at a time
    reqs = _requests(n=12, seed=9)
    srv = Server(max(r.need_bytes() for r in reqs) + 64 * 1024, nstreams=2, keep_results=True)
    done = srv.run(reqs, realtime=False)
    assert len(done) == 12 and all(r.status == 0 for r in done)
    for r in done:
        if r.kind == "decode":
            assert np.array_equal(r.result.cpu().numpy().view(r.x_np.dtype).reshape(r.x_np.shape), r.x_np)

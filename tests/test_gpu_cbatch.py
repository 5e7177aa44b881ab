"""Batched compression (sprintz_compress_batch_*): every container of a
mixed batch equals the oracle's bytes (classes coded by the persistent
batched encoder, and series that fall back to one call each), a corrupt-free
status, and replays of a captured HIP graph with eager work in between.
Every call goes through the C ABI."""
import sys

import numpy as np
import pytest

import datagen
import oracle
import paper_1808_02515_amd as spz

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "no GPU"
    spz.load()
    yield


def _mixed(seed: int, n: int):
    """(x, forecaster, seg_rows, hdr_group) of n series: D 1..16 in the
    batched classes plus D = 20 and 64, grouped headers and one-row and empty
    series that take the one-call path."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        D = int(rng.choice([1, 2, 3, 4, 5, 7, 8, 11, 16, 20, 64]))
        rows = int(rng.choice([0, 1, 9, int(rng.integers(10, 5000)), int(rng.integers(5000, 120000))]))
        kind = k % 3
        if kind == 0:
            x = datagen.ar2_uint16(rows, D, sigma=float(rng.uniform(1, 100)), seed=seed * 1000 + k)
        elif kind == 1:
            x = datagen.walk_int8(rows, D, sigma=float(rng.uniform(0.5, 20)), seed=seed * 1000 + k)
        else:
            x = datagen.uniform(rows, D, [np.uint8, np.int16][k % 2], seed=seed * 1000 + k)
        f = ["fire", "delta"][int(rng.integers(0, 2))]
        S = int(rng.choice([8, 64, 256, 1024, 2048]))
        G = 2 if k % 7 == 6 else 0
        out.append((x, f, S, G))
    return out


class _Batch:
    def __init__(self, cases):
        self.cases = cases
        self.xs = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x, _, _, _ in cases]
        n = len(cases)
        self.out = torch.zeros(n, dtype=torch.int64, device="cuda")
        self.status = torch.zeros(n, dtype=torch.int32, device="cuda")
        self.dsts = []
        self.wss = []
        items = []
        for k, ((x, f, S, G), xd) in enumerate(zip(cases, self.xs)):
            rows, D = x.shape
            p = spz.make_params(f, S, G)
            cap = spz.sprintz_compress_bound(rows, D, spz.dtype_code(xd), p)
            d = torch.full((max(cap, 16),), 0xA5, dtype=torch.uint8, device="cuda")
            self.dsts.append(d)
            # every fifth series gets the minimum workspace: one two-pass call inside the batch
            wsz = (spz.sprintz_workspace_size_min if k % 5 == 4 else spz.sprintz_workspace_size)(
                rows, D, spz.dtype_code(xd), p)
            w = torch.empty(max(wsz, 16), dtype=torch.uint8, device="cuda")
            self.wss.append(w)
            items.append(spz.spz_compress_item(xd.data_ptr(), rows, D, spz.dtype_code(xd), p, d.data_ptr(), cap,
                                               self.out.data_ptr() + 8 * k, w.data_ptr(), wsz))
        wsz = spz.sprintz_compress_batch_workspace_size(items)
        assert wsz > 0
        self.ws = torch.empty(wsz + 256, dtype=torch.uint8, device="cuda")
        base = (self.ws.data_ptr() + 255) & ~255
        self.plan = spz.sprintz_compress_batch_create_in(items, base, wsz, torch.cuda.current_stream().cuda_stream)

    def run(self, stream=None):
        s = stream if stream is not None else torch.cuda.current_stream()
        rc = spz.sprintz_compress_batch(self.plan, self.status.data_ptr(), s.cuda_stream)
        assert rc == spz.SPZ_OK, rc

    def check(self, label=""):
        torch.cuda.synchronize()
        assert int(self.status.abs().sum().item()) == 0
        sizes = self.out.cpu().tolist()
        for k, (x, f, S, G) in enumerate(self.cases):
            got = self.dsts[k][: sizes[k]].cpu().numpy().tobytes()
            ref = oracle.compress(x, f, S, G)
            assert got == ref, (label, k, x.shape, x.dtype, f, S, G)

    def close(self):
        spz.sprintz_compress_batch_destroy(self.plan)


def test_compress_batch_equals_oracle():
    cases = _mixed(seed=1, n=40)
    _say(f"case compress batch of {len(cases)} series")
    b = _Batch(cases)
    b.run()
    b.check("eager")
    b.close()


def test_compress_batch_many_small_and_some_large():
    # hundreds of short series of one class fill workgroups together with
    # large ones; two classes of 16-bit FIRE series
    # (first, with the full workspace) 5,001 segments: a series' offset scan
    # takes its sizes in rounds of 2,048
    cases = [(datagen.ar2_uint16(40_000 + 5, 4, seed=900), "delta", 8, 0)]
    for k in range(300):
        cases.append((datagen.ar2_uint16(int(1000 + 37 * k), 8, seed=700 + k), "fire", 1024, 0))
    for k in range(4):
        cases.append((datagen.ar2_uint16(400_000 + 8 * k, 4, seed=800 + k), "fire", 2048, 0))
    _say(f"case compress batch of {len(cases)} series")
    b = _Batch(cases)
    b.run()
    b.check("eager")
    b.close()


def test_compress_batch_graph_replays():
    cases = _mixed(seed=2, n=24)
    b = _Batch(cases)
    b.run()                       # warm up outside the capture
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        b.run(stream=s)
    for rep in range(3):
        for d in b.dsts:
            d.fill_(rep + 1)      # eager work between replays
        b.out.zero_()
        b.status.zero_()
        torch.cuda.synchronize()
        _say(f"case graph replay {rep}")
        g.replay()
        torch.cuda.synchronize()
        b.check(f"replay {rep}")
    b.close()

"""GPU parity of batched decompression (sprintz_batch_*).

Many containers, written by the CPU oracle, decoded in one call: every output
must equal its input exactly, and equal what sprintz_decompress gives for the
same container. Covers batched class shapes (D from 1 to 16, 8- and 16-bit,
both forecasters, several seg_rows in one plan), streams that take the
single-container path inside the same call (D = 20, grouped headers), empty
streams, repeated runs of one plan, corrupt containers, and replays of a
captured HIP graph."""
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


def _streams(seed=0, n=24):
    """(x, forecaster, seg_rows, hdr_group) of a mixed set of streams."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        D = int(rng.integers(1, 17))
        dt = [np.int8, np.uint8, np.int16, np.uint16][k % 4]
        rows = int(rng.integers(0, 5000)) if k % 7 else int(rng.integers(0, 20))
        S = int(rng.choice([16, 64, 256, 1024]))
        if (S * D * np.dtype(dt).itemsize) % 16:
            S = 1024
        x = datagen.ar2_uint16(rows, D, sigma=float(rng.uniform(0.5, 200)), seed=1000 + k).astype(dt)
        out.append((x, ["fire", "delta"][k % 3 == 0], S, 0))
    # single-container path inside the batch call
    out.append((datagen.walk_int8(3001, 20, seed=7), "fire", 1024, 0))
    out.append((datagen.ar2_uint16(2000, 8, seed=8), "fire", 256, 2))
    out.append((np.zeros((0, 4), np.int16), "fire", 1024, 0))
    return out


def _dev(b: bytes):
    return torch.from_numpy(np.frombuffer(b, dtype=np.uint8).copy()).cuda()


def _np(t, dtype):
    return t.cpu().numpy().view(dtype)


def test_batch_matches_inputs_and_single_calls():
    cases = _streams()
    blobs = [oracle.compress(x, f, S, G) for x, f, S, G in cases]
    conts = [_dev(b) for b in blobs]
    _say(f"batch of {len(conts)} streams")
    bd = spz.BatchDecoder(conts)
    for rep in range(2):
        for o in bd.outs:
            if o.numel():
                o.view(torch.uint8).fill_(0x55)
        bd.status.zero_()
        bd.run()
        torch.cuda.synchronize()
        assert int(bd.status.abs().sum().item()) == 0
        for i, (x, f, S, G) in enumerate(cases):
            y = _np(bd.outs[i], x.dtype).reshape(x.shape)
            assert np.array_equal(y, x), (rep, i, x.shape, x.dtype, f, S, G)
    for i, (x, f, S, G) in enumerate(cases):
        if x.size:
            one = spz.decompress(conts[i])
            assert torch.equal(one.view(torch.uint8), bd.outs[i].view(torch.uint8)), i
    bd.close()


def test_batch_many_small_streams_share_groups():
    # 300 short streams of one class: segments of many streams in one workgroup
    xs = [datagen.ar2_uint16(int(r), 2, sigma=30, seed=50 + k)
          for k, r in enumerate(np.random.default_rng(3).integers(8, 700, size=300))]
    conts = [_dev(oracle.compress(x, "fire", 64)) for x in xs]
    bd = spz.BatchDecoder(conts)
    bd.run()
    torch.cuda.synchronize()
    assert int(bd.status.abs().sum().item()) == 0
    for x, o in zip(xs, bd.outs):
        assert np.array_equal(_np(o, x.dtype).reshape(x.shape), x)
    bd.close()


def test_batch_corrupt_stream_is_flagged_and_others_decode():
    xs = [datagen.ar2_uint16(3000, 8, seed=60 + k) for k in range(4)]
    blobs = [bytearray(oracle.compress(x, "fire", 256)) for x in xs]
    ds = (64 + 8 * (int.from_bytes(blobs[1][28:32], "little") + 1) + 15) & ~15
    for p in range(ds + 100, len(blobs[1]), 97):
        blobs[1][p] ^= 0x5A
    conts = [_dev(bytes(b)) for b in blobs]
    guard = 4096
    outs = []
    for x in xs:
        big = torch.full((x.size * 2 + 2 * guard,), 0x77, dtype=torch.uint8, device="cuda")
        outs.append(big)
    views = [o[guard:guard + x.size * 2].view(torch.int16).view(x.shape) for o, x in zip(outs, xs)]
    bd = spz.BatchDecoder(conts, outs=views)
    bd.run()
    torch.cuda.synchronize()
    st = bd.status.cpu().numpy()
    assert st[1] != 0 and st[0] == 0 and st[2] == 0 and st[3] == 0
    for k in (0, 2, 3):
        assert np.array_equal(_np(views[k], np.uint16).reshape(xs[k].shape), xs[k])
    for o in outs:
        g = o.cpu().numpy()
        assert (g[:guard] == 0x77).all() and (g[-guard:] == 0x77).all()
    bd.close()


def test_batch_graph_replays():
    cases = _streams(seed=5, n=12)
    conts = [_dev(oracle.compress(x, f, S, G)) for x, f, S, G in cases]
    bd = spz.BatchDecoder(conts)
    s = torch.cuda.Stream()
    bd.run()           # warm up outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        bd.run(stream=s)
    for rep in range(3):
        for o in bd.outs:
            if o.numel():
                o.view(torch.uint8).fill_(rep + 1)          # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int(bd.status.abs().sum().item()) == 0
        for i, (x, f, S, G) in enumerate(cases):
            assert np.array_equal(_np(bd.outs[i], x.dtype).reshape(x.shape), x), (rep, i)
    bd.close()


def test_batch_large_plan_and_graph_replays():
    # a plan of over 256 MB in two classes (persistent grids that loop over
    # many groups): eager runs and replays of a captured graph are exact
    g = torch.Generator(device="cuda")
    g.manual_seed(11)
    xs = []
    for D in (4, 8):
        steps = torch.randint(-30, 31, (20_000_000 // D * 4, D), generator=g, device="cuda", dtype=torch.int32)
        xs.append((torch.cumsum(steps, 0) & 0xFFFF).to(torch.int32).to(torch.int16).contiguous())
    conts = [spz.compress(x, "fire", 2048) for x in xs]
    assert sum(x.numel() * 2 for x in xs) >= 256 << 20
    bd = spz.BatchDecoder(conts)
    bd.run()
    torch.cuda.synchronize()
    assert int(bd.status.abs().sum().item()) == 0
    for x, o in zip(xs, bd.outs):
        assert torch.equal(o.view(torch.int16), x)
    s = torch.cuda.Stream()
    gr = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gr, stream=s):
        bd.run(stream=s)
    for rep in range(3):
        for o in bd.outs:
            o.view(torch.uint8).fill_(rep + 1)
        torch.cuda.synchronize()
        gr.replay()
        torch.cuda.synchronize()
        assert int(bd.status.abs().sum().item()) == 0
        for x, o in zip(xs, bd.outs):
            assert torch.equal(o.view(torch.int16), x), rep
    bd.close()


def _entropy_cases(seed=21):
    """Entropy-coded oracle containers beside plain ones: batched classes
    (D 1..16, both widths), a single-container one (D = 20) and grouped
    headers; Laplace walks whose codes hit the length limit."""
    rng = np.random.default_rng(seed)
    cases = []
    for k in range(14):
        D = int(rng.choice([1, 2, 4, 8, 16]))
        rows = int(rng.integers(8, 4000))
        if k % 3 == 0:
            x = datagen.laplace_walk_uint16(rows, D, seed=300 + k)
        else:
            x = datagen.ar2_uint16(rows, D, sigma=float(rng.uniform(1, 100)), seed=300 + k).astype(
                [np.int8, np.uint16][k % 2])
        S = 1024 if (1024 * D * x.dtype.itemsize) % 16 == 0 else 2048
        cases.append((x, "fire", S, 0, k % 2))
    cases.append((datagen.walk_int8(1500, 20, seed=9), "fire", 1024, 0, 1))
    cases.append((datagen.ar2_uint16(1200, 8, seed=10), "fire", 256, 2, 1))
    return cases


def test_batch_entropy_coded_containers():
    cases = _entropy_cases()
    blobs = [oracle.compress(x, f, S, G, entropy=e) for x, f, S, G, e in cases]
    conts = [_dev(b) for b in blobs]
    _say(f"batch of {len(conts)} streams, {sum(e for *_, e in cases)} entropy-coded")
    bd = spz.BatchDecoder(conts)
    for rep in range(2):
        for o in bd.outs:
            o.view(torch.uint8).fill_(0x33)
        bd.status.zero_()
        bd.run()
        torch.cuda.synchronize()
        assert int(bd.status.abs().sum().item()) == 0
        for i, (x, f, S, G, e) in enumerate(cases):
            assert np.array_equal(_np(bd.outs[i], x.dtype).reshape(x.shape), x), (rep, i, x.shape, x.dtype, S, G, e)
    # a captured graph of the same call, replayed with eager work between
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        bd.run(stream=s)
    for rep in range(3):
        for o in bd.outs:
            o.view(torch.uint8).fill_(rep + 1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int(bd.status.abs().sum().item()) == 0
        for i, (x, f, S, G, e) in enumerate(cases):
            assert np.array_equal(_np(bd.outs[i], x.dtype).reshape(x.shape), x), ("replay", rep, i)
    bd.close()


def test_batch_corrupt_entropy_container_is_flagged():
    xs = [datagen.laplace_walk_uint16(3000, 4, seed=70 + k) for k in range(3)]
    blobs = [bytearray(oracle.compress(x, "fire", 1024, entropy=1)) for x in xs]
    ds = (64 + 8 * (int.from_bytes(blobs[1][28:32], "little") + 1) + 15) & ~15
    for p in range(ds + 200, len(blobs[1]), 61):
        blobs[1][p] ^= 0xA5
    conts = [_dev(bytes(b)) for b in blobs]
    bd = spz.BatchDecoder(conts)
    bd.run()
    torch.cuda.synchronize()
    st = bd.status.cpu().numpy()
    assert st[1] != 0 and st[0] == 0 and st[2] == 0
    for k in (0, 2):
        assert np.array_equal(_np(bd.outs[k], np.uint16).reshape(xs[k].shape), xs[k])
    bd.close()

"""GPU parity of the entropy stage (Section 4.4's Huffman coding of the
packed bytes; coder and format per reading R19).

Containers coded on the GPU must equal the oracle's byte for byte, and GPU
decoding of oracle-coded containers must return the input exactly. Covers
both widths, delta and FIRE, D from 1 to 16, small and large segments,
grouped headers, all-zero input, the workspace and the stream-ordered
allocation paths, corrupt coded segments and the unsupported cases."""
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


def _dev(b: bytes):
    return torch.from_numpy(np.frombuffer(b, dtype=np.uint8).copy()).cuda()


def _cases():
    rng = np.random.default_rng(31)
    out = []
    for k in range(24):
        D = int(rng.integers(1, 17))
        dt = [np.int8, np.uint16, np.uint8, np.int16][k % 4]
        rows = int(rng.integers(0, 9000))
        S = int(rng.choice([64, 256, 1024, 2048]))
        if (S * D * np.dtype(dt).itemsize) % 16 or S * D * np.dtype(dt).itemsize > 40000:
            S = 256
        sig = float(np.exp(rng.uniform(np.log(0.5), np.log(300))))
        x = datagen.ar2_uint16(rows, D, sigma=sig, seed=100 + k).astype(dt)
        out.append((x, ["fire", "delta"][k % 2], S, [0, 0, 2][k % 3]))
    out.append((np.zeros((5000, 3), np.int16), "fire", 1024, 0))
    out.append((datagen.uniform(4000, 4, np.uint8, seed=2), "delta", 512, 0))
    return out


def test_entropy_compress_matches_oracle_and_decodes():
    for i, (x, f, S, G) in enumerate(_cases()):
        _say(f"entropy case {i} shape={x.shape} dtype={x.dtype} f={f} S={S} G={G}")
        ref = oracle.compress(x, f, S, G, entropy=1)
        got = spz.compress(torch.from_numpy(x).cuda(), f, S, G, entropy=1).cpu().numpy().tobytes()
        assert len(got) == len(ref), (len(got), len(ref))
        if got != ref:
            k = next(j for j in range(len(ref)) if got[j] != ref[j])
            pytest.fail(f"case {i}: first differing byte {k}: gpu {got[k]:#x} oracle {ref[k]:#x}")
        y = spz.decompress(_dev(ref))
        assert np.array_equal(y.cpu().numpy().view(x.dtype), x), i


def test_entropy_large_stream_and_allocating_path():
    x = datagen.ar2_uint16(300000 + 5, 4, sigma=3, seed=7)
    ref = oracle.compress(x, "fire", 2048, entropy=1)
    _say(f"entropy large: {x.nbytes} B -> {len(ref)} B")
    got = spz.compress(torch.from_numpy(x).cuda(), "fire", 2048, entropy=1).cpu().numpy().tobytes()
    assert got == ref
    src = _dev(ref)
    info = spz.info_of(src)
    out = torch.empty(x.shape, dtype=torch.int16, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    # no workspace: the library allocates it on the stream
    rc = spz.sprintz_decompress(src.data_ptr(), src.numel(), info, out.data_ptr(), x.nbytes, st.data_ptr(),
                                torch.cuda.current_stream().cuda_stream)
    assert rc == spz.SPZ_OK
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    assert np.array_equal(out.cpu().numpy().view(np.uint16), x)


def test_entropy_corrupt_segments_flag_status_and_stay_in_bounds():
    x = datagen.ar2_uint16(20000, 4, seed=3)
    ref = bytearray(oracle.compress(x, "fire", 1024, entropy=1))
    info = spz.sprintz_get_info(bytes(ref[:64]))
    wsz = spz.sprintz_decompress_workspace_size(info)
    ds = (64 + 8 * (info.nseg + 1) + 15) & ~15
    rng = np.random.default_rng(8)

    def run(buf):
        src = _dev(bytes(buf))
        guard = 4096
        out = torch.full((info.decompressed_size + 2 * guard,), 0x5A, dtype=torch.uint8, device="cuda")
        ws = torch.full((wsz + 2 * guard,), 0x33, dtype=torch.uint8, device="cuda")
        st = torch.zeros(1, dtype=torch.int32, device="cuda")
        rc = spz.sprintz_decompress_ws(src.data_ptr(), src.numel(), info, out.data_ptr() + guard,
                                       info.decompressed_size, st.data_ptr(), ws.data_ptr() + guard, wsz,
                                       torch.cuda.current_stream().cuda_stream)
        assert rc == spz.SPZ_OK
        torch.cuda.synchronize()
        o, w = out.cpu().numpy(), ws.cpu().numpy()
        assert (o[:guard] == 0x5A).all() and (o[-guard:] == 0x5A).all()
        assert (w[:guard] == 0x33).all() and (w[-guard:] == 0x33).all()
        return int(st.item())

    _say("entropy corrupt: clean")
    assert run(ref) == 0
    bad = bytearray(ref)
    bad[ds + 4 + 10] = 0xFF        # code lengths of 15 bits
    _say("entropy corrupt: lengths")
    assert run(bad) != 0
    bad = bytearray(ref)
    bad[ds:ds + 4] = (1 << 30).to_bytes(4, "little")   # plain size beyond the stride
    _say("entropy corrupt: plain size")
    assert run(bad) != 0
    for k in range(12):
        bad = bytearray(ref)
        for _ in range(6):
            p = int(rng.integers(ds, len(bad)))
            bad[p] = int(rng.integers(0, 256))
        _say(f"entropy corrupt: random #{k}")
        run(bad)


def test_entropy_segments_larger_than_the_write_image():
    # coded segments above the write pass's 60 KiB LDS image are written in
    # place in the container: uniform 16-bit values at D = 16 (about 128 KiB
    # per 4096-row segment), a last segment of 3 rows, and a batch that
    # mixes them with small ones; bytes equal to the oracle's, exact decode
    for rows, D, S in ((8195, 16, 4096), (20000, 3, 16384)):
        x = datagen.uniform(rows, D, np.int16, seed=rows)
        xt = torch.from_numpy(x).cuda()
        _say(f"entropy large segments {rows}x{D} seg_rows={S}")
        got = spz.compress(xt, "fire", S, entropy=1).cpu().numpy().tobytes()
        assert got == oracle.compress(x, "fire", S, entropy=1)
        y = spz.decompress(_dev(got))
        assert torch.equal(y.view(torch.int16), xt)
    c0 = _dev(oracle.compress(datagen.uniform(8195, 16, np.int16, seed=5), "fire", 4096, entropy=1))
    c1 = _dev(oracle.compress(datagen.ar2_uint16(1000, 2, seed=1), "fire", 256, entropy=1))
    bd = spz.BatchDecoder([c0, c1])
    bd.run()
    torch.cuda.synchronize()
    assert int(bd.status.abs().sum().item()) == 0
    assert np.array_equal(bd.outs[0].cpu().numpy().view(np.int16), datagen.uniform(8195, 16, np.int16, seed=5))
    assert np.array_equal(bd.outs[1].cpu().numpy().view(np.uint16), datagen.ar2_uint16(1000, 2, seed=1))
    bd.close()


def test_entropy_length_limited_codes():
    # Laplace-step walks: every segment's byte counts give a Huffman tree
    # deeper than 11, so every code here comes from the halving rule
    x = datagen.laplace_walk_uint16(100000, 4, 3.0, seed=3)
    for f in ("fire", "delta"):
        ref = oracle.compress(x, f, 2048, entropy=1)
        got = spz.compress(torch.from_numpy(x.view(np.int16)).cuda(), f, 2048, entropy=1).cpu().numpy().tobytes()
        # byte 7 holds the dtype code (int16 here, uint16 in the reference)
        assert got[:7] == ref[:7] and got[8:] == ref[8:]
        y = spz.decompress(_dev(ref))
        assert np.array_equal(y.cpu().numpy().view(np.uint16), x)

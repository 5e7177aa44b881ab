"""CPU harness of the decoder kernels (no GPU): the kernels' own source is
built for the host with tests/emu (lanes of a workgroup as coroutines that
meet at barriers, hand-off points and DPP/shuffle operations; every plain
global access checked against the buffers the launch passes) under
AddressSanitizer and UndefinedBehaviorSanitizer, and every workgroup of the
launch the library would make is run.

It covers the one-segment form of the 65,536-sample int8 walk, the case kept
off the GPU (test_gpu_parity.py): the current decoder decodes it exactly with
no access outside its buffers. It also decodes a random corpus of oracle
containers (every decoder: the pipelined form for D = 7..16 and the
producer/consumer form for smaller D in the single-container kernel, the
batched kernel's producer/consumer form for every D <= 16, the walker for
grouped headers and D up to 80) and corrupted containers, which may only
change samples or set the status word."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import datagen
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EMU = os.path.join(ROOT, "tests", "emu")
CSRC = os.path.join(ROOT, "paper_1808_02515_amd", "csrc")


def _clang():
    for c in ("/opt/rocm/llvm/bin/clang++", shutil.which("clang++")):
        if c and os.path.exists(c):
            return c
    return None


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    cc = _clang()
    if cc is None:
        pytest.skip("no clang++ for the host build of the kernels")
    out = str(tmp_path_factory.mktemp("emu") / "emu_decode")
    subprocess.run([cc, "-std=c++17", "-O2", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    "-fno-omit-frame-pointer", "-I", EMU, "-I", CSRC, "-o", out, os.path.join(EMU, "emu_decode.cpp")],
                   check=True, timeout=600)
    return out


def _decode(harness, blob: bytes, tmp, shape, dtype, batch=False):
    c, o = os.path.join(tmp, "c.bin"), os.path.join(tmp, "o.bin")
    with open(c, "wb") as fh:
        fh.write(blob)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    r = subprocess.run([harness, c, o] + (["batch"] if batch else []), capture_output=True, text=True, timeout=600,
                       env=env)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-2000:]
    fields = dict(kv.split("=") for kv in r.stdout.split())
    y = np.fromfile(o, dtype=dtype).reshape(shape)
    return int(fields["status"]), int(fields["violations"]), y


@pytest.mark.parametrize("f", ["delta", "fire"])
def test_one_segment_walk_in_bounds(harness, tmp_path, f):
    # 65,536 x 1 int8 walk as one segment: one workgroup walks 1,024 chunks
    x = datagen.walk_int8()
    st, viol, y = _decode(harness, oracle.compress(x, f, 65536), str(tmp_path), x.shape, x.dtype)
    assert (st, viol) == (0, 0)
    assert np.array_equal(y, x)


def test_corpus_decodes_exactly_in_bounds(harness, tmp_path):
    rng = np.random.default_rng(0)
    for k in range(40):
        D = int(rng.choice([1, 2, 3, 4, 5, 8, 16, 20, 80]))
        rows = int(rng.choice([0, 1, 7, 8, 9, 100, 1000, 3000]))
        dt = [np.int8, np.uint16][k % 2]
        x = datagen.ar2_uint16(rows, D, sigma=float(rng.uniform(1, 100)), seed=k).astype(dt)
        f = ["fire", "delta"][k % 3 % 2]
        S = int(rng.choice([8, 64, 256, 1024]))
        G = [0, 0, 2][k % 3]
        blob = oracle.compress(x, f, S, G)
        # D <= 16 without header groups also through the batched kernel
        for batch in (False, True) if D <= 16 and G == 0 else (False,):
            st, viol, y = _decode(harness, blob, str(tmp_path), x.shape, x.dtype, batch)
            assert (st, viol) == (0, 0), (k, D, rows, dt, f, S, G, batch)
            assert np.array_equal(y, x), (k, D, rows, dt, f, S, G, batch)


def test_corrupted_containers_stay_in_bounds(harness, tmp_path):
    rng = np.random.default_rng(1)
    flagged = 0
    for k in range(60):
        D = int(rng.choice([1, 3, 8, 16, 20]))
        x = datagen.ar2_uint16(3000, D, seed=k).astype([np.int8, np.uint16][k % 2])
        S = int(rng.choice([64, 256, 1024]))
        blob = bytearray(oracle.compress(x, ["fire", "delta"][k % 2], S, [0, 0, 1][k % 3]))
        nseg = int.from_bytes(blob[28:32], "little")
        ds = (64 + 8 * (nseg + 1) + 15) & ~15
        for _ in range(int(rng.integers(1, 6))):
            p = int(rng.integers(64 if k % 4 == 0 else ds, len(blob)))   # offset table too, every fourth case
            blob[p] = int(rng.integers(0, 256))
        st, viol, _ = _decode(harness, bytes(blob), str(tmp_path), x.shape, x.dtype)
        assert viol == 0, k
        flagged += st != 0
        if D <= 16:
            _, viol, _ = _decode(harness, bytes(blob), str(tmp_path), x.shape, x.dtype, True)
            assert viol == 0, (k, "batch")
    assert flagged > 0

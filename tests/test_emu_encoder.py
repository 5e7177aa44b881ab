"""CPU harness of the single-pass encoder (no GPU): the source of
k_encode_sp, k_enc_scan and k_enc_compact is built for the host with
tests/emu (lanes of a workgroup as coroutines that meet at barriers,
wave-local syncs and DPP/shuffle operations; buffer resources and plain
global accesses checked against the buffers of the launch) under
AddressSanitizer and UndefinedBehaviorSanitizer. Every workgroup of the
launch the library makes is run, the workspace starts as garbage, and the
container must equal the oracle's bytes with no access outside the buffers.

Shapes stay small (a few seconds each): the emulated lanes run one at a
time."""
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
_CODE = {np.dtype(np.int8): 1, np.dtype(np.uint8): 2, np.dtype(np.int16): 3, np.dtype(np.uint16): 4}


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
    out = str(tmp_path_factory.mktemp("emu") / "emu_encode")
    subprocess.run([cc, "-std=c++17", "-O2", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    "-fno-omit-frame-pointer", "-I", EMU, "-I", CSRC, "-o", out, os.path.join(EMU, "emu_encode.cpp")],
                   check=True, timeout=600)
    return out


def _encode(harness, x: np.ndarray, f: str, S: int, ls: int, tmp):
    x = np.ascontiguousarray(x)
    i, o = os.path.join(tmp, "x.bin"), os.path.join(tmp, "c.bin")
    x.tofile(i)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    r = subprocess.run([harness, i, str(x.shape[0]), str(x.shape[1]), str(_CODE[x.dtype]), str(int(f == "fire")),
                        str(S), str(ls), o], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-2000:]
    fields = dict(kv.split("=") for kv in r.stdout.split())
    with open(o, "rb") as fh:
        blob = fh.read()
    return int(fields["status"]), int(fields["violations"]), blob


@pytest.mark.parametrize("x,f,S", [
    (datagen.ar2_uint16(20003, 8, seed=1), "fire", 1024),            # many segments, ragged tail
    (datagen.walk_int8(5003, 1, seed=2), "fire", 512),
    (datagen.ar2_uint16(3003, 3, seed=3).astype(np.int8), "delta", 64),
    (datagen.uniform(1000, 16, np.uint16, seed=4), "fire", 256),     # incompressible: full-width blocks
    (np.zeros((8 * 700 + 3, 1), np.uint8), "delta", 8192),           # one long zero run, split records
    (datagen.uniform(7, 2, np.int16, seed=5), "fire", 8),            # tail only
], ids=["u16-D8-fire", "i8-D1-fire", "i8-D3-delta", "u16-D16-noise", "u8-zero-run", "i16-tail-only"])
def test_encoder_matches_oracle_in_bounds(harness, tmp_path, x, f, S):
    st, viol, blob = _encode(harness, x, f, S, 1, str(tmp_path))
    assert (st, viol) == (0, 0)
    assert blob == oracle.compress(x, f, S)


def test_encoder_corpus(harness, tmp_path):
    rng = np.random.default_rng(7)
    for k in range(16):
        D = int(rng.choice([1, 2, 3, 8, 16]))
        rows = int(rng.choice([0, 1, 8, 9, 100, 777, 2000]))
        dt = [np.int8, np.uint8, np.int16, np.uint16][k % 4]
        x = datagen.ar2_uint16(rows, D, sigma=float(rng.uniform(1, 100)), seed=100 + k).astype(dt)
        if k % 5 == 4:
            x[: rows // 2] = 0                                      # runs of zero blocks into data
        f = ["fire", "delta"][k % 2]
        S = int(rng.choice([8, 64, 256, 1024]))
        ls = int(rng.choice([0, 1, 3]))
        st, viol, blob = _encode(harness, x, f, S, ls, str(tmp_path))
        assert (st, viol) == (0, 0), (k, D, rows, dt, f, S, ls)
        assert blob == oracle.compress(x, f, S, learn_shift=ls), (k, D, rows, dt, f, S, ls)

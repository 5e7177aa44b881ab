"""sprintz_compress_noalloc (the entry point for callers that cannot
allocate) against sprintz_compress with a caller workspace: the same container
bytes and sizes, on two calls in a row (the second with a smaller input, so
the static workspace still holds the first call's contents), plus the oracle's
bytes for both inputs and the host-side size limit. Every call goes through
the C ABI."""
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


def _dtype_code(x):
    return spz.SPZ_UINT16 if x.dtype == np.uint16 else spz.SPZ_INT8


def _compress_ws(xd, rows, D, code, p):
    """The existing entry point, with a workspace allocated here."""
    cap = spz.sprintz_compress_bound(rows, D, code, p)
    wsz = spz.sprintz_workspace_size(rows, D, code, p)
    dst = torch.zeros(cap, dtype=torch.uint8, device="cuda")
    ws = torch.empty(max(wsz, 8), dtype=torch.uint8, device="cuda")
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    rc = spz.sprintz_compress(xd.data_ptr(), rows, D, code, p, dst.data_ptr(), cap, out.data_ptr(), ws.data_ptr(),
                              ws.numel(), st.data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert rc == spz.SPZ_OK, rc
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    return dst[: int(out.item())].cpu().numpy().tobytes()


def _compress_noalloc(xd, rows, D, code, p):
    cap = spz.sprintz_compress_bound(rows, D, code, p)
    # a destination filled with garbage: every container byte must be written
    dst = torch.full((cap,), 0xA5, dtype=torch.uint8, device="cuda")
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    rc = spz.sprintz_compress_noalloc(xd.data_ptr(), rows, D, code, p, dst.data_ptr(), cap, out.data_ptr(),
                                      st.data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert rc == spz.SPZ_OK, rc
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    return dst[: int(out.item())].cpu().numpy().tobytes()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "no GPU"
    spz.load()
    yield


@pytest.mark.parametrize("f", ["fire", "delta"])
def test_noalloc_equals_workspace_form_twice(f):
    # first call: 600,003 x 8 uint16 rows, whose single-pass workspace does
    # not fit the static array (the two-pass encoder runs); then 131,075 x 8
    # (129 segments, single pass) and a smaller int8 stream over fewer
    # segments, each call smaller than the one before
    big = datagen.ar2_uint16(600003, 8, seed=10)
    p_big = spz.make_params(f, 1024)
    assert spz.sprintz_workspace_size(600003, 8, spz.SPZ_UINT16, p_big) > spz.NOALLOC_WORKSPACE_BYTES
    assert spz.sprintz_workspace_size(131075, 8, spz.SPZ_UINT16, p_big) <= spz.NOALLOC_WORKSPACE_BYTES
    cases = [(big, 1024), (datagen.ar2_uint16(131075, 8, seed=11), 1024), (datagen.walk_int8(20003, 1, seed=12), 512)]
    for x, S in cases:
        rows, D = x.shape
        code = _dtype_code(x)
        p = spz.make_params(f, S)
        _say(f"case noalloc f={f} shape={x.shape} dtype={x.dtype} S={S}")
        xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
        ref = _compress_ws(xd, rows, D, code, p)
        got = _compress_noalloc(xd, rows, D, code, p)
        assert len(got) == len(ref), (len(got), len(ref))
        assert got == ref
        assert got == oracle.compress(x, f, S)


def test_noalloc_refuses_more_segments_than_its_workspace():
    # 8 bytes per segment plus 8: 524,288 segments of 8 rows need 4 MiB + 8;
    # refused on the host (the pointers are never dereferenced)
    p = spz.make_params("fire", 8)
    rows = 524288 * 8
    assert spz.sprintz_workspace_size_min(rows, 1, spz.SPZ_INT8, p) > spz.NOALLOC_WORKSPACE_BYTES
    fake = 1 << 20
    rc = spz.sprintz_compress_noalloc(fake, rows, 1, spz.SPZ_INT8, p, fake, 1 << 40, fake, 0, 0)
    assert rc == spz.SPZ_ENOSPC
    # one segment fewer fits
    assert spz.sprintz_workspace_size_min(rows - 8, 1, spz.SPZ_INT8, p) <= spz.NOALLOC_WORKSPACE_BYTES

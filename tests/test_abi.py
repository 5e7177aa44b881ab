"""CPU checks of the C ABI: the library loads, exports every entry point that
include/sprintz.h declares, and its host-only logic (parameters, bounds,
header parsing, argument validation) behaves. No kernel is launched."""
import ctypes
import os
import re

import numpy as np
import pytest

import datagen
import oracle
import paper_1808_02515_amd as spz
from paper_1808_02515_amd import build as spz_build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(spz.LIB_PATH):
        spz_build.build()
    return spz.load()


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "sprintz.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b((?:sprintz|spz)_\w+)\s*\(", text)))


def test_header_declares_the_abi():
    names = _declared_functions()
    for n in ["sprintz_compress", "sprintz_decompress", "sprintz_get_info", "sprintz_compress_bound",
              "sprintz_workspace_size", "spz_params_default", "sprintz_strerror", "sprintz_format_version"]:
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for n in _declared_functions():
        assert hasattr(lib, n), n
        assert n in spz._SIGNATURES, n


def test_params_default(lib):
    p = spz.spz_params_default()
    assert p.struct_size == ctypes.sizeof(spz.spz_params)
    assert (p.forecaster, p.seg_rows, p.hdr_group, p.learn_shift, p.entropy) == (spz.SPZ_FIRE, 1024, 0, 1, 0)
    assert spz.sprintz_format_version() == 1
    assert spz.sprintz_strerror(spz.SPZ_ECORRUPT)


@pytest.mark.parametrize("dt,code", [(np.int8, 1), (np.uint16, 4)])
def test_bound_matches_oracle_bound(lib, dt, code):
    # two separately written bound formulas agree, and real output fits
    for rows, D, S, G in [(0, 3, 8, 0), (7, 1, 8, 0), (65536, 1, 1024, 0), (100003, 8, 512, 2), (1000, 64, 64, 1)]:
        p = spz.make_params("fire", S, G)
        assert spz.sprintz_compress_bound(rows, D, code, p) == oracle.compress_bound(rows, D, dt, S, G)
        nseg = -(-rows // S)
        assert spz.sprintz_workspace_size_min(rows, D, code, p) == 8 * nseg + 8
        ws = spz.sprintz_workspace_size(rows, D, code, p)
        if G == 0 and D <= 16:
            # the single-pass encoder: a slot of at least the segment's bound per segment
            one = oracle.compress_bound(min(rows, S), D, dt, S, G) - oracle.compress_bound(0, D, dt, S, G)
            assert ws >= nseg * one + 16 * nseg
        else:
            assert ws == 8 * nseg + 8


def test_get_info_parses_oracle_container(lib):
    x = datagen.ar2_uint16(1000, 5, seed=2)
    b = oracle.compress(x, "delta", seg_rows=64, hdr_group=2, learn_shift=2)
    info = spz.sprintz_get_info(b[:64])
    assert (info.rows, info.D, info.dtype, info.w, info.nseg) == (1000, 5, spz.SPZ_UINT16, 16, 16)
    assert (info.params.forecaster, info.params.seg_rows, info.params.hdr_group, info.params.learn_shift) == (0, 64, 2, 2)
    assert info.compressed_size == len(b)
    assert info.decompressed_size == x.nbytes
    bad = bytearray(b[:64])
    bad[0] ^= 1
    with pytest.raises(spz.SprintzError):
        spz.sprintz_get_info(bytes(bad))
    bad = bytearray(b[:64])
    bad[28] += 1  # segment count inconsistent with rows / seg_rows
    with pytest.raises(spz.SprintzError):
        spz.sprintz_get_info(bytes(bad))


def test_argument_validation_without_gpu(lib):
    # every call below is rejected on the host before any HIP call
    p = spz.make_params("fire", 1024)
    fake = 1 << 20  # never dereferenced
    assert spz.sprintz_compress(fake, 100, 0, 4, p, fake, 1 << 20, fake, fake, 1 << 10, 0, 0) == spz.SPZ_EINVAL
    assert spz.sprintz_compress(fake, 100, 3, 9, p, fake, 1 << 20, fake, fake, 1 << 10, 0, 0) == spz.SPZ_EINVAL
    assert spz.sprintz_compress(fake, 100, 129, 4, p, fake, 1 << 20, fake, fake, 1 << 10, 0, 0) == spz.SPZ_EUNSUPPORTED
    assert spz.sprintz_compress(fake, 100, 3, 4, p, fake, 10, fake, fake, 1 << 10, 0, 0) == spz.SPZ_ENOSPC
    assert spz.sprintz_compress(fake, 100, 3, 4, p, fake, 1 << 20, fake, fake, 0, 0, 0) == spz.SPZ_ENOSPC
    assert spz.sprintz_compress(fake, 100, 3, 4, p, fake + 8, 1 << 20, fake, fake, 1 << 10, 0, 0) == spz.SPZ_EINVAL
    for bad in [spz.make_params("fire", 12), spz.make_params("fire", 4), spz.make_params("fire", 1024, 256),
                spz.make_params("fire", 1024, 0, 9)]:
        assert spz.sprintz_compress(fake, 100, 3, 4, bad, fake, 1 << 20, fake, fake, 1 << 10, 0, 0) == spz.SPZ_EINVAL
    info = spz.sprintz_get_info(oracle.compress(np.zeros((16, 2), np.int8), "fire", 8)[:64])
    assert spz.sprintz_decompress(fake, 10, info, fake, 1 << 20, 0, 0) == spz.SPZ_ENOSPC
    assert spz.sprintz_decompress(fake, 1 << 20, info, fake, 3, 0, 0) == spz.SPZ_ENOSPC
    assert spz.sprintz_decompress(fake + 4, 1 << 20, info, fake, 1 << 20, 0, 0) == spz.SPZ_EINVAL


def test_header_sizes_that_wrap_are_rejected(lib):
    # a data_bytes near 2^64 would make data_start + data_bytes wrap, so the
    # container would look smaller than the buffer while its offset table
    # could point anywhere; get_info must refuse it before any launch
    b = bytearray(oracle.compress(datagen.ar2_uint16(1000, 3, seed=5), "fire", seg_rows=256)[:64])
    good = spz.sprintz_get_info(bytes(b))
    for data_bytes in [2**64 - 16, 2**64 - 96]:   # data start is 112 here
        bad = bytearray(b)
        bad[32:40] = data_bytes.to_bytes(8, "little")
        with pytest.raises(spz.SprintzError):
            spz.sprintz_get_info(bytes(bad))
    bad = bytearray(b)
    bad[32:40] = (int.from_bytes(b[32:40], "little") + 8).to_bytes(8, "little")  # not a multiple of 16
    with pytest.raises(spz.SprintzError):
        spz.sprintz_get_info(bytes(bad))
    # rows * D * bytes that wraps: D near 2^32 with a segment count that is
    # consistent with rows and seg_rows
    bad = bytearray(b)
    rows = 2**33
    bad[12:16] = (2**32 - 1).to_bytes(4, "little")
    bad[16:24] = rows.to_bytes(8, "little")
    bad[24:28] = (2**20).to_bytes(4, "little")
    bad[28:32] = (rows // 2**20).to_bytes(4, "little")
    bad[32:40] = (0).to_bytes(8, "little")
    with pytest.raises(spz.SprintzError):
        spz.sprintz_get_info(bytes(bad))
    # a hand-made info whose container size lies below the data start is
    # refused by the decoder's host check
    fake = 1 << 20  # never dereferenced
    info = spz.spz_info.from_buffer_copy(good)
    info.compressed_size = 16
    assert spz.sprintz_decompress(fake, 1 << 20, info, fake, 1 << 20, 0, 0) == spz.SPZ_EINVAL


def _tune_candidates(rows):
    ref = min(1 << 20, (max(rows, 8) + 7) // 8 * 8)
    return [ref] + [S for S in (256, 512, 1024, 2048, 4096) if S < ref]


@pytest.mark.parametrize("dt,code", [(np.int8, 1), (np.uint16, 4)])
def test_autotuned_sizes_hold_for_every_candidate(lib, dt, code):
    # seg_rows 0: bound and workspaces are the largest over the segment sizes
    # the autotuner may choose
    for rows, D in [(0, 3), (5, 1), (300, 2), (70000, 8), (3_000_000, 4)]:
        for G in (0, 2):
            p0 = spz.make_params("fire", 0, G)
            cands = _tune_candidates(rows)
            for fn in (spz.sprintz_compress_bound, spz.sprintz_workspace_size, spz.sprintz_workspace_size_min):
                assert fn(rows, D, code, p0) == max(fn(rows, D, code, spz.make_params("fire", S, G)) for S in cands)
            assert spz.sprintz_compress_bound(rows, D, code, p0) == max(
                oracle.compress_bound(rows, D, dt, S, G) for S in cands)


def test_noalloc_refuses_autotuned_segments(lib):
    fake = 1 << 20  # never dereferenced: refused before any HIP call
    p = spz.make_params("fire", 0)
    assert spz.sprintz_compress_noalloc(fake, 1000, 2, spz.SPZ_UINT16, p, fake, 1 << 20, fake, 0, 0) == spz.SPZ_EINVAL

"""CPU oracle of the Sprintz codec -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The GPU library never calls it and shares
no code with it.

Two independent implementations live here, both written from the paper
(Blalock, Madden & Guttag, "Sprintz", IMWUT 2018, Sections 4.1-4.3 and
Algorithms 1-3):

* ``sprintz_oracle.c`` -- plain scalar C, one bit at a time, loaded through
  ctypes (this module). It is fast enough to run the benchmark workloads.
* ``tiny.py`` -- a pure-Python twin for tiny inputs, used to cross-check the C
  code byte for byte.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sprintz_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle_sprintz.so")
_lib = None

DTYPE_CODE = {np.dtype(np.int8): 1, np.dtype(np.uint8): 2, np.dtype(np.int16): 3, np.dtype(np.uint16): 4}
CODE_DTYPE = {v: k for k, v in DTYPE_CODE.items()}
FORECASTERS = {"delta": 0, "fire": 1}

ERRORS = {0: "ok", -1: "invalid argument", -2: "no space", -3: "corrupt", -6: "no memory"}


class OracleError(RuntimeError):
    def __init__(self, rc: int):
        super().__init__(f"oracle error {rc}: {ERRORS.get(rc, 'unknown')}")
        self.rc = rc


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc into ``liboracle_sprintz.so``."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    u64, u32, sz, vp = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_size_t, ctypes.c_void_p
    lib.oracle_compress.argtypes = [vp, u64, u32, ctypes.c_int, ctypes.c_int, u32, ctypes.c_int, ctypes.c_int,
                                    vp, sz, ctypes.POINTER(sz)]
    lib.oracle_compress.restype = ctypes.c_int
    lib.oracle_decompress.argtypes = [vp, sz, vp, sz]
    lib.oracle_decompress.restype = ctypes.c_int
    lib.oracle_info.argtypes = [vp, sz, ctypes.POINTER(u64), ctypes.POINTER(u32), ctypes.POINTER(ctypes.c_int),
                                ctypes.POINTER(u64)]
    lib.oracle_info.restype = ctypes.c_int
    lib.oracle_compress_bound.argtypes = [u64, u32, ctypes.c_int, u32, ctypes.c_int]
    lib.oracle_compress_bound.restype = sz
    lib.oracle_residuals.argtypes = [vp, u64, u32, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int64, vp, vp]
    lib.oracle_residuals.restype = ctypes.c_int
    lib.oracle_zigzag.argtypes = [ctypes.c_int64]
    lib.oracle_zigzag.restype = u32
    lib.oracle_unzigzag.argtypes = [u32]
    lib.oracle_unzigzag.restype = ctypes.c_int64
    lib.oracle_required_bits.argtypes = [u32]
    lib.oracle_required_bits.restype = ctypes.c_int
    lib.oracle_code_of_nbits.argtypes = [ctypes.c_int, ctypes.c_int]
    lib.oracle_code_of_nbits.restype = ctypes.c_int
    lib.oracle_width_of_code.argtypes = [ctypes.c_int, ctypes.c_int]
    lib.oracle_width_of_code.restype = ctypes.c_int
    lib.oracle_huff_lengths.argtypes = [vp, vp]
    lib.oracle_huff_lengths.restype = ctypes.c_int
    lib.oracle_entropy_bound.argtypes = [vp, sz]
    lib.oracle_entropy_bound.restype = sz
    lib.oracle_entropy_encode.argtypes = [vp, sz, vp, sz, ctypes.POINTER(sz)]
    lib.oracle_entropy_encode.restype = ctypes.c_int
    lib.oracle_entropy_decode.argtypes = [vp, sz, vp, sz, ctypes.POINTER(sz)]
    lib.oracle_entropy_decode.restype = ctypes.c_int
    lib.oracle_entropy_plain_size.argtypes = [vp, sz]
    lib.oracle_entropy_plain_size.restype = sz
    lib.oracle_huff_encode_segment.argtypes = [vp, sz, vp, sz]
    lib.oracle_huff_encode_segment.restype = sz
    lib.oracle_huff_decode_segment.argtypes = [vp, sz, vp, sz, ctypes.POINTER(sz)]
    lib.oracle_huff_decode_segment.restype = ctypes.c_int
    _lib = lib
    return lib


def lib():
    return _load()


def _as_2d(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x)
    if x.ndim == 1:
        x = x.reshape(-1, 1)
    if x.ndim != 2 or x.dtype not in DTYPE_CODE:
        raise ValueError("expected a (rows, D) int8/uint8/int16/uint16 array")
    return x


def compress_bound(rows: int, D: int, dtype, seg_rows: int, hdr_group: int = 0) -> int:
    return int(_load().oracle_compress_bound(rows, D, DTYPE_CODE[np.dtype(dtype)], seg_rows, hdr_group))


def compress(x: np.ndarray, forecaster: str = "fire", seg_rows: int | None = None, hdr_group: int = 0,
             learn_shift: int = 1, entropy: int = 0) -> bytes:
    """Compress a (rows, D) array. ``seg_rows=None`` codes the whole series as
    one segment (the paper's single stream). ``entropy=1`` adds the Huffman
    stage to every segment."""
    x = _as_2d(x)
    rows, D = x.shape
    if seg_rows is None:
        seg_rows = max(8, ((rows + 7) // 8) * 8)
    cap = compress_bound(rows, D, x.dtype, seg_rows, hdr_group)
    out = np.zeros(max(cap, 1), dtype=np.uint8)
    size = ctypes.c_size_t(0)
    rc = _load().oracle_compress(x.ctypes.data, rows, D, DTYPE_CODE[x.dtype], FORECASTERS[forecaster], seg_rows,
                                 hdr_group, learn_shift, out.ctypes.data, cap, ctypes.byref(size))
    if rc != 0:
        raise OracleError(rc)
    plain = out[: size.value].tobytes()
    return entropy_encode(plain) if entropy else plain


def entropy_encode(plain: bytes) -> bytes:
    """Plain container -> Huffman-coded container (Section 4.4's entropy stage)."""
    src = np.frombuffer(plain, dtype=np.uint8)
    cap = int(_load().oracle_entropy_bound(src.ctypes.data, len(plain)))
    if cap == 0:
        raise OracleError(-1)
    out = np.zeros(cap, dtype=np.uint8)
    size = ctypes.c_size_t(0)
    rc = _load().oracle_entropy_encode(src.ctypes.data, len(plain), out.ctypes.data, cap, ctypes.byref(size))
    if rc != 0:
        raise OracleError(rc)
    return out[: size.value].tobytes()


def entropy_decode(coded: bytes) -> bytes:
    """Huffman-coded container -> the plain container it was made from."""
    src = np.frombuffer(coded, dtype=np.uint8)
    cap = int(_load().oracle_entropy_plain_size(src.ctypes.data, len(coded)))
    if cap == 0:
        raise OracleError(-3)
    out = np.zeros(cap, dtype=np.uint8)
    size = ctypes.c_size_t(0)
    rc = _load().oracle_entropy_decode(src.ctypes.data, len(coded), out.ctypes.data, cap, ctypes.byref(size))
    if rc != 0:
        raise OracleError(rc)
    return out[: size.value].tobytes()


def huff_lengths(counts) -> np.ndarray:
    """Code lengths (0 = absent) the entropy stage gives 256 byte counts."""
    c = np.ascontiguousarray(np.asarray(counts, dtype=np.uint64))
    assert c.shape == (256,)
    out = np.zeros(256, dtype=np.uint8)
    rc = _load().oracle_huff_lengths(c.ctypes.data, out.ctypes.data)
    if rc != 0:
        raise OracleError(rc)
    return out


def huff_encode_segment(plain: bytes) -> bytes:
    """Entropy-code one plain segment (length a multiple of 16)."""
    src = np.frombuffer(plain, dtype=np.uint8)
    cap = 4 + 128 + 64 + (len(plain) * 11 + 7) // 8 + 16 + 16
    out = np.zeros(cap, dtype=np.uint8)
    n = int(_load().oracle_huff_encode_segment(src.ctypes.data, len(plain), out.ctypes.data, cap))
    if n == 0:
        raise OracleError(-1)
    return out[:n].tobytes()


def huff_decode_segment(seg: bytes, cap: int) -> bytes:
    src = np.frombuffer(seg, dtype=np.uint8)
    out = np.zeros(max(cap, 1), dtype=np.uint8)
    n = ctypes.c_size_t(0)
    rc = _load().oracle_huff_decode_segment(src.ctypes.data, len(seg), out.ctypes.data, cap, ctypes.byref(n))
    if rc != 0:
        raise OracleError(rc)
    return out[: n.value].tobytes()


def info(buf: bytes) -> tuple[int, int, np.dtype, int]:
    """(rows, D, dtype, total container bytes) from a container header."""
    src = np.frombuffer(buf, dtype=np.uint8)
    rows, D, dt, total = ctypes.c_uint64(), ctypes.c_uint32(), ctypes.c_int(), ctypes.c_uint64()
    rc = _load().oracle_info(src.ctypes.data, len(buf), ctypes.byref(rows), ctypes.byref(D), ctypes.byref(dt),
                             ctypes.byref(total))
    if rc != 0:
        raise OracleError(rc)
    return rows.value, D.value, CODE_DTYPE[dt.value], total.value


def decompress(buf: bytes) -> np.ndarray:
    rows, D, dt, _ = info(buf)
    out = np.zeros((rows, D), dtype=dt)
    src = np.frombuffer(buf, dtype=np.uint8)
    rc = _load().oracle_decompress(src.ctypes.data, len(buf), out.ctypes.data, out.nbytes)
    if rc != 0:
        raise OracleError(rc)
    return out


def decompress_rc(buf: bytes) -> int:
    """Return code of decoding ``buf`` (for corruption tests)."""
    src = np.frombuffer(buf, dtype=np.uint8)
    try:
        rows, D, dt, _ = info(buf)
    except OracleError as e:
        return e.rc
    out = np.zeros((rows, D), dtype=dt)
    return int(_load().oracle_decompress(src.ctypes.data, len(buf), out.ctypes.data, out.nbytes))


def residuals(x: np.ndarray, forecaster: str = "fire", learn_shift: int = 1,
              fixed_alpha: int | None = None) -> tuple[np.ndarray, np.ndarray]:
    """Forecaster errors (signed w-bit) of the full blocks of ``x`` coded as
    one segment, and the per-block FIRE coefficient alpha (in units of 2^-w).
    ``fixed_alpha`` holds alpha constant (no training)."""
    x = _as_2d(x)
    rows, D = x.shape
    nblk = rows // 8
    resid = np.zeros((nblk * 8, D), dtype=np.int64)
    alpha = np.zeros((nblk, D), dtype=np.int64)
    rc = _load().oracle_residuals(x.ctypes.data, rows, D, DTYPE_CODE[x.dtype], FORECASTERS[forecaster], learn_shift,
                                  0 if fixed_alpha is None else 1, 0 if fixed_alpha is None else int(fixed_alpha),
                                  resid.ctypes.data, alpha.ctypes.data)
    if rc != 0:
        raise OracleError(rc)
    return resid, alpha


def zigzag(e: int) -> int:
    return int(_load().oracle_zigzag(int(e)))


def unzigzag(z: int) -> int:
    return int(_load().oracle_unzigzag(int(z)))


def required_bits(z: int) -> int:
    return int(_load().oracle_required_bits(int(z)))


def code_of_nbits(nbits: int, w: int) -> int:
    return int(_load().oracle_code_of_nbits(nbits, w))


def width_of_code(code: int, w: int) -> int:
    return int(_load().oracle_width_of_code(code, w))

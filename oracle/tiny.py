"""Pure-Python twin of the Sprintz oracle -- test infrastructure only.

Written separately from ``sprintz_oracle.c`` (no shared code) from the same
paper and the same readings, for tiny inputs: bit strings are Python integers
and every step is spelled out. The tests compare the two byte for byte.

Paper: Blalock, Madden & Guttag, "Sprintz" (IMWUT 2018): Algorithm 1
(encodeBlock), Algorithm 2 (decodeBlock), Algorithm 3 (FIRE) with the
practical changes of Section 4.2.2, bit packing of Section 4.3.
"""
from __future__ import annotations

import struct

import numpy as np

_W = {np.dtype(np.int8): 8, np.dtype(np.uint8): 8, np.dtype(np.int16): 16, np.dtype(np.uint16): 16}
_DT = {np.dtype(np.int8): 1, np.dtype(np.uint8): 2, np.dtype(np.int16): 3, np.dtype(np.uint16): 4}


class _Bits:
    """Append-only LSB-first bit string."""

    def __init__(self):
        self.value = 0
        self.n = 0

    def put(self, v: int, k: int):
        assert 0 <= v < (1 << k) or k == 0 and v == 0
        self.value |= v << self.n
        self.n += k

    def pad_to_byte(self):
        self.n = -(-self.n // 8) * 8

    def to_bytes(self) -> bytes:
        assert self.n % 8 == 0
        return self.value.to_bytes(self.n // 8, "little") if self.n else b""


def _wrap_signed(v: int, w: int) -> int:
    v &= (1 << w) - 1
    return v - (1 << w) if v >> (w - 1) else v


def _block_residuals(rows, state, w, fire, learn_shift):
    """Run predict/train over one block (list of 8 rows of D ints).
    Returns the errors [8][D]; state = dict of lists prev, delta, acc."""
    D = len(rows[0])
    sh = learn_shift + 2
    lo, hi = -(1 << (w - 1)) << sh, (1 << w) << sh
    alpha = [(a >> sh) if fire else 0 for a in state["acc"]]  # Python >> is a floor shift
    grad = [0] * D
    errs = []
    for i, row in enumerate(rows):
        er = []
        for j in range(D):
            pred = state["prev"][j] + ((alpha[j] * state["delta"][j]) >> w) if fire else state["prev"][j]
            e = _wrap_signed(row[j] - pred, w)
            if fire and i % 2 == 1:
                grad[j] += ((e > 0) - (e < 0)) * state["delta"][j]
            state["delta"][j] = _wrap_signed(row[j] - state["prev"][j], w)
            state["prev"][j] = row[j]
            er.append(e)
        errs.append(er)
    if fire:
        for j in range(D):
            state["acc"][j] = min(hi, max(lo, state["acc"][j] + grad[j]))
    return errs


def _zz(e: int) -> int:
    return 2 * e if e >= 0 else -2 * e - 1


def _segment_bytes(vals, D, w, fire, learn_shift, G):
    """vals: list of rows (unsigned w-bit ints) of one segment."""
    hb = {8: 3, 16: 4}[w]
    nblk, tail = divmod(len(vals), 8)
    state = {"prev": [0] * D, "delta": [0] * D, "acc": [0] * D}
    recs = []  # (codes, payload bytes)
    run = 0
    for b in range(nblk):
        errs = _block_residuals(vals[8 * b: 8 * b + 8], state, w, fire, learn_shift)
        z = [[_zz(e) for e in r] for r in errs]
        need = [max(z[i][j].bit_length() for i in range(8)) for j in range(D)]
        if all(n == 0 for n in need):
            run += 1
            if run == 65535:
                recs.append(([0] * D, struct.pack("<H", run)))
                run = 0
            continue
        if run:
            recs.append(([0] * D, struct.pack("<H", run)))
            run = 0
        codes = [min(n, w - 1) for n in need]
        widths = [w if c == w - 1 else c for c in codes]
        bits = _Bits()
        if D * w <= 32:
            for j in range(D):
                for i in range(8):
                    bits.put(z[i][j], widths[j])
        else:
            for i in range(8):
                for j in range(D):
                    bits.put(z[i][j], widths[j])
                bits.pad_to_byte()
        recs.append((codes, bits.to_bytes()))
    if run:
        recs.append(([0] * D, struct.pack("<H", run)))
    out = bytearray(struct.pack("<I", len(recs)))
    g = G if G else max(len(recs), 1)
    for s in range(0, len(recs), g):
        grp = recs[s: s + g]
        hdr = _Bits()
        for codes, _ in grp:
            for c in codes:
                hdr.put(c, hb)
        hdr.pad_to_byte()
        out += hdr.to_bytes()
        for _, p in grp:
            out += p
    for r in vals[8 * nblk:]:
        for v in r:
            out += int(v).to_bytes(w // 8, "little")
    out += b"\0" * (-len(out) % 16)
    return bytes(out)


def compress(x: np.ndarray, forecaster: str = "fire", seg_rows: int | None = None, hdr_group: int = 0,
             learn_shift: int = 1) -> bytes:
    x = np.ascontiguousarray(x)
    if x.ndim == 1:
        x = x.reshape(-1, 1)
    rows, D = x.shape
    w = _W[x.dtype]
    S = seg_rows if seg_rows is not None else max(8, -(-rows // 8) * 8)
    u = x.view({8: np.uint8, 16: np.uint16}[w]).astype(np.int64).tolist()
    nseg = -(-rows // S) if rows else 0
    segs = [_segment_bytes(u[s * S:(s + 1) * S], D, w, forecaster == "fire", learn_shift, hdr_group)
            for s in range(nseg)]
    offs = [0]
    for sb in segs:
        offs.append(offs[-1] + len(sb))
    head = b"SPZ1" + struct.pack("<HBBBBBBIQIIQ", 1, w, _DT[x.dtype], 1 if forecaster == "fire" else 0,
                                 learn_shift, hdr_group, 0, D, rows, S, nseg, offs[-1])
    head += b"\0" * (64 - len(head))
    table = b"".join(struct.pack("<Q", o) for o in offs)
    pre = head + table
    pre += b"\0" * (-len(pre) % 16)
    return pre + b"".join(segs)

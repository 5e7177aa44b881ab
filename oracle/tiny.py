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


# ---------------------------------------------------------------------------
# Entropy stage (Section 4.4, Entropy Coding): Huffman coding of the packed
# bytes of each segment, in this library's own format (reading R19). Written
# from the reading, not from the C oracle: the tree is built by merging lists
# of the leaves below each node, and every merge adds one bit to each of them.
# ---------------------------------------------------------------------------
HUF_MAXLEN = 11
HUF_NSUB = 16


def _halve_up(c: int) -> int:
    return (c + 1) // 2


def huff_lengths(counts, halve=_halve_up, max_rounds=None, limit=HUF_MAXLEN) -> list:
    """Code length of each byte value 0..255 (0 = absent). Two-queue Huffman
    construction over the present values sorted by (count, value): the next
    node is the front leaf unless the front internal node weighs strictly
    less. While a length exceeds 11 bits, every count goes through `halve`
    and the construction starts again (`max_rounds` caps the number of
    halvings, `limit` is the longest allowed length; these parameters exist so
    that tests can plant other rules)."""
    present = [v for v in range(256) if counts[v] > 0]
    lengths = [0] * 256
    if len(present) == 1:
        lengths[present[0]] = 1
    if len(present) <= 1:
        return lengths
    weight = {v: int(counts[v]) for v in present}
    rounds = 0
    while True:
        leaves = [(weight[v], [v]) for v in sorted(present, key=lambda v: (weight[v], v))]
        inner = []
        depth = dict.fromkeys(present, 0)
        li = ii = 0
        for _ in range(len(present) - 1):
            picked = []
            for _t in range(2):
                if li < len(leaves) and (ii >= len(inner) or leaves[li][0] <= inner[ii][0]):
                    picked.append(leaves[li])
                    li += 1
                else:
                    picked.append(inner[ii])
                    ii += 1
            below = picked[0][1] + picked[1][1]
            for v in below:
                depth[v] += 1
            inner.append((picked[0][0] + picked[1][0], below))
        if max(depth.values()) <= limit or (max_rounds is not None and rounds >= max_rounds):
            for v in present:
                lengths[v] = depth[v]
            return lengths
        weight = {v: halve(weight[v]) for v in present}
        rounds += 1


def huff_canonical(lengths) -> dict:
    """value -> (code, length): values in (length, value) order get
    consecutive codes, shifted left once per extra bit of length."""
    lengths = [int(l) for l in lengths]
    codes, code, prev = {}, 0, None
    for v in sorted((v for v in range(256) if lengths[v]), key=lambda v: (lengths[v], v)):
        if prev is not None:
            code = (code + 1) << (lengths[v] - prev)
        codes[v] = (code, lengths[v])
        prev = lengths[v]
    return codes


def huff_encode_segment(plain: bytes, **rule) -> bytes:
    """u32 n | 128 bytes of 4-bit lengths (even values low) | 16 x u32
    sub-stream sizes | 16 sub-streams | zero pad to 16 bytes."""
    n = len(plain)
    assert n % HUF_NSUB == 0
    counts = [0] * 256
    for b in plain:
        counts[b] += 1
    lengths = huff_lengths(counts, **rule)
    codes = huff_canonical(lengths)
    m = n // HUF_NSUB
    subs = []
    for k in range(HUF_NSUB):
        bits = _Bits()
        for b in plain[k * m:(k + 1) * m]:
            code, l = codes[b]
            for t in reversed(range(l)):      # most significant bit first
                bits.put((code >> t) & 1, 1)
        bits.pad_to_byte()
        subs.append(bits.to_bytes())
    out = bytearray(struct.pack("<I", n))
    out += bytes(lengths[v] | (lengths[v + 1] << 4) for v in range(0, 256, 2))
    out += b"".join(struct.pack("<I", len(s)) for s in subs)
    out += b"".join(subs)
    out += b"\0" * (-len(out) % 16)
    return bytes(out)


def entropy_encode(plain_container: bytes) -> bytes:
    """A plain container with every segment replaced by its Huffman-coded
    form; header byte 11 = 1, offsets and data size describe the coded
    segments."""
    nseg = struct.unpack_from("<I", plain_container, 28)[0]
    data_start = -(-(64 + 8 * (nseg + 1)) // 16) * 16
    offs = struct.unpack_from(f"<{nseg + 1}Q", plain_container, 64)
    coded = [huff_encode_segment(plain_container[data_start + offs[s]:data_start + offs[s + 1]])
             for s in range(nseg)]
    new = [0]
    for c in coded:
        new.append(new[-1] + len(c))
    head = bytearray(plain_container[:64])
    head[11] = 1
    head[32:40] = struct.pack("<Q", new[-1])
    pre = bytes(head) + b"".join(struct.pack("<Q", o) for o in new)
    pre += b"\0" * (data_start - len(pre))
    return pre + b"".join(coded)

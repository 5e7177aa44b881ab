"""Pins of the oracle's entropy stage (Section 4.4: Huffman coding of the
bit-packed bytes; the coder and its format follow reading R19).

The lengths are pinned to what holds for any Huffman code, computed here
without the oracle: the optimal total cost from a heap-based construction
(library heapq, arbitrary tie-breaking), the Kraft equality, and the
length limit. The byte format is pinned to a hand-worked segment
(tests/golden/huffman_hand.txt); containers round-trip exactly."""
import heapq
import os

import numpy as np
import pytest

import datagen
import oracle
import oracle.tiny as tiny

GOLD = os.path.join(os.path.dirname(__file__), "golden", "huffman_hand.txt")


def _heap_huffman(counts):
    """Optimal (unlimited) Huffman cost sum(count * length) and the tree depth
    by the textbook heap construction: the cost is the sum of all merged
    weights."""
    h = [(int(c), 0, k) for k, c in enumerate(counts) if c > 0]
    if len(h) < 2:
        return sum(c for c, _, _ in h), len(h)
    heapq.heapify(h)
    cost, uid = 0, 256
    while len(h) > 1:
        (a, da, _), (b, db, _) = heapq.heappop(h), heapq.heappop(h)
        cost += a + b
        heapq.heappush(h, (a + b, max(da, db) + 1, uid))
        uid += 1
    return cost, h[0][1]


def _heap_cost(counts):
    return _heap_huffman(counts)[0]


def _kraft(lengths):
    return sum(2.0 ** -int(l) for l in lengths if l > 0)


def _canonical(lengths):
    codes, c, prev = {}, 0, None
    for v in sorted((v for v in range(256) if lengths[v]), key=lambda v: (lengths[v], v)):
        if prev is not None:
            c = (c + 1) << (int(lengths[v]) - prev)
        codes[v] = (c, int(lengths[v]))
        prev = int(lengths[v])
    return codes


def test_hand_worked_segment():
    lines = [l.split() for l in open(GOLD) if l.strip() and not l.startswith("#")]
    kv = {l[0]: l[1:] for l in lines}
    word, rep = kv["plain_repeat"][0].encode(), int(kv["plain_repeat"][1])
    plain = word * rep
    want = bytes.fromhex(kv["segment_hex"][0])
    counts = np.bincount(np.frombuffer(plain, np.uint8), minlength=256)
    lens = oracle.huff_lengths(counts)
    for item in kv["lengths"]:
        sym, l = item.split("=")
        assert lens[ord(sym)] == int(l)
    assert oracle.huff_encode_segment(plain) == want
    assert oracle.huff_decode_segment(want, len(plain)) == plain


@pytest.mark.parametrize("seed", range(12))
def test_lengths_are_optimal_and_complete(seed):
    rng = np.random.default_rng(seed)
    nsym = [2, 3, 5, 17, 100, 256][seed % 6]
    counts = np.zeros(256, np.uint64)
    syms = rng.choice(256, size=nsym, replace=False)
    counts[syms] = rng.integers(1, 1000, size=nsym)
    lens = oracle.huff_lengths(counts)
    assert ((lens > 0) == (counts > 0)).all()
    cost, depth = _heap_huffman(counts)
    assert lens.max() <= 11
    if depth <= 11:
        # no length limit needed: the code is an optimal Huffman code
        assert int((counts * lens).sum()) == cost
        assert _kraft(lens) == 1.0
    else:
        assert _kraft(lens) <= 1.0 and int((counts * lens).sum()) >= cost


def test_length_limit():
    # Fibonacci counts give a maximally skewed tree (depth 24 unlimited)
    fib = [1, 1]
    while len(fib) < 25:
        fib.append(fib[-1] + fib[-2])
    counts = np.zeros(256, np.uint64)
    counts[:25] = fib
    lens = oracle.huff_lengths(counts)
    assert lens.max() <= 11 and (lens[:25] > 0).all() and (lens[25:] == 0).all()
    assert _kraft(lens) <= 1.0
    # the limit is only applied when needed: a small skewed set keeps its depths
    counts = np.zeros(256, np.uint64)
    counts[:6] = fib[:6]
    assert int((counts * oracle.huff_lengths(counts)).sum()) == _heap_cost(counts)


def test_single_and_empty_alphabets():
    counts = np.zeros(256, np.uint64)
    assert (oracle.huff_lengths(counts) == 0).all()
    counts[200] = 77
    lens = oracle.huff_lengths(counts)
    assert lens[200] == 1 and lens.sum() == 1
    seg = oracle.huff_encode_segment(bytes([200]) * 32)
    assert oracle.huff_decode_segment(seg, 32) == bytes([200]) * 32


def test_canonical_codes_are_prefix_free():
    rng = np.random.default_rng(5)
    counts = rng.integers(0, 50, size=256).astype(np.uint64)
    lens = oracle.huff_lengths(counts)
    codes = _canonical(lens)
    strs = sorted(format(c, f"0{l}b") for c, l in codes.values())
    for a, b in zip(strs, strs[1:]):
        assert not b.startswith(a)


@pytest.mark.parametrize("f", ["delta", "fire"])
def test_entropy_containers_round_trip(f):
    for x, S in [(datagen.ar2_uint16(5003, 4, seed=1), 512), (datagen.walk_int8(4099, 1, seed=2), 1024),
                 (datagen.uniform(777, 3, np.uint8, seed=3), 64), (np.zeros((0, 2), np.int16), 64),
                 (np.zeros((4096, 2), np.int16), 1024)]:
        plain = oracle.compress(x, f, S)
        coded = oracle.compress(x, f, S, entropy=1)
        assert coded[11] == 1 and plain[11] == 0
        assert oracle.entropy_decode(coded) == plain
        assert np.array_equal(oracle.decompress(coded), x)


def test_entropy_corrupt_segment_is_rejected():
    x = datagen.ar2_uint16(3000, 4, seed=4)
    coded = bytearray(oracle.compress(x, "fire", 512, entropy=1))
    ds = (64 + 8 * (int.from_bytes(coded[28:32], "little") + 1) + 15) & ~15
    coded[ds + 4 + 64] = 0xFF     # a code length of 15 bits
    assert oracle.decompress_rc(bytes(coded)) == -3


def test_full_alphabet_optimal():
    rng = np.random.default_rng(9)
    counts = rng.integers(200, 1000, size=256).astype(np.uint64)
    lens = oracle.huff_lengths(counts)
    cost, depth = _heap_huffman(counts)
    assert depth <= 11
    assert int((counts * lens).sum()) == cost and _kraft(lens) == 1.0


LIMIT_GOLD = os.path.join(os.path.dirname(__file__), "golden", "huffman_limit_hand.txt")


def _limit_golden():
    kv = {}
    for line in open(LIMIT_GOLD):
        if line.strip() and not line.startswith("#"):
            parts = line.split()
            kv[parts[0]] = parts[1:]

    def table(key, conv):
        return {ord(it.split("=")[0]): conv(it.split("=")[1]) for it in kv[key]}

    return (table("counts", int), table("halved", int), table("lengths", int), table("codes", str),
            bytes.fromhex(kv["len_table_48_54"][0]))


def _decode_with(codes, stream: bytes, count: int) -> bytes:
    """Prefix-decode `count` symbols of a byte-aligned LSB-first bit stream in
    which each code is stored from its first (most significant) bit on."""
    inv = {c: v for v, c in codes.items()}
    bits = "".join(format(b, "08b")[::-1] for b in stream)
    out, cur = bytearray(), ""
    for ch in bits:
        cur += ch
        if cur in inv:
            out.append(inv[cur])
            cur = ""
            if len(out) == count:
                break
    assert len(out) == count
    return bytes(out)


def test_length_limited_code_hand_worked():
    counts_d, halved_d, lengths_d, codes_d, len_table = _limit_golden()
    counts = np.zeros(256, np.uint64)
    for v, c in counts_d.items():
        counts[v] = c
    assert sum(counts_d.values()) % 16 == 0
    # the golden's own halving arithmetic, and that the unlimited tree is too deep
    assert {v: (c + 1) // 2 for v, c in counts_d.items()} == halved_d
    assert max(tiny.huff_lengths(list(counts), max_rounds=0)) == 12
    want = np.zeros(256, np.uint8)
    for v, l in lengths_d.items():
        want[v] = l
    assert list(oracle.huff_lengths(counts)) == list(want)          # the C oracle
    assert tiny.huff_lengths(list(counts)) == list(want)            # the Python twin
    assert tiny.huff_canonical(list(want)) == {v: (int(s, 2), len(s)) for v, s in codes_d.items()}
    # a coded segment of these bytes in a seeded order: its length table and
    # every sub-stream decode with the hand-worked codes
    rng = np.random.default_rng(21)
    plain = bytes(rng.permutation(np.repeat(np.array(list(counts_d)), list(counts_d.values()))).astype(np.uint8))
    seg = oracle.huff_encode_segment(plain)
    assert seg == tiny.huff_encode_segment(plain)
    assert int.from_bytes(seg[:4], "little") == len(plain)
    table = seg[4:132]
    assert table[48:55] == len_table and not any(table[:48]) and not any(table[55:])
    m = len(plain) // 16
    sizes = [int.from_bytes(seg[132 + 4 * k:136 + 4 * k], "little") for k in range(16)]
    pos = 196
    for k in range(16):
        sub = plain[k * m:(k + 1) * m]
        assert sizes[k] == -(-sum(lengths_d[b] for b in sub) // 8)
        assert _decode_with(codes_d, seg[pos:pos + sizes[k]], m) == sub
        pos += sizes[k]


def test_length_limit_golden_rejects_other_rules():
    # the hand-worked case tells the reading's rule apart from near misses,
    # each planted in the Python twin
    counts_d, _, lengths_d, _, _ = _limit_golden()
    counts = [0] * 256
    for v, c in counts_d.items():
        counts[v] = c
    want = [0] * 256
    for v, l in lengths_d.items():
        want[v] = l
    assert tiny.huff_lengths(counts) == want
    assert tiny.huff_lengths(counts, halve=lambda c: c // 2 + 1) != want        # other rounding of the halving
    assert tiny.huff_lengths(counts, halve=lambda c: max(1, c // 2)) != want    # floor, kept present
    assert tiny.huff_lengths(counts, max_rounds=0) != want                      # one halving fewer
    assert tiny.huff_lengths(counts, limit=10) != want                          # limit off by one
    assert tiny.huff_lengths(counts, limit=12) != want


def _plain_segments(rng):
    """Plain segments of oracle containers: Laplace walks (the 4 GiB D = 4
    uint16 workload's recipe, at small sizes), AR(2), int8 walks, uniform
    bytes, plus raw byte strings of skewed distributions."""
    segs = []
    for k in range(6):
        x = datagen.laplace_walk_uint16(2048 * 4 + 16 * k, 4, scale=3.0, seed=30 + k)
        c = oracle.compress(x, "fire", 2048)
        nseg = int.from_bytes(c[28:32], "little")
        ds = (64 + 8 * (nseg + 1) + 15) & ~15
        offs = [int.from_bytes(c[64 + 8 * s:72 + 8 * s], "little") for s in range(nseg + 1)]
        segs += [c[ds + offs[s]:ds + offs[s + 1]] for s in range(nseg)]
    for x, S in [(datagen.ar2_uint16(4096, 8, seed=40), 512), (datagen.walk_int8(8192, 1, seed=41), 1024),
                 (datagen.uniform(2048, 2, np.uint8, seed=42), 256)]:
        c = oracle.compress(x, "delta", S)
        nseg = int.from_bytes(c[28:32], "little")
        ds = (64 + 8 * (nseg + 1) + 15) & ~15
        offs = [int.from_bytes(c[64 + 8 * s:72 + 8 * s], "little") for s in range(nseg + 1)]
        segs += [c[ds + offs[s]:ds + offs[s + 1]] for s in range(nseg)]
    for k in range(60):
        n = 16 * int(rng.integers(1, 200))
        p = np.minimum(rng.geometric(float(rng.uniform(0.05, 0.9)), size=n) - 1, 255).astype(np.uint8)
        segs.append(p.tobytes())
    return segs


def test_c_oracle_equals_python_twin_on_many_segments():
    rng = np.random.default_rng(3)
    segs = _plain_segments(rng)
    assert len(segs) >= 100
    limited = 0
    for s in segs:
        counts = np.bincount(np.frombuffer(s, np.uint8), minlength=256)
        if max(tiny.huff_lengths(list(counts), max_rounds=0)) > 11:
            limited += 1
        assert oracle.huff_encode_segment(s) == tiny.huff_encode_segment(s)
    assert limited >= 20, limited   # the length limit is exercised, not only the plain construction
    # whole containers, header and offsets included
    x = datagen.laplace_walk_uint16(2048 * 3 + 5, 4, scale=3.0, seed=50)
    plain = oracle.compress(x, "fire", 2048)
    assert oracle.entropy_encode(plain) == tiny.entropy_encode(plain)

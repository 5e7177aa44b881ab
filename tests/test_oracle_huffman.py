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

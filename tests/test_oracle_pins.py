"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every check here compares the oracle with something other than itself:
closed forms, brute force, hand-derived bytes, the paper's worked examples,
special cases of the FIRE model that reduce to textbook predictors, and the
lossless round trip. Paper: Blalock et al., "Sprintz", IMWUT 2018.
"""
import os

import numpy as np
import pytest

import datagen
import oracle
from oracle import tiny

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _sext(v, w):
    v = np.asarray(v, dtype=np.int64) & ((1 << w) - 1)
    return np.where(v >= (1 << (w - 1)), v - (1 << w), v)


# --------------------------------------------------------------------------
# Zigzag (Section 4.3): each integer maps to twice its absolute value, or
# twice its absolute value minus one if negative.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("w", [8, 16])
def test_zigzag_exhaustive(w):
    lib = oracle.lib()
    es = range(-(1 << (w - 1)), 1 << (w - 1))
    seen = set()
    for e in es:
        z = lib.oracle_zigzag(e)
        assert z == (2 * abs(e) if e >= 0 else 2 * abs(e) - 1)
        assert lib.oracle_unzigzag(z) == e
        seen.add(z)
    # a bijection onto the w-bit range
    assert seen == set(range(1 << w))


def test_zigzag_orders_by_magnitude():
    # farther from zero -> larger code
    for e in range(-100, 100):
        assert oracle.zigzag(e) < oracle.zigzag(abs(e) + 1)


# --------------------------------------------------------------------------
# Bit widths (Section 4.3)
# --------------------------------------------------------------------------
def test_required_bits_brute_force():
    for z in list(range(0, 70000)) + [2**31 - 1, 2**32 - 1]:
        k = 0
        while z >= (1 << k):
            k += 1
        assert oracle.required_bits(z) == k


def test_paper_example_sixteen_needs_five_bits():
    # Section 4.3: largest zigzag value 16 = 00010000 has three leading zeros
    # in 8 bits, so 8 - 3 = 5 bits are needed.
    assert oracle.required_bits(16) == 5


@pytest.mark.parametrize("w", [8, 16])
def test_width_w_minus_one_stored_as_w(w):
    # Section 4.3: header fields have log2(w) bits, so a width of w-1 is
    # treated as w by encoder and decoder.
    for n in range(w + 1):
        c = oracle.code_of_nbits(n, w)
        assert 0 <= c < (1 << (3 if w == 8 else 4))
        width = oracle.width_of_code(c, w)
        assert width >= n
        assert width == (w if n >= w - 1 else n)


def test_seven_bit_block_stored_with_eight_bits():
    # a block of 8-bit data whose largest error needs 7 bits occupies 8 bytes
    # (column-major, one column): 8 values x 8 bits.
    x = np.array([0, 63, 0, 0, 0, 0, 0, 0], dtype=np.int8)  # delta errors 0, 63, -63, 0.. -> zigzag 126 -> 7 bits
    b = oracle.compress(x, "delta", seg_rows=8)
    seg = b[80:]
    assert seg[:4] == (1).to_bytes(4, "little")
    assert seg[4] == 7                              # code 7
    assert len(seg) == 16 and seg[5:13] == bytes([0, 126, 125, 0, 0, 0, 0, 0])  # 8 full bytes


# --------------------------------------------------------------------------
# Delta coding (Section 4.2.1): prediction is the previous sample, x_0 = 0.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dt", [np.int8, np.uint8, np.int16, np.uint16])
def test_delta_residuals_closed_form(dt):
    w = np.dtype(dt).itemsize * 8
    x = datagen.uniform(80, 5, dt, seed=11)
    e, alpha = oracle.residuals(x, "delta")
    u = x.view(np.uint8 if w == 8 else np.uint16).astype(np.int64)
    prev = np.vstack([np.zeros((1, 5), np.int64), u[:-1]])
    assert np.array_equal(e, _sext(u - prev, w))
    assert not alpha.any()


def test_paper_isolated_spike_example():
    # Section 5.7: {0, -1, 0, 0} delta-codes to {0, -1, 1, 0}; zigzag
    # {0, 1, 2, 0} needs 2 bits where the raw zigzag {0, 1, 0, 0} needs 1.
    x = np.array([0, -1, 0, 0, 0, 0, 0, 0], dtype=np.int8)
    e, _ = oracle.residuals(x, "delta")
    assert e[:4, 0].tolist() == [0, -1, 1, 0]
    assert [oracle.zigzag(v) for v in e[:4, 0]] == [0, 1, 2, 0]
    b = oracle.compress(x, "delta", seg_rows=8)
    assert b[80 + 4] == 2                                   # 2-bit column
    assert max(oracle.required_bits(oracle.zigzag(v)) for v in [0, -1, 0, 0]) == 1


def test_delta_decode_is_cumsum():
    # decoding delta errors is a running sum modulo 2^w (numpy cumsum)
    x = datagen.walk_int8(4000, 3, seed=4)
    e, _ = oracle.residuals(x, "delta")
    rec = np.cumsum(e, axis=0) % 256
    assert np.array_equal(rec, x[: len(e)].view(np.uint8).astype(np.int64))


# --------------------------------------------------------------------------
# FIRE (Section 4.2.2). The model x_i = x_{i-1} + alpha (x_{i-1} - x_{i-2})
# reduces to delta coding at alpha = 0, to double delta at alpha = 1 and to
# the mean of the two previous samples at alpha = -1/2. alpha is in units of
# 2^-w, so these are 0, 2^w and -2^(w-1).
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dt", [np.uint8, np.int16])
def test_fire_alpha_zero_is_delta(dt):
    x = datagen.uniform(160, 4, dt, seed=12)
    e0, a0 = oracle.residuals(x, "fire", fixed_alpha=0)
    ed, _ = oracle.residuals(x, "delta")
    assert np.array_equal(e0, ed) and not a0.any()


@pytest.mark.parametrize("dt", [np.uint8, np.int8, np.uint16, np.int16])
def test_fire_alpha_one_is_double_delta(dt):
    w = np.dtype(dt).itemsize * 8
    x = datagen.uniform(160, 3, dt, seed=13)
    e, a = oracle.residuals(x, "fire", fixed_alpha=1 << w)
    assert (a == (1 << w)).all()
    u = x.view(np.uint8 if w == 8 else np.uint16).astype(np.int64)
    p1 = np.vstack([np.zeros((1, 3), np.int64), u[:-1]])
    p2 = np.vstack([np.zeros((2, 3), np.int64), u[:-2]])
    assert np.array_equal(e, _sext(u - 2 * p1 + p2, w))


@pytest.mark.parametrize("w", [8, 16])
def test_fire_alpha_minus_half_is_mean_of_previous_two(w):
    # no wrap-around: values in the middle of the range, small steps
    rng = np.random.default_rng(14)
    mid = 1 << (w - 1)
    u = mid + rng.integers(-(1 << (w - 3)), 1 << (w - 3), size=(96, 2))
    x = u.astype(np.uint8 if w == 8 else np.uint16)
    e, _ = oracle.residuals(x, "fire", fixed_alpha=-(1 << (w - 1)))
    p1 = np.vstack([np.zeros((1, 2), np.int64), u[:-1]])
    p2 = np.vstack([np.zeros((2, 2), np.int64), u[:-2]])
    # rows 0 and 1 see the zero start; from row 2 on the mean predictor holds
    assert np.array_equal(e[2:], (u - (p1 + p2) // 2)[2:])


def test_fire_first_block_is_delta():
    x = datagen.ar2_uint16(64, 8, seed=3)
    ef, af = oracle.residuals(x, "fire")
    ed, _ = oracle.residuals(x, "delta")
    assert not af[0].any()                          # accumulator starts at 0
    assert np.array_equal(ef[:8], ed[:8])


def _ramp(slope, n, dt=np.uint8):
    w = np.dtype(dt).itemsize * 8
    return ((slope * np.arange(n)) % (1 << w)).astype(dt).reshape(-1, 1)


def test_fire_learns_positive_ramp_hand_derived():
    # slope +5 on 8-bit data (wrapping). Block 0: gradients at rows 3, 5, 7
    # (row 1 sees delta 0) give acc = 15; each later block adds 4 x 5 = 20
    # while alpha < 256, so acc_b = 20 b - 5 and alpha_b = floor(acc_b / 8).
    # At b = 103 the accumulator saturates at 2^8 x 8, alpha = 256 (double
    # delta) and every error is 0 from then on ("constant slopes", Section 5.7).
    nb = 140
    x = _ramp(5, 8 * nb)
    e, a = oracle.residuals(x, "fire")
    expect = [0] + [min(256, (20 * b - 5) // 8) for b in range(1, nb)]
    assert a[:, 0].tolist() == expect
    assert a[102, 0] == 254 and a[103, 0] == 256
    assert (e[8 * 103:] == 0).all() and (e[8 * 102:8 * 103] != 0).any()
    # the tail of the stream becomes one run-length record
    b = oracle.compress(x, "fire")
    nrec = int.from_bytes(b[80:84], "little")
    assert nrec == 103 + 1


def test_fire_learns_negative_ramp_hand_derived():
    # slope -3: errors are negative while alpha <= 170, each odd row adds
    # (-1)(-3) = 3, so acc_b = 12 b - 3; floor rounding makes alpha = 172 at
    # b = 115, where floor(-3 * 172 / 256) = -3 and the error vanishes.
    nb = 150
    x = _ramp(-3, 8 * nb)
    e, a = oracle.residuals(x, "fire")
    expect = [0] + [(12 * b - 3) // 8 for b in range(1, 115)] + [172] * (nb - 115)
    assert a[:, 0].tolist() == expect
    assert (e[8 * 115:] == 0).all() and (e[8 * 114:8 * 115] != 0).any()


def test_delta_never_learns_ramp():
    x = _ramp(5, 8 * 50)
    e, _ = oracle.residuals(x, "delta")
    assert (e[1:] == 5).all()


def test_constant_run_residuals():
    # delta: zero errors from the second row of a constant run; FIRE: from
    # the third (the jump into the run leaves a nonzero delta once).
    x = datagen.walk_int8(400, 2, sigma=6, const_frac=0.0, seed=21).astype(np.int64)
    x[200:260] = x[200]
    x = x.astype(np.int8)
    ed, _ = oracle.residuals(x, "delta")
    ef, _ = oracle.residuals(x, "fire")
    assert (ed[201:260] == 0).all()
    assert (ef[202:260] == 0).all()


# --------------------------------------------------------------------------
# Run-length coding (Algorithm 1): a run of all-zero blocks is D zero
# headers plus the number of blocks. Counts are u16 (split at 65535).
# --------------------------------------------------------------------------
@pytest.mark.parametrize("f", ["delta", "fire"])
def test_all_zero_closed_form(f):
    for D, dt, rows in [(1, np.int8, 8 * 10), (5, np.uint16, 8 * 3 + 5), (16, np.int16, 8 * 700)]:
        x = np.zeros((rows, D), dtype=dt)
        b = oracle.compress(x, f)
        w = np.dtype(dt).itemsize * 8
        hb = 3 if w == 8 else 4
        nblk, tail = divmod(rows, 8)
        seg = 4 + (D * hb + 7) // 8 + 2 + tail * D * (w // 8)
        seg += -seg % 16
        assert len(b) == 80 + seg
        assert int.from_bytes(b[80:84], "little") == 1
        assert int.from_bytes(b[80 + 4 + (D * hb + 7) // 8:][:2], "little") == nblk
        assert np.array_equal(oracle.decompress(b), x)


def test_rle_count_split_at_u16_limit():
    rows = 8 * (65535 + 1)
    x = np.zeros((rows, 1), dtype=np.uint8)
    b = oracle.compress(x, "delta")
    seg = b[80:]
    assert int.from_bytes(seg[:4], "little") == 2            # two RLE records
    assert seg[4] == 0                                       # 2 x 3 zero header bits, padded
    assert int.from_bytes(seg[5:7], "little") == 65535
    assert int.from_bytes(seg[7:9], "little") == 1
    assert len(seg) == 16
    assert np.array_equal(oracle.decompress(b), x)


# --------------------------------------------------------------------------
# Hand-derived containers (tests/golden)
# --------------------------------------------------------------------------
def _load_golden(name):
    inp, params, hexs = None, None, []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            tok = line.split()
            if tok[0] == "input":
                dt = np.dtype(tok[1])
                D = int(tok[2])
                vals = [int(v) for v in tok[3:]]
                inp = np.array(vals, dtype=np.int64).astype(dt).reshape(-1, D)
            elif tok[0] == "params":
                params = (tok[1], int(tok[2]), int(tok[3]), int(tok[4]))
            elif tok[0] == "hex":
                hexs.append("".join(tok[1:]))
    return inp, params, bytes.fromhex("".join(hexs))


@pytest.mark.parametrize("name", ["hand_delta_d1_w8.txt", "hand_delta_d3_w16_rle.txt"])
def test_golden_hand_derived(name):
    x, (f, S, G, ls), expect = _load_golden(name)
    got = oracle.compress(x, f, seg_rows=S, hdr_group=G, learn_shift=ls)
    assert got == expect
    assert np.array_equal(oracle.decompress(expect), x)


# --------------------------------------------------------------------------
# Lossless round trip (Section 1: the codec is lossless) and size bound
# --------------------------------------------------------------------------
def _cases(n, seed):
    rng = np.random.default_rng(seed)
    for _ in range(n):
        rows = int(rng.integers(0, 300))
        D = int(rng.integers(1, 81))
        dt = [np.int8, np.uint8, np.int16, np.uint16][int(rng.integers(0, 4))]
        kind = int(rng.integers(0, 4))
        if kind == 0:
            x = datagen.uniform(rows, D, dt, seed=int(rng.integers(1 << 30)))
        elif kind == 1:
            x = np.zeros((rows, D), dtype=dt)
        elif kind == 2:
            info = np.iinfo(dt)
            x = rng.choice([info.min, info.max, 0, -1 if info.min < 0 else 1], size=(rows, D)).astype(dt)
        else:
            x = (np.cumsum(rng.integers(-3, 4, size=(rows, D)), axis=0)).astype(dt)
        f = ["delta", "fire"][int(rng.integers(0, 2))]
        S = [8, 16, 64, None][int(rng.integers(0, 4))]
        G = [0, 1, 2, 8][int(rng.integers(0, 4))]
        yield x, f, S, G


def test_round_trip_random_shapes():
    for x, f, S, G in _cases(400, 7):
        b = oracle.compress(x, f, seg_rows=S, hdr_group=G)
        Seff = S if S is not None else max(8, -(-len(x) // 8) * 8)
        assert len(b) <= oracle.compress_bound(len(x), x.shape[1], x.dtype, Seff, G)
        assert len(b) % 16 == 0
        y = oracle.decompress(b)
        assert y.dtype == x.dtype and np.array_equal(x, y)


@pytest.mark.parametrize("w", [8, 16])
def test_round_trip_exhaustive_three_symbols(w):
    # every 8-row univariate input over {0, 1, 2^w - 1}: 3^8 cases
    dt = np.uint8 if w == 8 else np.uint16
    M = 1 << w
    sym = np.array([0, 1, M - 1], dtype=np.int64)
    idx = np.indices((3,) * 8).reshape(8, -1).T
    allx = sym[idx].astype(dt)
    for f in ("delta", "fire"):
        for x in allx:
            x = x.reshape(8, 1)
            assert np.array_equal(oracle.decompress(oracle.compress(x, f, seg_rows=8)), x)


# --------------------------------------------------------------------------
# Cross-check against the independent pure-Python twin
# --------------------------------------------------------------------------
def test_cross_oracle_byte_for_byte():
    rng = np.random.default_rng(99)
    n = 0
    for x, f, S, G in _cases(400, 8):
        if x.size > 6000:
            continue
        ls = int(rng.integers(0, 3))
        assert oracle.compress(x, f, S, G, ls) == tiny.compress(x, f, S, G, ls)
        n += 1
    # learned FIRE state over many blocks
    x = datagen.ar2_uint16(800, 3, seed=5)
    assert oracle.compress(x, "fire", 256) == tiny.compress(x, "fire", 256)
    x = datagen.walk_int8(1600, 2, seed=6)
    assert oracle.compress(x, "fire", None, 2) == tiny.compress(x, "fire", None, 2)
    assert n > 150


# --------------------------------------------------------------------------
# Corruption: defined errors, never a crash
# --------------------------------------------------------------------------
def test_corruption_is_detected_or_harmless():
    x = datagen.ar2_uint16(2000, 8, seed=8)
    b = bytearray(oracle.compress(x, "fire", 256))
    for cut in [0, 10, 63, 64, 80, len(b) // 2, len(b) - 16]:
        assert oracle.decompress_rc(bytes(b[:cut])) == -3
    rng = np.random.default_rng(1)
    for _ in range(300):
        c = bytearray(b)
        k = int(rng.integers(0, len(c)))
        c[k] ^= 1 << int(rng.integers(0, 8))
        assert oracle.decompress_rc(bytes(c)) in (0, -3)

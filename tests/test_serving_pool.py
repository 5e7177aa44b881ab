"""Host logic of the serving loop: the first-fit arena allocator (CPU only)."""
import random

import pytest

torch = pytest.importorskip("torch")

from paper_1808_02515_amd.serving import ALIGN, DevicePool


def test_pool_first_fit_and_coalescing():
    p = DevicePool(64 * ALIGN, device="cpu")
    a = p.alloc(1)
    b = p.alloc(3 * ALIGN)
    c = p.alloc(ALIGN + 1)
    assert a == (0, ALIGN) and b == (ALIGN, 3 * ALIGN) and c == (4 * ALIGN, 2 * ALIGN)
    assert p.alloc(59 * ALIGN) is None
    p.release(*b)
    assert p.alloc(3 * ALIGN) == (ALIGN, 3 * ALIGN)      # the hole is reused first
    p.release(ALIGN, 3 * ALIGN)
    p.release(*a)
    p.release(*c)
    assert p.free == [(0, 64 * ALIGN)] and p.used == 0


def test_pool_random_never_overlaps():
    rng = random.Random(3)
    p = DevicePool(1000 * ALIGN, device="cpu")
    live = []
    for _ in range(3000):
        if live and rng.random() < 0.45:
            p.release(*live.pop(rng.randrange(len(live))))
        else:
            a = p.alloc(rng.randint(1, 40 * ALIGN))
            if a is not None:
                live.append(a)
        spans = sorted(live)
        for (o1, n1), (o2, _) in zip(spans, spans[1:]):
            assert o1 + n1 <= o2
        assert p.used == sum(n for _, n in live)
        assert p.used + sum(n for _, n in p.free) == p.size
    for a in live:
        p.release(*a)
    assert p.free == [(0, p.size)]

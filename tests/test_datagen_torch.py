"""The GPU forms of the input recipes (datagen.*_torch), checked on the CPU
against the sequential definitions they replace."""
import numpy as np
import pytest
from scipy.signal import lfilter

import datagen

torch = pytest.importorskip("torch")


def test_clipped_walk_scan_equals_sequential_clip():
    steps = np.random.default_rng(0).integers(-90, 91, size=(3001, 4))
    got = datagen.clipped_walk_torch(torch.from_numpy(steps), -128, 127).numpy()
    want = np.zeros_like(steps)
    x = np.zeros(4, dtype=np.int64)
    for t in range(len(steps)):           # the definition, one step at a time
        x = np.clip(x + steps[t], -128, 127)
        want[t] = x
    assert np.array_equal(got, want)


def test_ar2_scan_equals_recursive_filter():
    e = np.random.default_rng(1).normal(0, 20, size=(4000, 3))
    got = datagen.ar2_filter_torch(torch.from_numpy(e)).numpy()
    want = lfilter([1.0], [1.0, -1.6, 0.7], e, axis=0)
    assert np.abs(got - want).max() < 1e-9 * np.abs(want).max()


def test_torch_recipes_shapes_and_statistics():
    g = torch.Generator()
    g.manual_seed(5)
    x = datagen.ar2_uint16_torch(50000, 4, 20.0, 0.2, g, "cpu").numpy().view(np.uint16)
    flat = np.all(x[1:] == x[:-1], axis=1).mean()
    assert x.shape == (50000, 4) and 0.19 <= flat <= 0.25
    assert 60 < x[:, 0].astype(np.float64).std() < 110        # AR(2) std is about 4.2 sigma
    y = datagen.walk_int8_torch(50000, 2, 2.0, 0.15, g, "cpu").numpy()
    assert y.dtype == np.int8 and y.shape == (50000, 2)
    rows, D, dt, sigma = datagen.batch_stream_params(7)
    z = datagen.batch_stream_torch(7, device="cpu")
    assert z.shape == (rows, D) and z.element_size() == dt.itemsize


def test_wrap_walk_matches_numpy():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(4)
    steps = np.rint(rng.laplace(0.0, 3.0, size=(5000, 4))).astype(np.int64)
    want = ((32768 + np.cumsum(steps, axis=0)) % 65536).astype(np.uint16)
    got = datagen.wrap_walk_torch(torch.from_numpy(steps)).numpy().view(np.uint16)
    assert np.array_equal(got, want)


def test_laplace_walk_torch_chunks_and_scale():
    torch = pytest.importorskip("torch")
    g = torch.Generator()
    g.manual_seed(1)
    x = datagen.laplace_walk_uint16_torch(20000, 3, 3.0, g, "cpu", chunk=777).numpy().view(np.uint16)
    d = (np.diff(x.astype(np.int64), axis=0) + 32768) % 65536 - 32768
    # continuity across chunks and Laplace(0, 3) steps: mean |step| = 3 (rounded: about 3.0)
    assert np.abs(d).max() < 200 and abs(np.abs(d).mean() - 3.0) < 0.15
    assert x[0].astype(np.int64).tolist() != [0, 0, 0]

"""Seeded synthetic inputs for the Sprintz codec (tests and benchmark).

This module holds no codec arithmetic: it only draws the integer time series
that both the CPU oracle and the GPU library are fed. The paper's own speed
experiments use synthetic data too (Section 5.4: uniform random values at
full range); the shaped generators below mimic sensor streams -- random
walks, stationary AR(2) columns and constant runs -- because the datasets of
the paper's ratio experiments (UCR, PAMAP, MSRC-12, UCI Gas, AMPDs) are not
available here. Every generator is a pure function of its seed.

Workloads (sizes as in the benchmark configuration list):
  * ``walk_int8``   -- 65,536 x 1 int8 random walk, N(0, 2) integer steps,
                       clipped to [-128, 127], 15 % of samples in constant runs
                       of 8..256 rows; seed 0.
  * ``ar2_uint16``  -- 4,194,304 x 8 uint16, each column AR(2) with
                       coefficients (1.6, -0.7) and N(0, 20) noise, offset
                       32768 and clipped; 20 % of rows in flat runs of 8..256
                       rows in which every column repeats the previous row;
                       seed 1.
  * ``batch_stream``-- one stream of the 10,000-stream batch (seed 2e6 + k).
  * ``laplace_walk_uint16`` -- D=4 uint16 walks with Laplace(0, 3) steps,
                       wrapping modulo 2^16 (the Huffman workload); seed 3.
  * ``uniform``     -- full-range uniform values (the paper's speed workload).
"""
from __future__ import annotations

import numpy as np
from scipy.signal import lfilter


def _run_mask(rng: np.random.Generator, n: int, coverage: float, lo: int = 8, hi: int = 256) -> np.ndarray:
    """Boolean mask of length n made of runs of U{lo..hi} positions, added
    at uniform random starts until at least ``coverage`` of n is covered."""
    mask = np.zeros(n, dtype=bool)
    if n == 0 or coverage <= 0:
        return mask
    target = coverage * n
    covered = 0
    while covered < target:
        L = int(rng.integers(lo, hi + 1))
        L = min(L, n)
        s = int(rng.integers(0, n - L + 1))
        before = int(mask[s:s + L].sum())
        mask[s:s + L] = True
        covered += L - before
    return mask


def clipped_walk(start: int, steps: np.ndarray, lo: int, hi: int) -> np.ndarray:
    """x_t = clip(x_{t-1} + steps_t, lo, hi), x_{-1} = start, along axis 0.

    The map y -> clip(y + a, lo, hi) composes into maps of the same form
    y -> min(max(y + A, B), C), so the recursion is evaluated with a
    log-step prefix composition (exact integers, vectorised)."""
    steps = np.asarray(steps, dtype=np.int64)
    A = steps.copy()
    B = np.full_like(A, lo)
    C = np.full_like(A, hi)
    n = A.shape[0]
    k = 1
    while k < n:
        # compose earlier map (t-k) then later map (t) for t >= k
        a1, b1, c1 = A[:-k], B[:-k], C[:-k]
        a2, b2, c2 = A[k:], B[k:], C[k:]
        nA = a1 + a2
        nC = np.minimum(np.maximum(c1 + a2, b2), c2)
        nB = np.minimum(np.maximum(b1 + a2, b2), nC)
        A = np.concatenate([A[:k], nA])
        B = np.concatenate([B[:k], nB])
        C = np.concatenate([C[:k], nC])
        k *= 2
    return np.minimum(np.maximum(start + A, B), C)


def walk_int8(rows: int = 65536, D: int = 1, sigma: float = 2.0, const_frac: float = 0.15,
              seed: int = 0) -> np.ndarray:
    """int8 random walk from 0 with rint(N(0, sigma)) steps clipped to the
    int8 range; ``const_frac`` of the rows lie in constant runs."""
    rng = np.random.default_rng(seed)
    inc = np.rint(rng.normal(0.0, sigma, size=(rows, D))).astype(np.int64)
    mask = _run_mask(rng, rows, const_frac)
    inc[mask] = 0
    x = clipped_walk(0, inc, -128, 127)
    return x.astype(np.int8)


def ar2_uint16(rows: int = 4194304, D: int = 8, sigma: float = 20.0, flat_frac: float = 0.20,
               seed: int = 1) -> np.ndarray:
    """uint16 columns y_t = 1.6 y_{t-1} - 0.7 y_{t-2} + N(0, sigma), offset by
    32768 and clipped; ``flat_frac`` of the rows repeat the previous row in
    every column."""
    rng = np.random.default_rng(seed)
    noise = rng.normal(0.0, sigma, size=(rows, D))
    y = lfilter([1.0], [1.0, -1.6, 0.7], noise, axis=0)
    x = np.clip(np.rint(y) + 32768, 0, 65535).astype(np.uint16)
    mask = _run_mask(rng, rows, flat_frac)
    src = np.where(mask, 0, np.arange(rows))
    src = np.maximum.accumulate(src) if rows else src
    return np.ascontiguousarray(x[src])


def uniform(rows: int, D: int, dtype, seed: int = 5) -> np.ndarray:
    """Full-range uniform values: the paper's incompressible speed workload."""
    rng = np.random.default_rng(seed)
    info = np.iinfo(dtype)
    return rng.integers(info.min, info.max + 1, size=(rows, D), dtype=np.int64).astype(dtype)


def laplace_walk_uint16(rows: int, D: int = 4, scale: float = 3.0, seed: int = 3) -> np.ndarray:
    """uint16 walks from 32768 with rint(Laplace(0, scale)) steps, wrapping
    modulo 2^16."""
    rng = np.random.default_rng(seed)
    inc = np.rint(rng.laplace(0.0, scale, size=(rows, D))).astype(np.int64)
    x = (32768 + np.cumsum(inc, axis=0)) % 65536
    return x.astype(np.uint16)


def batch_stream_params(k: int) -> tuple[int, int, np.dtype, float]:
    """(rows, D, dtype, sigma) of stream k of the batch workload: rows
    log-uniform in [1e3, 1e6), D uniform in {1,2,4,8,16}, even k int8 and odd
    k uint16, noise sigma log-uniform in [0.5, 200)."""
    rng = np.random.default_rng(2_000_000 + k)
    rows = int(np.floor(np.exp(rng.uniform(np.log(1e3), np.log(1e6)))))
    D = int(rng.choice([1, 2, 4, 8, 16]))
    sigma = float(np.exp(rng.uniform(np.log(0.5), np.log(200.0))))
    dt = np.dtype(np.int8) if k % 2 == 0 else np.dtype(np.uint16)
    return rows, D, dt, sigma


def batch_stream(k: int, max_rows: int | None = None) -> np.ndarray:
    """Stream k of the batch workload (generators of the two single-stream
    workloads with the stream's own sigma). ``max_rows`` truncates."""
    rows, D, dt, sigma = batch_stream_params(k)
    if max_rows is not None:
        rows = min(rows, max_rows)
    if dt == np.int8:
        return walk_int8(rows, D, sigma=sigma, seed=3_000_000 + k)
    return ar2_uint16(rows, D, sigma=sigma, seed=3_000_000 + k)


# ---------------------------------------------------------------------------
# The same recipes drawn on a GPU with torch (seeded torch generators; the
# numbers differ from the numpy draws above, the distributions do not). Used
# for the 10,000-stream batch workload, whose 13.5 GB would take an hour to
# draw on the CPU.
# ---------------------------------------------------------------------------
def _torch_run_mask(n: int, coverage: float, gen, device, lo: int = 8, hi: int = 256):
    """Boolean mask of runs of U{lo..hi} positions at uniform random starts,
    added in rounds until at least ``coverage`` of n is covered."""
    import torch
    mask = torch.zeros(n, dtype=torch.bool, device=device)
    if n == 0 or coverage <= 0:
        return mask
    while int(mask.sum().item()) < coverage * n:
        need = coverage * n - int(mask.sum().item())
        m = max(1, int(need / ((lo + hi) / 2)) + 1)
        starts = torch.randint(0, n, (m,), generator=gen, device=device)
        lens = torch.randint(lo, hi + 1, (m,), generator=gen, device=device)
        diff = torch.zeros(n + 1, dtype=torch.int32, device=device)
        diff.index_add_(0, starts, torch.ones(m, dtype=torch.int32, device=device))
        diff.index_add_(0, torch.clamp(starts + lens, max=n), -torch.ones(m, dtype=torch.int32, device=device))
        mask |= torch.cumsum(diff[:n], 0) > 0
    return mask


def clipped_walk_torch(steps, lo: int, hi: int):
    """x_t = clip(x_{t-1} + steps_t, lo, hi) from x_{-1} = 0 along dim 0, by a
    Hillis-Steele scan over the maps x -> clip(x + a, l, h), which compose as
    (a1, l1, h1) then (a2, l2, h2) = (a1 + a2, clip(l1 + a2, l2, h2),
    clip(h1 + a2, l2, h2))."""
    import torch
    a = steps.to(torch.int64)
    L = torch.full_like(a, lo)
    H = torch.full_like(a, hi)
    n = a.shape[0]
    d = 1
    while d < n:
        a2, L2, H2 = a[d:], L[d:], H[d:]
        a1, L1, H1 = a[:-d], L[:-d], H[:-d]
        na = a1 + a2
        nL = torch.minimum(torch.maximum(L1 + a2, L2), H2)
        nH = torch.minimum(torch.maximum(H1 + a2, L2), H2)
        a = torch.cat([a[:d], na])
        L = torch.cat([L[:d], nL])
        H = torch.cat([H[:d], nH])
        d *= 2
    return torch.minimum(torch.maximum(a, L), H)


def walk_int8_torch(rows: int, D: int, sigma: float, const_frac: float, gen, device):
    import torch
    steps = torch.round(torch.randn((rows, D), generator=gen, device=device) * sigma)
    mask = _torch_run_mask(rows, const_frac, gen, device)
    steps[mask] = 0
    return clipped_walk_torch(steps, -128, 127).to(torch.int8).contiguous()


def ar2_filter_torch(e):
    """y_t = 1.6 y_{t-1} - 0.7 y_{t-2} + e_t along dim 0 from y = 0 (float64),
    as an inclusive Hillis-Steele scan of the state s_t = (y_t, y_{t-1}) =
    A s_{t-1} + (e_t, 0): after step j, v_t = sum_{k < 2^j} A^k u_{t-k}."""
    import torch
    n = e.shape[0]
    v0 = e.to(torch.float64)                 # first state component
    v1 = torch.zeros_like(v0)                # second state component
    P = [[1.6, -0.7], [1.0, 0.0]]            # A^(2^j)
    d = 1
    while d < n:
        a, b, c, dd = P[0][0], P[0][1], P[1][0], P[1][1]
        s0 = a * v0[:-d] + b * v1[:-d]
        s1 = c * v0[:-d] + dd * v1[:-d]
        v0 = torch.cat([v0[:d], v0[d:] + s0])
        v1 = torch.cat([v1[:d], v1[d:] + s1])
        P = [[a * a + b * c, a * b + b * dd], [c * a + dd * c, c * b + dd * dd]]
        d *= 2
    return v0


def ar2_uint16_torch(rows: int, D: int, sigma: float, flat_frac: float, gen, device):
    import torch
    burn = 256   # the filter forgets its zero start: |root| = 0.837, 0.837^256 < 1e-19
    e = torch.randn((rows + burn, D), generator=gen, device=device, dtype=torch.float64) * sigma
    y = ar2_filter_torch(e)[burn:]
    x = torch.clamp(torch.round(y) + 32768, 0, 65535).to(torch.int32)
    flat = _torch_run_mask(rows, flat_frac, gen, device)
    if rows:
        idx = torch.arange(rows, device=device)
        idx = torch.where(flat, torch.zeros_like(idx), idx)
        idx = torch.cummax(idx, 0).values
        x = x[idx]
    return x.to(torch.int16).contiguous()   # uint16 bit patterns


def wrap_walk_torch(steps, start: int = 32768):
    """x_t = (start + steps_0 + ... + steps_t) mod 2^16 per column, as int16
    bit patterns (the wrapping random walk of the entropy workload)."""
    import torch
    x = torch.cumsum(steps.to(torch.int64), dim=0) + start
    return torch.remainder(x, 65536).to(torch.int32).to(torch.int16)


def laplace_walk_uint16_torch(rows: int, D: int, scale: float, gen, device, chunk: int = 1 << 25):
    """``laplace_walk_uint16`` drawn on the GPU in row chunks: steps
    rint(Laplace(0, scale)) by the inverse CDF of a uniform draw, wrapped
    walks from 32768 (scans run column by column along contiguous memory).
    Returns int16 bit patterns."""
    import torch
    out = torch.empty((rows, D), dtype=torch.int16, device=device)
    carry = torch.full((D, 1), 32768, dtype=torch.int64, device=device)
    for r0 in range(0, rows, chunk):
        n = min(chunk, rows - r0)
        u = torch.rand((D, n), generator=gen, device=device, dtype=torch.float64) - 0.5
        inc = torch.round(-scale * torch.sign(u) * torch.log1p(-2.0 * u.abs())).to(torch.int64)
        x = torch.cumsum(inc, dim=1) + carry
        out[r0:r0 + n] = torch.remainder(x, 65536).to(torch.int32).to(torch.int16).t()
        carry = x[:, -1:].clone()
    return out


def batch_stream_torch(k: int, device="cuda"):
    """Stream k of the batch workload drawn on the GPU (same rows, D, dtype
    and sigma as ``batch_stream_params(k)``); uint16 streams come back as
    int16 tensors holding the uint16 bit patterns."""
    import torch
    rows, D, dt, sigma = batch_stream_params(k)
    gen = torch.Generator(device=device)
    gen.manual_seed(3_000_000 + k)
    if dt == np.int8:
        return walk_int8_torch(rows, D, sigma, 0.15, gen, device)
    return ar2_uint16_torch(rows, D, sigma, 0.20, gen, device)

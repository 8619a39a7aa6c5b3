"""Seeded synthetic inputs for the paper's workloads.

This module holds no FFT or decomposition arithmetic: it only draws random
numbers, so both the GPU path's tests and the oracle can be fed the very same
values.  Seeds are ``numpy.random.Generator(PCG64(13026189 + k))``.

Workloads (the paper measures no data set; these stand in for its N x N x N,
N^4 and N^5 arrays of complex points):

* ``uniform``      re, im i.i.d. U[-1, 1)
* ``gaussian``     re, im i.i.d. N(0, 1)
* ``log_uniform``  re = +-10^u, im = +-10^v, u, v ~ U[-6, 0), random signs
* ``batch_items``  mixed 3-D/4-D/5-D items, every size drawn from the
                   2^a 3^b 5^c values in [12, 192], total points <= 2^22,
                   N_p uniform in [1, 64]
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 13026189


def rng(k: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + int(k)))


def uniform(shape, seed: int, dtype=np.complex64) -> np.ndarray:
    """re, im i.i.d. U[-1, 1), drawn in float64 then cast to ``dtype``."""
    g = rng(seed)
    n = int(np.prod(shape))
    out = np.empty(n, dtype=dtype)
    real_dt = np.float32 if dtype == np.complex64 else np.float64
    view = out.view(real_dt).reshape(n, 2)
    step = 1 << 24
    for s in range(0, n, step):
        e = min(n, s + step)
        view[s:e] = g.uniform(-1.0, 1.0, size=(e - s, 2)).astype(real_dt)
    return out.reshape(shape)


def gaussian(shape, seed: int, dtype=np.complex64) -> np.ndarray:
    """re, im i.i.d. N(0, 1), drawn in float64 then cast to ``dtype``."""
    g = rng(seed)
    n = int(np.prod(shape))
    out = np.empty(n, dtype=dtype)
    real_dt = np.float32 if dtype == np.complex64 else np.float64
    view = out.view(real_dt).reshape(n, 2)
    step = 1 << 24
    for s in range(0, n, step):
        e = min(n, s + step)
        view[s:e] = g.standard_normal(size=(e - s, 2)).astype(real_dt)
    return out.reshape(shape)


def log_uniform(shape, seed: int, dtype=np.complex64) -> np.ndarray:
    """re = +-10^u, im = +-10^v with u, v ~ U[-6, 0) and random signs."""
    g = rng(seed)
    n = int(np.prod(shape))
    out = np.empty(n, dtype=dtype)
    real_dt = np.float32 if dtype == np.complex64 else np.float64
    view = out.view(real_dt).reshape(n, 2)
    step = 1 << 24
    for s in range(0, n, step):
        e = min(n, s + step)
        mag = 10.0 ** g.uniform(-6.0, 0.0, size=(e - s, 2))
        sgn = np.where(g.random(size=(e - s, 2)) < 0.5, -1.0, 1.0)
        view[s:e] = (mag * sgn).astype(real_dt)
    return out.reshape(shape)


# the 36 values 2^a 3^b 5^c in [12, 192]
SMOOTH_SIZES = sorted({2 ** a * 3 ** b * 5 ** c
                       for a in range(8) for b in range(5) for c in range(4)
                       if 12 <= 2 ** a * 3 ** b * 5 ** c <= 192})


def batch_items(n_items: int = 256, seed: int = 5, max_points: int = 1 << 22):
    """List of (dims, P) for the batched workload.

    M ~ U{3, 4, 5}; each size ~ U over SMOOTH_SIZES; an item whose point count
    exceeds ``max_points`` is redrawn; P ~ U{1..64}, not capped.  (With every
    size >= 12 and M >= 3 an item has at least 144 rows along any axis, so
    P <= 64 never reaches the row-split level M of Eq. (13).)
    """
    g = rng(seed)
    items = []
    while len(items) < n_items:
        M = int(g.integers(3, 6))
        dims = tuple(int(SMOOTH_SIZES[i]) for i in g.integers(0, len(SMOOTH_SIZES), size=M))
        if int(np.prod(dims)) > max_points:
            continue
        P = int(g.integers(1, 65))
        items.append((dims, P))
    return items

"""Host logic of the order study: the canonical order table, the relabelling
that turns any transpose into a first transpose, and order completion."""
import itertools

import numpy as np
import pytest

from oracle import decomp, orders
from paper_1302_6189_amd import fftrw, order_study


@pytest.mark.parametrize("M", [3, 4, 5])
def test_table_is_canonical(M):
    perms, seq = order_study.order_table(M)
    assert len(seq) == fftrw.fft_order_count(M)
    rng = np.random.default_rng(M)
    for i in list(rng.integers(0, len(seq), 100)) + [0, len(seq) - 1]:
        assert tuple(perms[j] for j in seq[i]) == tuple(fftrw.fft_order_at(M, int(i)))


def test_relabelling_preserves_the_amount():
    # checked against the oracle's point-by-point count on unequal sizes
    dims, P = (6, 4, 5, 3), 7
    perms = list(itertools.permutations(range(4)))
    rng = np.random.default_rng(3)
    for _ in range(25):
        a, b = (perms[i] for i in rng.choice(len(perms), 2, replace=False))
        if a[-1] == b[-1]:
            continue
        D, sig = order_study.relabel(dims, a, b)
        assert decomp.pair_volume(dims, P, a, b) == decomp.pair_volume(D, P, tuple(range(4)), sig)


@pytest.mark.parametrize("M", [3, 4, 5])
def test_completed_orders_are_valid(M):
    for s in itertools.permutations(range(M)):
        if s[-1] == M - 1:
            continue
        o = order_study.complete_order(M, s)
        assert o[1] == s and orders.is_valid_order(o, M)


def test_composition_sums_the_stages():
    perms, seq = order_study.order_table(3)
    X = np.arange(36, dtype=float).reshape(6, 6)
    F = np.array([100.0, 200, 300, 400, 500, 600])
    t = order_study.composed_times(seq, X, F)
    for i, row in enumerate(seq):
        want = sum(F[r] for r in row) + sum(X[row[k], row[k + 1]] for k in range(2)) + X[row[-1], 0]
        assert t[i] == want

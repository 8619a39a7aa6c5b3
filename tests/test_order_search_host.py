"""The library's order search (a dynamic program over the current
decomposition and the axes already transformed) against exhaustive
enumeration for 5-D, and for 6-D -- where the 2,985,984,000,000 orders cannot
be listed -- against the oracle's amounts of the orders it returns, the
closed forms of the 1-D regime, random orders, and the 3+3 family of
Section 3.3."""
import itertools
import math

import numpy as np
import pytest

from oracle import decomp, orders
from paper_1302_6189_amd import fftrw
from tests.test_oracle_claims import order_table


def _perm_index(M):
    return {p: i for i, p in enumerate(itertools.permutations(range(M)))}


def _oracle_pairs(dims, P, ownership="literal"):
    """Point-by-point amounts of every transpose between two permutations
    with different last axes (lexicographic permutation indices)."""
    M = len(dims)
    perms = list(itertools.permutations(range(M)))
    fn = decomp.pair_volume if ownership == "literal" else decomp.pair_volume_matched
    tab = np.full((len(perms), len(perms)), -1, dtype=np.int64)
    for a, pa in enumerate(perms):
        for b, pb in enumerate(perms):
            if pa[-1] != pb[-1]:
                tab[a, b] = fn(dims, P, pa, pb)
    return tab


def _order_amount(tab, order, M):
    idx = _perm_index(M)
    return int(sum(tab[idx[order[t]], idx[order[t + 1]]] for t in range(M - 1)))


@pytest.mark.parametrize("dims,P,own", [((2, 3, 2, 2, 3), 7, "literal"), ((3, 2, 2, 2, 2), 20, "literal"),
                                        ((2, 2, 3, 2, 2), 12, "matched")])
def test_five_d_search_matches_exhaustive(dims, P, own):
    M = 5
    tab = _oracle_pairs(dims, P, own)
    _, seq = order_table(M)
    seq = seq[np.lexsort(seq.T[::-1])]          # canonical order: lexicographic in permutation indices
    tot = sum(tab[seq[:, t], seq[:, t + 1]] for t in range(M - 1))
    assert len(tot) == fftrw.fft_order_count(M)
    r = fftrw.fft_order_search(dims, P, ownership=fftrw.OWN_LITERAL if own == "literal" else fftrw.OWN_MATCHED)
    assert r["best_volume"] == tot.min() and r["worst_volume"] == tot.max()
    assert r["n_best"] == np.count_nonzero(tot == tot.min()) and r["n_worst"] == np.count_nonzero(tot == tot.max())
    assert r["best_index"] == int(np.argmin(tot)) and r["worst_index"] == int(np.argmax(tot))


def _random_orders(M, n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        order, used = [tuple(range(M))], {M - 1}
        for _t in range(M - 1):
            while True:
                p = tuple(int(a) for a in rng.permutation(M))
                if p[-1] not in used:
                    break
            used.add(p[-1])
            order.append(p)
        out.append(tuple(order))
    return out


@pytest.mark.parametrize("dims,P", [((2, 2, 2, 2, 2, 2), 6), ((2, 3, 2, 2, 3, 2), 20), ((4, 4, 4, 4, 4, 4), 64),
                                    ((3, 2, 4, 2, 2, 3), 100)])
def test_six_d_search_against_oracle_amounts(dims, P):
    M = 6
    r = fftrw.fft_order_search(dims, P)
    for key, vol in (("best_order", "best_volume"), ("worst_order", "worst_volume")):
        o = r[key]
        assert orders.is_valid_order(o, M)
        steps, _ = decomp.order_volumes(dims, P, o)
        assert sum(steps) == r[vol]
        assert fftrw.fft_order_index(o) == r[key.replace("order", "index")]
    assert 1 <= r["n_best"] <= fftrw.fft_order_count(M)
    # no random order beats the optimum or exceeds the worst
    tab = fftrw.fft_transpose_volumes(dims, P)
    for o in _random_orders(M, 300, P):
        v = _order_amount(tab, o, M)
        assert r["best_volume"] <= v <= r["worst_volume"]
    # the library's table agrees with the oracle on a sample of transposes
    perms = list(itertools.permutations(range(M)))
    rng = np.random.default_rng(P)
    for _ in range(40):
        a, b = (int(i) for i in rng.integers(0, len(perms), 2))
        if tab[a, b] >= 0:
            assert tab[a, b] == decomp.pair_volume(dims, P, perms[a], perms[b])


@pytest.mark.parametrize("dims,P", [((4,) * 6, 2), ((4,) * 6, 4), ((2, 4, 6, 4, 2, 8), 2)])
def test_six_d_one_d_regime_closed_forms(dims, P):
    # every decomposition splits its leading axis (N_p divides it): a
    # transpose keeping the leading axis moves nothing, one changing it moves
    # T - T/N_p; the best order changes it once, the worst at every step
    T = math.prod(dims)
    r = fftrw.fft_order_search(dims, P)
    assert r["best_volume"] == T - T // P
    assert r["worst_volume"] == 5 * (T - T // P)


def test_six_d_optimum_is_the_three_plus_three_family():
    # 4^6 over 64 processes: the optimal orders are exactly the 2,304 orders of
    # the 3+3 form the paper expects for 6-D
    dims, P = (4,) * 6, 64
    r = fftrw.fft_order_search(dims, P)
    fam = orders.form_orders(6, 3)
    assert r["n_best"] == len(fam) == 2304
    # oracle amounts through the relabelling symmetry of equal sizes
    ident = tuple(range(6))
    cache = {}

    def amount(a, b):
        inv = [0] * 6
        for i, ax in enumerate(a):
            inv[ax] = i
        rho = tuple(inv[x] for x in b)
        if rho not in cache:
            cache[rho] = decomp.pair_volume(dims, P, ident, rho)
        return cache[rho]

    for o in fam:
        assert sum(amount(o[t], o[t + 1]) for t in range(5)) == r["best_volume"]

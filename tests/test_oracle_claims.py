"""The oracle against the numbers the paper prints (Sections 3.1, 3.3, 4).

For an array with equal sizes N in every axis, relabelling the axes maps
decompositions onto each other, so the amount of a transpose pi -> sigma
equals that of identity -> pi^{-1} o sigma.  The studies below use this to
evaluate each distinct pair once; the symmetry itself is checked first.
"""
import itertools
import os
import random

import numpy as np
import pytest

from oracle import decomp, orders

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _claims():
    out = {}
    with open(os.path.join(GOLDEN, "paper_claims.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()[:2]
                out[k] = float(v)
    return out


def _listed(M):
    with open(os.path.join(GOLDEN, "paper_best_orders.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    return [orders.parse_order(s) for m, s in rows if int(m) == M]


def _relabel(a, b):
    inv = [0] * len(a)
    for i, ax in enumerate(a):
        inv[ax] = i
    return tuple(inv[x] for x in b)


_ORDER_CACHE = {}


def order_table(M):
    """Every valid order as a row of permutation indices (numpy), built stage
    by stage: a later stage may use any permutation whose last axis is unused."""
    if M not in _ORDER_CACHE:
        perms = list(itertools.permutations(range(M)))
        seq = np.zeros((1, 1), dtype=np.int16)  # the natural order is permutation 0
        used = np.array([1 << (M - 1)], dtype=np.int64)
        for _ in range(1, M):
            parts, uparts = [], []
            for pi, p in enumerate(perms):
                ok = (used & (1 << p[-1])) == 0
                rows = seq[ok]
                parts.append(np.hstack([rows, np.full((len(rows), 1), pi, dtype=np.int16)]))
                uparts.append(used[ok] | (1 << p[-1]))
            seq, used = np.vstack(parts), np.concatenate(uparts)
        _ORDER_CACHE[M] = (perms, seq)
    return _ORDER_CACHE[M]


class Study:
    def __init__(self, perms, seq, res):
        self.perms, self.seq, self.res = perms, seq, res

    def order(self, row):
        return tuple(self.perms[i] for i in self.seq[row])

    def index_of(self, order):
        idx = [self.perms.index(p) for p in order]
        hit = np.flatnonzero((self.seq == np.array(idx, dtype=np.int16)).all(axis=1))
        return int(hit[0])


_STUDIES = {}


def study(M, N, Ps, ownership="literal"):
    """Total amount of every order of an N^M array for each N_p (memoised)."""
    key = (M, N, tuple(Ps), ownership)
    if key not in _STUDIES:
        _STUDIES[key] = _study(M, N, Ps, ownership)
    return _STUDIES[key]


def _study(M, N, Ps, ownership):
    dims = (N,) * M
    ident = tuple(range(M))
    fn = decomp.pair_volume if ownership == "literal" else decomp.pair_volume_matched
    perms, seq = order_table(M)
    res = {}
    for P in Ps:
        cache = {}
        pv = np.zeros((len(perms), len(perms)), dtype=np.int64)
        for a in range(len(perms)):
            for b in range(len(perms)):
                if perms[a][-1] == perms[b][-1]:
                    continue
                c = _relabel(perms[a], perms[b])
                if c not in cache:
                    cache[c] = fn(dims, P, ident, c)
                pv[a, b] = cache[c]
        tot = np.zeros(len(seq), dtype=np.int64)
        for t in range(M - 1):
            tot += pv[seq[:, t], seq[:, t + 1]]
        res[P] = tot
    return Study(perms, seq, res)


@pytest.mark.parametrize("M,N,P", [(3, 6, 5), (3, 8, 48), (4, 4, 20), (5, 3, 30)])
def test_relabelling_symmetry(M, N, P):
    perms = list(itertools.permutations(range(M)))
    rng = random.Random(M * 100 + P)
    dims = (N,) * M
    for _ in range(6):
        a, b = rng.sample(perms, 2)
        assert decomp.pair_volume(dims, P, a, b) == decomp.pair_volume(dims, P, tuple(range(M)), _relabel(a, b))


def test_order_table_matches_table1():
    with open(os.path.join(GOLDEN, "table1_order_counts.txt")) as f:
        t1 = {int(l.split()[0]): int(l.split()[1]) for l in f if l.strip() and not l.startswith("#")}
    for M in (3, 4, 5):
        perms, seq = order_table(M)
        assert len(seq) == t1[M] and len({tuple(r) for r in seq.tolist()}) == t1[M]
        for r in seq[:: max(1, len(seq) // 500)]:
            assert orders.is_valid_order(tuple(perms[i] for i in r), M)


def test_three_d_ratios():
    c = _claims()
    N = 64
    res = study(3, N, list(range(2, N + 1)) + [128, 256, 512, 1024, 2048, 4096]).res
    for P, v in res.items():
        r = max(v) / min(v)
        if P <= N:
            assert r == c["ratio3d_upto_N"], P          # "twice" for N_p <= N, ragged N_p too
    upper = max(max(res[P]) / min(res[P]) for P in res if N < P <= N * N)
    assert round(upper, 1) == c["ratio3d_N_to_N2_max"]


def test_four_d_ratios():
    c = _claims()
    N = 8
    res = study(4, N, [2 ** i for i in range(1, 10)]).res
    for P, v in res.items():
        if P <= N * N:
            assert max(v) / min(v) == c["ratio4d_upto_N2"]
    upper = max(max(res[P]) / min(res[P]) for P in res if N * N < P <= N ** 3)
    assert round(upper, 1) == c["ratio4d_N2_to_N3_max"]


def test_five_d_ratios():
    c = _claims()
    N = 8
    res = study(5, N, [2 ** i for i in range(1, 13)]).res
    for P, v in res.items():
        if P <= N * N:
            assert max(v) / min(v) == c["ratio5d_upto_N2"]
    mid = [max(res[P]) / min(res[P]) for P in res if N * N < P <= N ** 3]
    assert round(min(mid), 1) == c["ratio5d_N2_to_N3_min"]
    assert round(max(mid), 1) == c["ratio5d_N2_to_N3_max"]
    top = max(max(res[P]) / min(res[P]) for P in res if N ** 3 < P <= N ** 4)
    assert round(top, 1) == c["ratio5d_N3_to_N4_max"]


def _always_best(st):
    mask = np.ones(len(st.seq), dtype=bool)
    for v in st.res.values():
        mask &= v == v.min()
    return {st.order(i) for i in np.flatnonzero(mask)}


def test_matched_always_best_three_d():
    assert _always_best(study(3, 8, [2 ** i for i in range(1, 7)], "matched")) == set(_listed(3))


def test_matched_always_best_four_d():
    assert _always_best(study(4, 8, [2 ** i for i in range(1, 10)], "matched")) == set(_listed(4))


def test_matched_always_best_five_d():
    c = _claims()
    best = _always_best(study(5, 4, [2 ** i for i in range(1, 9)], "matched"))
    assert len(best) == c["count5d_always_best"]
    assert set(_listed(5)) <= best


def test_always_best_sets_have_the_balanced_forms():
    # Section 3.3 describes the best orders by their shape: 1+2 or 2+1 for
    # 3-D, 2+2 (neither 1+3 nor 3+1) for 4-D, 2+3 or 3+2 for 5-D.  Under the
    # matched reading: the always-best 3-D set is exactly F(1+2) + F(2+1), the
    # 4-D set exactly F(2+2); the 96 always-best 5-D orders are 48 of F(2+3)
    # and 48 of F(3+2), and none has an unbalanced form.
    fam = {(M, m1): set(orders.form_orders(M, m1)) for M in (3, 4, 5) for m1 in range(1, M)}
    b3 = _always_best(study(3, 8, [2 ** i for i in range(1, 7)], "matched"))
    assert b3 == fam[3, 1] | fam[3, 2]
    b4 = _always_best(study(4, 8, [2 ** i for i in range(1, 10)], "matched"))
    assert b4 == fam[4, 2] and not b4 & (fam[4, 1] | fam[4, 3])
    b5 = _always_best(study(5, 4, [2 ** i for i in range(1, 9)], "matched"))
    assert len(b5 & fam[5, 2]) == len(b5 & fam[5, 3]) == 48
    assert b5 <= fam[5, 2] | fam[5, 3]
    assert set(_listed(5)) <= fam[5, 2] and set(_listed(4)) == fam[4, 2]


def test_literal_reading_does_not_give_the_listed_sets():
    # recorded for the readings table: under R1 the listed 3-D orders split
    # into two exactly-best and two within 1% (N = 64, N_p = 128)
    st = study(3, 64, [128])
    v = st.res[128]
    listed = [st.index_of(o) for o in _listed(3)]
    best = min(v)
    assert sorted(v[i] == best for i in listed) == [False, False, True, True]
    assert all(v[i] / best < 1.01 for i in listed)


def test_comparison_with_two_d_method():
    c = _claims()
    N = 64
    res = study(3, N, [16, 32, 64, 2048, 4096]).res
    gain = {P: decomp.amount_2d_method(N, P) / min(v) - 1 for P, v in res.items()}
    assert round(100 * gain[16], 1) == c["vs2d_64cube_min_percent"]
    assert round(100 * gain[64], 1) == c["vs2d_64cube_max_percent"]
    assert all(c["vs2d_64cube_min_percent"] <= round(100 * gain[P], 1) <= c["vs2d_64cube_max_percent"]
               for P in (16, 32, 64))
    for P in (2048, 4096):
        assert P >= c["vs2d_64cube_gap_zero_from"] and gain[P] < 0.005


def test_comparison_with_three_d_method_row_split():
    # Section 4: beyond 4,096 processes only the 3-D method (Eq. (23)) and this
    # one work on 64^3, and every decomposition is at level M.  With the split
    # rows' own FFTs done by binary exchange (ceil(log2 c) all-point stages for
    # a row over c processes) the advantage peaks at 8,192 processes, 11.6x.
    c = _claims()
    N = 64
    dims = (N, N, N)
    Ps = [8192 * 2 ** j for j in range(6)]
    st = study(3, N, Ps)
    ratio = {}
    for P in Ps:
        split = {p: decomp.split_row_volume(dims, P, p) for p in st.perms}
        tot = st.res[P] + np.array([sum(split[st.perms[i]] for i in row) for row in st.seq])
        ratio[P] = decomp.amount_3d_method(N, P) / tot.min()
    assert round(ratio[8192], 1) == c["vs3d_64cube_max_at_8192"]
    assert max(ratio, key=ratio.get) == 8192
    # the transposes alone would give 29.2x: the split rows' exchanges matter
    assert round(decomp.amount_3d_method(N, 8192) / st.res[8192].min(), 1) == 29.2


def test_comparison_with_four_d_method():
    c = _claims()
    N = 16
    res = study(4, N, [2 ** i for i in range(1, 13)]).res
    best_ratio = max(decomp.amount_4d_method(N, P) / min(v) for P, v in res.items())
    assert round(best_ratio) == c["vs4d_16pow4_max"]

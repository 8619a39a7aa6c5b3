"""Pins for the decomposition and communication-amount oracle (Section 3).

Checked against: the structure Eqs. (4)-(19) imply (partition, balance,
whole rows, minimal level), hand-worked small cases, the closed forms of the
1-D regime, Eq. (21) (the slab method's amount), and brute force.
"""
import itertools
from math import prod

import numpy as np
import pytest

from oracle import decomp, orders, pipeline


def _perms(M):
    return list(itertools.permutations(range(M)))


@pytest.mark.parametrize("dims,P", [((4, 3, 5), 1), ((4, 3, 5), 3), ((4, 3, 5), 4), ((4, 3, 5), 5),
                                    ((4, 3, 5), 12), ((4, 3, 5), 13), ((4, 3, 5), 60),
                                    ((6, 6, 6, 6), 7), ((6, 6, 6, 6), 48), ((6, 6, 6, 6), 216),
                                    ((2, 3, 2, 5, 2), 9), ((2, 3, 2, 5, 2), 100)])
def test_ranges_partition_and_balance(dims, P):
    T = prod(dims)
    for perm in _perms(len(dims)):
        pd = [dims[a] for a in perm]
        k = decomp.level(pd, P)
        R = prod(pd[:k])
        # level is minimal (the cases of Eq. (13))
        assert P <= R and (k == 1 or P > prod(pd[:k - 1]))
        W = prod(pd[k:])
        prev_end = -1
        for p in range(P):
            xs, xe = decomp.local_range(pd, P, p)
            assert xs == prev_end + 1          # contiguous, in process order
            prev_end = xe
            n = xe - xs + 1
            assert n % W == 0                  # whole rows over the first k axes
            assert n // W in (R // P, -(-R // P))  # floor or ceil of R/N_p rows
        assert prev_end == T - 1


def test_worked_case_2d_decomposition():
    # Eqs. (10)-(11): N_1 < N_p <= N_1 N_2 in abc order -> whole c-lines;
    # N = (4, 3, 5), N_p = 6 gives 12 (a, b) rows, two per process.
    dims, P = (4, 3, 5), 6
    got = [decomp.decomp(dims, P, (0, 1, 2), p) for p in range(P)]
    assert [g[0] for g in got] == [2] * P
    # process 0: rows (0,0),(0,1) -> points 0..9; process 5: rows (3,1),(3,2)
    assert got[0][1:] == (0, 9, (0, 0, 0), (0, 1, 4))
    assert got[1][1:] == (10, 19, (0, 2, 0), (1, 0, 4))
    assert got[5][1:] == (50, 59, (3, 1, 0), (3, 2, 4))
    for (_k, _xs, _xe, s, e) in got:
        assert s[2] == 0 and e[2] == dims[2] - 1   # from X(a_s, b_s, 0) to X(a_e, b_e, N_3 - 1)


def test_worked_case_1d_decomposition():
    # N_p <= N_1: blocks of complete bc-planes (slab), Eq. (4) first case
    dims, P = (8, 3, 5), 3
    got = [decomp.decomp(dims, P, (0, 1, 2), p) for p in range(P)]
    # floor(8p/3) = 0, 2, 5, 8 -> a-ranges [0,1], [2,4], [5,7]
    assert [(g[3][0], g[4][0]) for g in got] == [(0, 1), (2, 4), (5, 7)]
    for (k, _xs, _xe, s, e) in got:
        assert k == 1 and s[1:] == (0, 0) and e[1:] == (2, 4)


def test_start_end_round_trip():
    dims = (5, 6, 7, 4)
    for perm in _perms(4)[:6]:
        pd = [dims[a] for a in perm]
        for P in (3, 7, 31, 200, 839):
            for p in range(P):
                k, xs, xe, s, e = decomp.decomp(dims, P, perm, p)
                back_s = sum(s[r] * prod(pd[r + 1:]) for r in range(4))
                back_e = sum(e[r] * prod(pd[r + 1:]) for r in range(4))
                assert (back_s, back_e) == (xs, xe)


def test_level_m_refused():
    with pytest.raises(decomp.RowSplitError):
        decomp.level([4, 4, 4], 65)
    # P = T is still level 3 (every point its own process) -- allowed by Eq. (13)
    assert decomp.level([4, 4, 4], 64) == 3


def test_owners_brute_force():
    dims, P = (4, 6, 5), 7
    for perm in _perms(3):
        own = decomp.owners(dims, P, perm)
        b = decomp.boundaries(dims, P, perm)
        pd = [dims[a] for a in perm]
        for idx in np.ndindex(*dims):
            x = sum(idx[perm[r]] * prod(pd[r + 1:]) for r in range(3))
            p = [q for q in range(P) if b[q] <= x < b[q + 1]]
            assert p == [own[idx]]


def _one_d_closed_form(N, M, P):
    # a transpose that changes the leading axis moves T - (T/N^2) sum_p n_p^2
    T = N ** M
    n = [(N * (p + 1)) // P - (N * p) // P for p in range(P)]
    return T - (T // (N * N)) * sum(v * v for v in n)


@pytest.mark.parametrize("N,M", [(8, 3), (12, 3), (6, 4), (4, 5)])
def test_one_d_regime_closed_form(N, M):
    dims = (N,) * M
    for P in range(2, N + 1):
        for a, b in [(p, q) for p in _perms(M) for q in _perms(M) if p[-1] != q[-1]][:40]:
            v = decomp.pair_volume(dims, P, a, b)
            if a[0] == b[0]:
                assert v == 0            # same leading axis: every point stays
            else:
                assert v == _one_d_closed_form(N, M, P)


@pytest.mark.parametrize("N", [8, 16, 64])
def test_best_order_equals_slab_method(N):
    # Eq. (21): A_1D = N^3 - N^3/N_p, matched by the best order when N_p | N
    O = list(orders.all_orders(3))
    for P in [d for d in range(2, N + 1) if N % d == 0]:
        best = min(sum(decomp.order_volumes((N,) * 3, P, o)[0]) for o in O)
        assert best == decomp.amount_1d_method(N, P)


def test_two_d_regime_closed_forms():
    # 3-D, N_p = q N with q | N (canonical indices 0..7), derived by hand from
    # Eqs. (4)-(9): {0,7}: T(1-1/q)+T-N^2 ; {1,5}: T(1-1/q)+T-N^2/q ;
    # {2,6}: 2T-N^2-N^2/q ; {3,4}: 2T-2N^2/q
    N = 16
    T = N ** 3
    O = list(orders.all_orders(3))
    for q in (2, 4, 8, 16):
        P = q * N
        v = [sum(decomp.order_volumes((N,) * 3, P, o)[0]) for o in O]
        assert v[0] == v[7] == T * (q - 1) // q + T - N * N
        assert v[1] == v[5] == T * (q - 1) // q + T - N * N // q
        assert v[2] == v[6] == 2 * T - N * N - N * N // q
        assert v[3] == v[4] == 2 * T - 2 * N * N // q


def test_pair_matrix_sums():
    dims, P = (6, 5, 4, 3), 11
    for a, b in [((0, 1, 2, 3), (0, 1, 3, 2)), ((0, 1, 3, 2), (3, 2, 0, 1)), ((1, 0, 3, 2), (2, 3, 1, 0))]:
        C = decomp.pair_matrix(dims, P, a, b)
        assert C.sum() == prod(dims)
        assert prod(dims) - np.trace(C) == decomp.pair_volume(dims, P, a, b)
        ba, bb = decomp.boundaries(dims, P, a), decomp.boundaries(dims, P, b)
        assert np.array_equal(C.sum(axis=1), np.diff(ba))
        assert np.array_equal(C.sum(axis=0), np.diff(bb))


def test_matched_never_exceeds_literal():
    dims = (6, 6, 6)
    for P in (4, 7, 13, 36, 100):
        for a, b in [((0, 1, 2), (0, 2, 1)), ((0, 2, 1), (1, 2, 0)), ((2, 0, 1), (2, 1, 0))]:
            lit = decomp.pair_volume(dims, P, a, b)
            mat = decomp.pair_volume_matched(dims, P, a, b)
            assert mat <= lit
            # brute force for tiny P: best over all relabellings
            if P <= 7:
                C = decomp.pair_matrix(dims, P, a, b)
                best = max(sum(C[i, s[i]] for i in range(P)) for s in itertools.permutations(range(P)))
                assert mat == prod(dims) - best


def test_32cube_four_process_volumes():
    # 32^3, N_p = 4: slabs of 8 a-planes; a leading-axis change moves 3/4 of T
    dims, P = (32, 32, 32), 4
    O = list(orders.all_orders(3))
    steps = [decomp.order_volumes(dims, P, o)[0] for o in O]
    assert steps[0] == steps[1] == [0, 24576]
    assert steps[5] == steps[7] == [24576, 0]
    assert steps[2] == steps[3] == steps[4] == steps[6] == [24576, 24576]
    for p in range(P):
        assert decomp.decomp(dims, P, (0, 1, 2), p) == (1, 8192 * p, 8192 * p + 8191,
                                                         (8 * p, 0, 0), (8 * p + 7, 31, 31))


def test_permute_layout_is_a_transpose():
    x = np.arange(2 * 3 * 4).reshape(2, 3, 4)
    y = pipeline.permute_layout(x, (0, 1, 2), (2, 0, 1))
    assert y.shape == (4, 2, 3) and y[3, 1, 2] == x[1, 2, 3]
    z = pipeline.permute_layout(y, (2, 0, 1), (1, 2, 0))
    assert z.shape == (3, 4, 2) and z[2, 3, 1] == x[1, 2, 3]


@pytest.mark.parametrize("dims,P,want", [((8, 8, 8), 128, 512), ((8, 8, 8), 512, 1536), ((4, 4, 4, 4), 256, 512),
                                         ((8, 8, 8), 64, 0), ((2, 4, 8, 4), 32, 0)])
def test_split_row_volume_closed_form(dims, P, want):
    # powers of two, equal rows: every row of N points is split over
    # s = P N / T processes and sends N log2(s) points (0 below level M)
    for perm in _perms(len(dims))[:6]:
        assert decomp.split_row_volume(dims, P, perm) == want


def test_split_row_volume_mixed_levels():
    # (8, 4, 2) over 32 processes: rows along 8 are split over 4 processes,
    # along 4 over 2, rows along 2 stay whole (level 2)
    dims, P = (8, 4, 2), 32
    for perm in _perms(3):
        n_last = dims[perm[-1]]
        assert decomp.split_row_volume(dims, P, perm) == {8: 64 * 2, 4: 64 * 1, 2: 0}[n_last]


@pytest.mark.parametrize("dims,P", [((4, 4, 4), 20), ((6, 5, 4), 50), ((3, 4, 2, 5), 77), ((2, 3, 2, 2, 3), 40)])
def test_split_row_volume_from_ranges(dims, P):
    # ragged: processes per row counted from the ranges of Eqs. (14)-(15)
    # (which processes' [x^s, x^e] meet the row), not from point owners
    M = len(dims)
    for perm in _perms(M)[:8]:
        pd = [dims[a] for a in perm]
        N, T = pd[-1], prod(pd)
        rng = [decomp.decomp(dims, P, perm, p)[1:3] for p in range(P)]
        want = 0
        if decomp.level(pd, P) == M:
            for r in range(T // N):
                c = sum(1 for xs, xe in rng if xs <= r * N + N - 1 and xe >= r * N)
                want += N * (c - 1).bit_length()
        assert decomp.split_row_volume(dims, P, perm) == want

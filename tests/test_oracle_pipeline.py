"""Pins of the oracle's Fig. 4 pipeline (explicit per-process arrays, pack /
all-to-all / unpack) against the M-D DFT, the point-by-point owner count, and
at N_p = T a closed form that needs no owner formula at all."""
from math import prod

import numpy as np
import pytest

from oracle import decomp, dft, orders, pipeline

from paper_1302_6189_amd import inputs


def _x(dims, seed):
    return inputs.uniform(dims, seed, np.complex128)


def _orders(M, n, seed):
    """n valid orders of Eq. (20) drawn at random: the identity, then each
    decomposition a random permutation whose last axis has not been last."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        order, done = [tuple(range(M))], {M - 1}
        for _t in range(M - 1):
            while True:
                p = tuple(int(a) for a in rng.permutation(M))
                if p[-1] not in done:
                    break
            done.add(p[-1])
            order.append(p)
        assert orders.is_valid_order(order, M)
        out.append(order)
    return out


@pytest.mark.parametrize("dims,P", [((6, 4, 5), 1), ((6, 4, 5), 3), ((6, 4, 5), 7), ((4, 3, 5, 2), 5)])
def test_decomposed_equals_axis_by_axis(dims, P):
    # same rows, same 1-D FFTs: bit-identical to the axis-by-axis transform;
    # moved points equal the point-by-point owner count
    x = _x(dims, P)
    for order in _orders(len(dims), 6, P):
        y, steps, ret = pipeline.fftn_decomposed(x, P, order)
        assert np.array_equal(y, dft.fftn_direct(x, orders.fft_axis_sequence(order)))
        want_steps, want_ret = decomp.order_volumes(dims, P, order)
        assert steps == want_steps and ret == want_ret


def test_decomposed_against_brute_force_and_round_trip():
    dims, P = (3, 4, 2), 5
    x = _x(dims, 11)
    order = orders.parse_order("abc->acb->bca")
    y, _, _ = pipeline.fftn_decomposed(x, P, order)
    assert dft.rel_l2(y, dft.dft_bruteforce(x)) < 1e-12
    z, _, _ = pipeline.fftn_decomposed(y, P, order, sign=+1)
    assert dft.rel_l2(z, x) < 1e-13


def _moved_at_one_point_each(dims, perm_a, perm_b) -> int:
    # N_p = T: process p owns exactly position p of each decomposition, so a
    # point moves iff its position differs between the two layouts
    T = prod(dims)
    nat = np.arange(T).reshape(dims)
    pos_a = np.empty(T, dtype=np.int64)
    pos_b = np.empty(T, dtype=np.int64)
    pos_a[np.transpose(nat, perm_a).reshape(-1)] = np.arange(T)
    pos_b[np.transpose(nat, perm_b).reshape(-1)] = np.arange(T)
    return int(np.count_nonzero(pos_a != pos_b))


@pytest.mark.parametrize("dims,P", [((4, 4, 4), 17), ((4, 4, 4), 20), ((4, 4, 4), 64), ((8, 4, 2), 10),
                                    ((3, 2, 2, 4), 20), ((2, 3, 2, 2, 2), 48)])
def test_row_split_regime(dims, P):
    # level M in some decomposition: values still equal the M-D DFT, amounts
    # equal the point-by-point count
    M = len(dims)
    x = _x(dims, P + 1)
    seen_split = False
    for order in _orders(M, 6, P):
        seen_split |= any(decomp.level([dims[a] for a in p], P) == M for p in order)
        y, steps, ret = pipeline.fftn_decomposed(x, P, order)
        assert dft.rel_l2(y, dft.dft_bruteforce(x)) < 1e-12
        want_steps, want_ret = decomp.order_volumes(dims, P, order)
        assert steps == want_steps and ret == want_ret
        z, _, _ = pipeline.fftn_decomposed(y, P, order, sign=+1)
        assert dft.rel_l2(z, x) < 1e-12
    assert seen_split


@pytest.mark.parametrize("dims", [(4, 4, 4), (3, 5, 2), (2, 3, 2, 2), (2, 2, 3, 2, 2)])
def test_one_point_per_process_closed_form(dims):
    T = prod(dims)
    M = len(dims)
    ident = tuple(range(M))
    x = _x(dims, 5)
    for order in _orders(M, 5, T):
        _, steps, ret = pipeline.fftn_decomposed(x, T, order)
        want = [_moved_at_one_point_each(dims, order[t], order[t + 1]) for t in range(M - 1)]
        assert steps == want
        assert ret == _moved_at_one_point_each(dims, order[-1], ident)

"""Pins for the split-row reading (level M of Eq. (13)): the binary-exchange
FFT run on explicit per-process blocks (oracle/rowsplit.py) against the DFT of
Eq. (1), and the points it exchanges against decomp.split_row_volume."""
import itertools
from math import prod

import numpy as np
import pytest

from oracle import decomp, dft, rowsplit


@pytest.mark.parametrize("c", [1, 2, 4, 8, 16])
@pytest.mark.parametrize("b", [1, 2, 3, 5, 8])
def test_binary_exchange_row_is_the_dft(c, b):
    # values: the row's DFT (brute force, Eq. (2) in one dimension), both
    # directions; exchange: every stage moves the whole row once
    rng = np.random.default_rng(13026189 + 17 * c + b)
    N = c * b
    x = rng.uniform(-1, 1, N) + 1j * rng.uniform(-1, 1, N)
    blocks = [x[i * b:(i + 1) * b] for i in range(c)]
    for sign in (-1, 1):
        X, sent = rowsplit.binary_exchange_row(blocks, sign)
        ref = dft.dft_bruteforce(x, sign)
        assert dft.rel_l2(X, ref) < 1e-13, (c, b, sign)
        assert sent == N * (c.bit_length() - 1)


def test_binary_exchange_refuses_uneven_splits():
    with pytest.raises(ValueError):
        rowsplit.binary_exchange_row([np.zeros(2)] * 3)
    with pytest.raises(ValueError):
        rowsplit.binary_exchange_row([np.zeros(2), np.zeros(3)])


@pytest.mark.parametrize("dims,P", [((8, 8, 8), 128), ((8, 8, 8), 512), ((4, 4, 4, 4), 256), ((8, 4, 2), 32),
                                    ((16, 4, 8), 256), ((2, 4, 8, 4), 128), ((2, 4, 8, 4), 256)])
def test_split_row_volume_is_what_the_exchange_moves(dims, P):
    # For every decomposition at level M whose ranges split each row into
    # equal power-of-two pieces, run each row's binary exchange on the
    # processes' own points (ranges from Eqs. (14)-(15)) and add up the
    # points that cross processes: the sum must be split_row_volume, and the
    # rows' results the 1-D DFT along the last axis of the decomposition.
    rng = np.random.default_rng(13026189 + P)
    checked = 0
    for perm in itertools.permutations(range(len(dims))):
        pd = [dims[a] for a in perm]
        N, T = pd[-1], prod(pd)
        if decomp.level(pd, P) < len(dims):
            assert decomp.split_row_volume(dims, P, perm) == 0
            continue
        bnd = decomp.boundaries(dims, P, perm)
        x = rng.uniform(-1, 1, T) + 1j * rng.uniform(-1, 1, T)
        sent = 0
        out = np.empty(T, dtype=np.complex128)
        for r in range(T // N):
            lo, hi = r * N, (r + 1) * N
            cuts = sorted({int(v) for v in bnd if lo < v < hi})
            edges = [lo] + cuts + [hi]
            blocks = [x[a:e] for a, e in zip(edges[:-1], edges[1:])]
            X, s = rowsplit.binary_exchange_row(blocks)
            out[lo:hi] = X
            sent += s
        assert sent == decomp.split_row_volume(dims, P, perm), perm
        assert dft.rel_l2(out, dft.fft1d_rows(x.reshape(-1, N)).reshape(-1)) < 1e-12
        checked += 1
    assert checked > 0

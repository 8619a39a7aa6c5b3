"""Pins for the FP64 transform oracle (Eqs. (1)-(2)).

The oracle is checked against things other than itself: textbook DFT values,
closed forms (delta, constant, single frequency, shift theorem, Parseval),
brute force on tiny grids, and numpy's FFT as an independent library routine.
"""
import numpy as np
import pytest

from oracle import dft

RNG = np.random.default_rng(1302)


def _rand(shape):
    return RNG.uniform(-1, 1, shape) + 1j * RNG.uniform(-1, 1, shape)


def test_textbook_four_point():
    # DFT of (1, 2, 3, 4) with w = exp(-2 pi i / 4) = -i:
    # (10, -2+2i, -2, -2-2i) -- worked by hand from Eq. (1)
    x = np.array([1, 2, 3, 4], dtype=np.complex128)
    want = np.array([10, -2 + 2j, -2, -2 - 2j])
    assert np.allclose(dft.dft_bruteforce(x), want, atol=1e-13)
    assert np.allclose(dft.fftn_direct(x), want, atol=1e-13)


def test_textbook_three_point():
    # length 3: Xbar(1) = 1 + 2 w + 3 w^2 with w = exp(-2 pi i/3)
    w = complex(-0.5, -np.sqrt(3) / 2)
    x = np.array([1, 2, 3], dtype=np.complex128)
    want = np.array([6, 1 + 2 * w + 3 * w * w, 1 + 2 * w * w + 3 * w ** 4])
    assert np.allclose(dft.fftn_direct(x), want, atol=1e-13)


@pytest.mark.parametrize("shape", [(4, 6, 5), (8, 8, 8), (2, 3, 4, 5), (4, 4, 4, 4, 4), (7, 11), (12, 3, 9)])
def test_bruteforce_matches_numpy(shape):
    x = _rand(shape)
    assert dft.rel_l2(dft.dft_bruteforce(x), np.fft.fftn(x)) < 1e-12


@pytest.mark.parametrize("shape", [(4, 6, 5), (8, 8, 8), (2, 3, 4, 5), (4, 4, 4, 4, 4), (7, 11, 13), (16, 12, 10)])
def test_recursive_matches_bruteforce(shape):
    x = _rand(shape)
    assert dft.rel_l2(dft.fftn_direct(x), dft.dft_bruteforce(x)) < 1e-12


@pytest.mark.parametrize("n", list(range(1, 65)) + [96, 125, 128, 162, 180, 192, 243, 256, 512, 1000, 1024])
def test_recursive_1d_matches_numpy(n):
    x = _rand((3, n))
    assert dft.rel_l2(dft.fft1d_rows(x), np.fft.fft(x, axis=-1)) < 1e-12
    assert dft.rel_l2(dft.fft1d_rows(x, sign=+1), np.fft.ifft(x, axis=-1) * n) < 1e-12


def test_large_grid_matches_numpy():
    x = _rand((64, 64, 64))
    assert dft.rel_l2(dft.fftn_direct(x), np.fft.fftn(x)) < 1e-13


def test_delta_and_constant():
    dims = (6, 8, 10)
    d = np.zeros(dims, dtype=np.complex128)
    d[0, 0, 0] = 1
    assert np.allclose(dft.fftn_direct(d), np.ones(dims), atol=1e-14)
    ones = np.ones(dims, dtype=np.complex128)
    y = dft.fftn_direct(ones)
    want = np.zeros(dims, dtype=np.complex128)
    want[0, 0, 0] = np.prod(dims)
    assert np.abs(y - want).max() < 1e-11


def test_single_frequency():
    dims = (8, 12, 5)
    k0 = (3, 7, 2)
    j = np.indices(dims)
    phase = sum(j[r] * k0[r] / dims[r] for r in range(3))
    x = np.exp(2j * np.pi * phase)           # = prod_r w_{N_r}^{-k0_r j_r}
    y = dft.fftn_direct(x)
    want = np.zeros(dims, dtype=np.complex128)
    want[k0] = np.prod(dims)
    assert np.abs(y - want).max() < 1e-10


def test_shift_theorem():
    dims = (8, 6, 10)
    s = (3, 1, 4)
    x = _rand(dims)
    xs = np.roll(x, shift=s, axis=(0, 1, 2))  # xs(j) = x(j - s)
    k = np.indices(dims)
    factor = np.exp(-2j * np.pi * sum(k[r] * s[r] / dims[r] for r in range(3)))
    assert dft.rel_l2(dft.fftn_direct(xs), factor * dft.fftn_direct(x)) < 1e-13


def test_parseval_and_linearity():
    dims = (16, 9, 10)
    x, z = _rand(dims), _rand(dims)
    X = dft.fftn_direct(x)
    T = x.size
    assert abs(np.sum(np.abs(X) ** 2) - T * np.sum(np.abs(x) ** 2)) < 1e-10 * T * np.sum(np.abs(x) ** 2)
    a, b = 0.3 - 1.2j, 2.0 + 0.5j
    assert dft.rel_l2(dft.fftn_direct(a * x + b * z), a * X + b * dft.fftn_direct(z)) < 1e-13


def test_round_trip():
    x = _rand((12, 10, 8, 6))
    assert dft.rel_l2(dft.ifftn_direct(dft.fftn_direct(x)), x) < 1e-14


def test_axis_sequence_does_not_change_the_result():
    x = _rand((8, 6, 10))
    ref = dft.fftn_direct(x)
    for seq in ([0, 1, 2], [1, 2, 0], [2, 0, 1]):
        assert dft.rel_l2(dft.fftn_direct(x, seq), ref) < 1e-14


def test_planted_mistake_is_caught():
    # a wrong sign in the roots of unity must fail the numpy pin
    x = _rand((8, 8))
    wrong = np.conj(dft.fftn_direct(np.conj(x), sign=+1))  # equals the forward transform
    assert dft.rel_l2(wrong, np.fft.fftn(x)) < 1e-13
    assert dft.rel_l2(dft.fftn_direct(x, sign=+1), np.fft.fftn(x)) > 0.1

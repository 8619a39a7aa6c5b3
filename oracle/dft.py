"""FP64 oracle for the transform itself (Section 2, Eqs. (1)-(2)).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.

* ``dft_bruteforce``  -- Eq. (2) summed literally over every input point.
* ``fft1d_rows``      -- Eq. (1) on contiguous rows, through the recursive
                         mixed-radix C code in ``oracle/c/oracle_fft.c``.
* ``fftn_direct``     -- Eq. (2) computed as M single 1-D steps, one axis at a
                         time, in a caller-given axis sequence (the
                         separability remark right after Eq. (2)).
* invariants used by the tests: Parseval, shift theorem, single frequency.

Sign convention: forward uses w_N = exp(-2 pi i / N) with no normalisation
(Eq. (1)).  The inverse (which the paper does not define) uses
w_N = exp(+2 pi i / N) and divides by the total point count T, so that
inverse(forward(x)) = x.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "c", "liboracle.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build_oracle
            build_oracle.build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.oracle_fft_rows.restype = ctypes.c_int
        lib.oracle_fft_rows.argtypes = [ctypes.c_void_p, ctypes.c_int64,
                                        ctypes.c_int64, ctypes.c_int]
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_set_threads.restype = None
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def num_threads() -> int:
    """Threads the C oracle's OpenMP regions use."""
    return int(_load().oracle_num_threads())


def set_threads(n: int) -> None:
    """Threads for the C oracle's later OpenMP regions."""
    _load().oracle_set_threads(int(n))


# ----------------------------------------------------------------------------
# Eq. (2), literally.
# ----------------------------------------------------------------------------
def dft_bruteforce(x: np.ndarray, sign: int = -1) -> np.ndarray:
    """Eq. (2) evaluated as one sum over all T input points per output point.

    Xbar(k) = sum_j prod_r w_{N_r}^{j_r k_r} X(j), with each exponent j_r k_r
    reduced modulo N_r exactly before the complex exponential.  O(T^2); meant
    for T up to a few thousand points.
    """
    x = np.asarray(x, dtype=np.complex128)
    dims = x.shape
    T = x.size
    # coordinates of every point, one column per dimension
    coords = np.indices(dims).reshape(len(dims), T)
    xf = x.reshape(T)
    out = np.empty(T, dtype=np.complex128)
    chunk = max(1, 2_000_000 // max(T, 1))
    for k0 in range(0, T, chunk):
        k1 = min(T, k0 + chunk)
        # phase(k, j) = sum_r ((j_r k_r) mod N_r) / N_r   (a fraction of a turn)
        phase = np.zeros((k1 - k0, T), dtype=np.float64)
        for r, n in enumerate(dims):
            kr = coords[r, k0:k1][:, None].astype(np.int64)
            jr = coords[r][None, :].astype(np.int64)
            phase += ((kr * jr) % n) / float(n)
        w = np.exp(sign * 2j * np.pi * phase)
        out[k0:k1] = w @ xf
    return out.reshape(dims)


# ----------------------------------------------------------------------------
# Eq. (1) on rows through the C recursion.
# ----------------------------------------------------------------------------
def fft1d_rows(x: np.ndarray, sign: int = -1) -> np.ndarray:
    """1-D DFT (Eq. (1)) along the last axis of ``x``; returns a new array."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.complex128)).copy()
    n = a.shape[-1] if a.ndim else 1
    rows = a.size // max(n, 1)
    if a.size:
        rc = _load().oracle_fft_rows(a.ctypes.data, rows, n, int(sign))
        if rc != 0:
            raise RuntimeError("oracle_fft_rows failed")
    return a


def fft_along_axis(x: np.ndarray, axis: int, sign: int = -1) -> np.ndarray:
    """1-D DFT along one axis of an M-D array (moved last, transformed, moved back)."""
    moved = np.moveaxis(np.asarray(x, dtype=np.complex128), axis, -1)
    return np.moveaxis(fft1d_rows(moved, sign), -1, axis)


def fftn_direct(x: np.ndarray, axis_seq=None, sign: int = -1) -> np.ndarray:
    """M-D DFT of Eq. (2) as M single 1-D steps (the remark after Eq. (2)).

    ``axis_seq`` is the order in which axes are transformed; the default is
    last axis first, as the paper describes (Section 2).  Mathematically the
    result does not depend on the sequence; in floating point it does, at
    rounding level.
    """
    a = np.asarray(x, dtype=np.complex128)
    if axis_seq is None:
        axis_seq = list(range(a.ndim))[::-1]
    for ax in axis_seq:
        a = fft_along_axis(a, ax, sign)
    return a


def ifftn_direct(x: np.ndarray, axis_seq=None) -> np.ndarray:
    """Inverse M-D DFT: conjugate roots of unity, then divide by T."""
    a = fftn_direct(x, axis_seq, sign=+1)
    return a / a.size


# ----------------------------------------------------------------------------
# Error metrics used by every parity test.
# ----------------------------------------------------------------------------
def rel_l2(y: np.ndarray, ref: np.ndarray) -> float:
    y = np.asarray(y, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    den = np.linalg.norm(ref.ravel())
    num = np.linalg.norm((y - ref).ravel())
    return float(num / den) if den > 0 else float(num)


def max_abs(y: np.ndarray, ref: np.ndarray) -> float:
    d = np.abs(np.asarray(y, dtype=np.complex128) - np.asarray(ref, dtype=np.complex128))
    return float(d.max()) if d.size else 0.0


def max_abs_rel(y: np.ndarray, ref: np.ndarray) -> float:
    """max|y - ref| / max|ref|."""
    m = float(np.abs(np.asarray(ref)).max()) if np.asarray(ref).size else 0.0
    return max_abs(y, ref) / m if m > 0 else max_abs(y, ref)

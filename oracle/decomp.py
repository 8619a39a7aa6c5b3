"""Integer oracle for the row-wise adaptive decomposition (Section 3).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.

Conventions
-----------
* ``dims`` = (N_1, ..., N_M) of the natural array X(j_1, ..., j_M), j_1 slowest.
* A *decomposition* (one stage of a transpose order) is a permutation ``perm``
  of the axis indices written slowest -> fastest, e.g. (2, 0, 1) is the
  paper's "cab".  ``perm[i]`` is the natural axis at position i; the permuted
  sizes are N'_i = dims[perm[i]].
* Eq. (12) maps a point to its 1-D index in that order:
  X_1 = sum_r x'_r * prod_{s > r} N'_s, where x'_r is its coordinate along
  axis perm[r].

Everything here follows the equations literally and point by point; nothing
is derived in closed form.  The closed forms live in the tests, as pins.

Readings (the paper leaves them implicit):
* Ownership R1 ("literal"): process myid owns [x^s_myid, x^e_myid] of
  Eqs. (14)-(15) in *every* decomposition; a point is communicated in a
  transpose when its owner changes (Fig. 2's "overlap between the areas
  assigned to it").
* Ownership R2 ("matched"): before each transpose the new ranges may be
  handed to processes under any one-to-one relabelling; the relabelling that
  keeps the most points in place is used, so the amount is T minus a
  maximum-weight perfect matching of the overlap matrix.
* The amount of one transpose order is summed over the M-1 transposes between
  consecutive decompositions; the first distribution and the final return to
  natural order are not counted (this is what makes the best order equal the
  1-D method's amount of Eq. (21) when N_p divides N).
"""
from __future__ import annotations

from math import prod

import numpy as np


class RowSplitError(ValueError):
    """N_p exceeds the number of points (no level of Eq. (13) applies)."""


# ----------------------------------------------------------------------------
# Eq. (13): the level and the split function f_{M-D}.
# ----------------------------------------------------------------------------
def level(pdims, P: int) -> int:
    """Smallest k (1-based) with N_p <= N'_1 ... N'_k (the cases of Eq. (13))."""
    acc = 1
    for k, n in enumerate(pdims, start=1):
        acc *= int(n)
        if P <= acc:
            return k
    raise RowSplitError(f"N_p={P} exceeds the {acc} points of the array")


def f_md(pdims, P: int, myid: int) -> int:
    """Eq. (13): floor(N'_1..N'_k * myid / N_p) * N'_{k+1}..N'_M."""
    k = level(pdims, P)
    head = prod(int(n) for n in pdims[:k])
    tail = prod(int(n) for n in pdims[k:])
    return (head * myid // P) * tail


def local_range(pdims, P: int, myid: int):
    """Eqs. (14)-(15): (x^s, x^e) of process myid, inclusive."""
    return f_md(pdims, P, myid), f_md(pdims, P, myid + 1) - 1


def to_md(pdims, x: int):
    """Eqs. (16)-(19): successive floor divisions of a 1-D index."""
    coords = []
    rest = int(x)
    for r in range(len(pdims)):
        w = prod(int(n) for n in pdims[r + 1:])
        c = rest // w
        coords.append(c)
        rest -= c * w
    return tuple(coords)


def decomp(dims, P: int, perm, myid: int):
    """Level, 1-D range and M-D start/end points of process myid.

    Returns (k, xs, xe, start, end); start/end are coordinates in the permuted
    order (start[i] runs along natural axis perm[i]), as in Eqs. (16)-(19).
    """
    pdims = [int(dims[a]) for a in perm]
    k = level(pdims, P)
    xs, xe = local_range(pdims, P, myid)
    return k, xs, xe, to_md(pdims, xs), to_md(pdims, xe)


def boundaries(dims, P: int, perm) -> np.ndarray:
    """f(0), f(1), ..., f(N_p) for one decomposition, as int64."""
    pdims = [int(dims[a]) for a in perm]
    return np.array([f_md(pdims, P, p) for p in range(P + 1)], dtype=np.int64)


# ----------------------------------------------------------------------------
# Owners point by point.
# ----------------------------------------------------------------------------
def linear_index(dims, perm, lead_slice=None) -> np.ndarray:
    """Eq. (12) in the order ``perm`` for every point of the natural array.

    Returned in natural layout (shape dims).  ``lead_slice`` restricts natural
    axis 0 to a sub-range, to bound memory on large arrays.
    """
    M = len(dims)
    pdims = [int(dims[a]) for a in perm]
    stride_of_axis = [0] * M
    for r in range(M):
        stride_of_axis[perm[r]] = prod(pdims[r + 1:])
    rng = [np.arange(int(n), dtype=np.int64) for n in dims]
    if lead_slice is not None:
        rng[0] = rng[0][lead_slice]
    out = np.zeros([len(a) for a in rng], dtype=np.int64)
    for ax in range(M):
        shape = [1] * M
        shape[ax] = len(rng[ax])
        out += (rng[ax] * stride_of_axis[ax]).reshape(shape)
    return out


def owners(dims, P: int, perm, lead_slice=None) -> np.ndarray:
    """Owner (process id) of every point in decomposition ``perm``.

    The owner of a point is the process p with x^s_p <= X_1 <= x^e_p, found by
    searching the boundaries f(0..N_p) of Eqs. (14)-(15).
    """
    b = boundaries(dims, P, perm)
    x = linear_index(dims, perm, lead_slice)
    return (np.searchsorted(b, x, side="right") - 1).astype(np.int64)


def _chunks(dims, max_points=1 << 24):
    n0 = int(dims[0])
    per = max(1, prod(int(n) for n in dims[1:]))
    step = max(1, max_points // per)
    for s in range(0, n0, step):
        yield slice(s, min(n0, s + step))


def pair_volume(dims, P: int, perm_a, perm_b) -> int:
    """R1 amount of one transpose: points whose owner differs between the two."""
    moved = 0
    for sl in _chunks(dims):
        oa = owners(dims, P, perm_a, sl)
        ob = owners(dims, P, perm_b, sl)
        moved += int(np.count_nonzero(oa != ob))
    return moved


def pair_matrix(dims, P: int, perm_a, perm_b) -> np.ndarray:
    """C[p][q] = number of points owned by p before and by q after a transpose."""
    C = np.zeros(P * P, dtype=np.int64)
    for sl in _chunks(dims):
        oa = owners(dims, P, perm_a, sl).ravel()
        ob = owners(dims, P, perm_b, sl).ravel()
        C += np.bincount(oa * P + ob, minlength=P * P)
    return C.reshape(P, P)


def pair_volume_matched(dims, P: int, perm_a, perm_b) -> int:
    """R2 amount: T minus the maximum number of points kept under a
    one-to-one relabelling of the new ranges (an assignment problem, solved
    with scipy's linear_sum_assignment as a library step)."""
    from scipy.optimize import linear_sum_assignment
    C = pair_matrix(dims, P, perm_a, perm_b)
    rows, cols = linear_sum_assignment(C, maximize=True)
    return int(prod(int(n) for n in dims) - C[rows, cols].sum())


def order_volumes(dims, P: int, order, ownership: str = "literal"):
    """Per-transpose amounts V_1..V_{M-1} of one transpose order, plus the
    return transpose (last decomposition -> natural order) reported apart."""
    fn = pair_volume if ownership == "literal" else pair_volume_matched
    steps = [fn(dims, P, order[t], order[t + 1]) for t in range(len(order) - 1)]
    ret = fn(dims, P, order[-1], tuple(range(len(dims))))
    return steps, ret


# ----------------------------------------------------------------------------
# Comparison models, Eqs. (21)-(25), evaluated as printed in real arithmetic.
# ----------------------------------------------------------------------------
def split_row_volume(dims, P: int, perm) -> int:
    """Points the 1-D FFTs along the last axis of ``perm`` would exchange when
    that decomposition is at level M, under the binary-exchange reading (the
    paper does not say how a split row is transformed): a row held by c > 1
    processes runs ceil(log2 c) butterfly stages across processes, each
    sending all N points of the row.  0 below level M.

    The reading was chosen because it reproduces the 11.6 printed for the
    64^3 comparison with the 3-D method in Section 4, so that check confirms
    the choice rather than the paper's intent.  Given the reading, the count
    is pinned against the points an executed binary exchange sends
    (rowsplit.binary_exchange_row, whose result is checked against the DFT)."""
    pdims = [int(dims[a]) for a in perm]
    M = len(pdims)
    if level(pdims, P) < M:
        return 0
    N = pdims[-1]
    # owners of every point in the layout of perm, row by row
    b = boundaries(dims, P, perm)
    x = np.arange(prod(pdims), dtype=np.int64)
    own = np.sort((np.searchsorted(b, x, side="right") - 1).reshape(-1, N), axis=1)
    distinct = 1 + np.count_nonzero(np.diff(own, axis=1), axis=1)   # processes per row
    return int(sum(N * (int(c) - 1).bit_length() for c in distinct))   # ceil(log2 c) for c >= 1


def order_split_volumes(dims, P: int, order):
    """split_row_volume of each FFT step of an order."""
    return [split_row_volume(dims, P, perm) for perm in order]


def amount_1d_method(N: float, Np: float) -> float:
    """Eq. (21): slab method, N^3 - N^3/N_p."""
    return N ** 3 - N ** 3 / Np


def amount_2d_method(N: float, Np: float) -> float:
    """Eq. (22): pencil method, 2N^3 - 2 N_p (N^2/N_p)^(3/2)."""
    return 2 * N ** 3 - 2 * Np * (N ** 2 / Np) ** 1.5


def amount_3d_method(N: float, Np: float) -> float:
    """Eq. (23): volumetric method, 3N^3 (N / cbrt(N^3/N_p) - 1)."""
    return 3 * N ** 3 * (N / (N ** 3 / Np) ** (1.0 / 3.0) - 1)


def amount_4d_method(N: float, Np: float) -> float:
    """Eq. (24): 4N^4 (N / (N^4/N_p)^(1/4) - 1)."""
    return 4 * N ** 4 * (N / (N ** 4 / Np) ** 0.25 - 1)


def amount_5d_method(N: float, Np: float) -> float:
    """Eq. (25): 5N^5 (N / (N^5/N_p)^(1/5) - 1)."""
    return 5 * N ** 5 * (N / (N ** 5 / Np) ** 0.2 - 1)

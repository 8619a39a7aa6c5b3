"""The parallel M-D FFT of Fig. 4, run with explicit per-process arrays.

TEST INFRASTRUCTURE ONLY: imported by tests and the smoke check, never by the
product path.

N_p processes are simulated one array each.  For t = 1..M:
  * Step t: every process runs 1-D FFTs along the last axis of pi_t over the
    whole rows it holds (they are whole when the level of Eq. (13) is below
    M).  At level M (N_p larger than the number of rows, the last case of
    Eq. (13)) ranges cut rows along the FFT axis, and the paper does not say
    how such a row is transformed.  Reading taken here: the processes that
    share a row transform it as one row (their ranges are consecutive pieces
    of the pi_t-order array) and each keeps its own piece; the communication
    this needs is not part of the transposes' amounts, which are counted as
    at any other level.
  * Transpose: each process packs its points into one segment per destination
    (the owner in the next decomposition), an all-to-all moves every segment
    whose destination is another process (counted, in points), and each
    receiver unpacks its segments into its new range.  After pi_M the data go
    back to the natural order (Fig. 4's last transpose), counted apart.

Segment convention (shared knowledge of sender and receiver, not sent): a
segment lists the sender's points in ascending order of their index in the
sender's decomposition; the receiver lists its new positions sorted by
(source process, index in the source's decomposition) and fills them from the
concatenated segments in that order.  Ownership follows the literal reading
(R1): process myid holds range myid of every decomposition.
"""
from __future__ import annotations

from math import prod

import numpy as np

from . import decomp
from .dft import fft1d_rows


def _coords_from_linear(pdims, xlin: np.ndarray) -> np.ndarray:
    """Eqs. (16)-(19) applied to many 1-D indices at once: (M, n) coordinates
    in the permuted order."""
    M = len(pdims)
    out = np.empty((M, xlin.size), dtype=np.int64)
    rest = xlin.astype(np.int64).copy()
    for r in range(M):
        w = prod(int(n) for n in pdims[r + 1:])
        out[r] = rest // w
        rest -= out[r] * w
    return out


def _linear_from_natural(dims, perm, nat: np.ndarray) -> np.ndarray:
    """Eq. (12) in the order perm, from natural coordinates (M, n)."""
    pdims = [int(dims[a]) for a in perm]
    x = np.zeros(nat.shape[1], dtype=np.int64)
    for r in range(len(perm)):
        x = x * pdims[r] + nat[perm[r]]
    return x


def _natural_from_linear(dims, perm, xlin: np.ndarray) -> np.ndarray:
    pdims = [int(dims[a]) for a in perm]
    pc = _coords_from_linear(pdims, xlin)
    nat = np.empty_like(pc)
    for r in range(len(perm)):
        nat[perm[r]] = pc[r]
    return nat


def _transpose(local, dims, P, perm_a, perm_b):
    """All-to-all from decomposition perm_a to perm_b; returns (new local
    arrays, number of points sent to another process)."""
    ba = decomp.boundaries(dims, P, perm_a)
    bb = decomp.boundaries(dims, P, perm_b)
    # pack: every sender splits its points by destination
    send = []
    for p in range(P):
        xa = np.arange(ba[p], ba[p + 1], dtype=np.int64)
        nat = _natural_from_linear(dims, perm_a, xa)
        xb = _linear_from_natural(dims, perm_b, nat)
        dest = np.searchsorted(bb, xb, side="right") - 1
        order = np.argsort(dest, kind="stable")        # ascending x_a inside a segment
        counts = np.bincount(dest, minlength=P)
        offs = np.concatenate([[0], np.cumsum(counts)])
        vals = local[p][order]
        send.append([vals[offs[q]:offs[q + 1]] for q in range(P)])
    # exchange: segments to other processes are the communication
    moved = 0
    recv = [[None] * P for _ in range(P)]
    for p in range(P):
        for q in range(P):
            seg = send[p][q]
            if p != q:
                moved += seg.size
                recv[q][p] = seg.copy()
            else:
                recv[q][p] = seg
    # unpack: each receiver places the concatenated segments
    new_local = []
    for q in range(P):
        xb = np.arange(bb[q], bb[q + 1], dtype=np.int64)
        nat = _natural_from_linear(dims, perm_b, xb)
        xa = _linear_from_natural(dims, perm_a, nat)
        src = np.searchsorted(ba, xa, side="right") - 1
        place = np.lexsort((xa, src))                   # by (source, x_a)
        buf = np.concatenate([recv[q][p] for p in range(P)])
        out = np.empty(xb.size, dtype=buf.dtype)
        out[place] = buf
        new_local.append(out)
    return new_local, moved


def fftn_decomposed(x: np.ndarray, P: int, order, sign: int = -1):
    """Run Fig. 4 on N_p simulated processes.

    Returns (result in natural order, [V_1..V_{M-1}], return-transpose amount).
    ``order`` is a sequence of M permutations with order[0] the identity.
    """
    x = np.asarray(x, dtype=np.complex128)
    dims = x.shape
    M = len(dims)
    ident = tuple(range(M))
    b0 = decomp.boundaries(dims, P, ident)
    flat = x.reshape(-1)
    local = [flat[b0[p]:b0[p + 1]].copy() for p in range(P)]
    moved_steps = []
    moved_return = 0
    for t in range(M):
        perm = order[t]
        n_last = int(dims[perm[-1]])
        if decomp.level([dims[a] for a in perm], P) < M:
            local = [fft1d_rows(a.reshape(-1, n_last), sign).reshape(-1) for a in local]
        else:
            # level M: split rows are transformed whole, pieces stay in place
            sizes = [a.size for a in local]
            whole = fft1d_rows(np.concatenate(local).reshape(-1, n_last), sign).reshape(-1)
            local = np.split(whole, np.cumsum(sizes)[:-1])
        nxt = order[t + 1] if t + 1 < M else ident
        local, moved = _transpose(local, dims, P, perm, nxt)
        if t + 1 < M:
            moved_steps.append(moved)
        else:
            moved_return = moved
    out = np.concatenate(local).reshape(dims)
    if sign == +1:
        out = out / out.size
    return out, moved_steps, moved_return


def permute_layout(x: np.ndarray, perm_a, perm_b) -> np.ndarray:
    """Data movement of one transpose on a whole array held in layout perm_a
    (an array whose axes are natural axes perm_a[0], perm_a[1], ...): returns
    the same points laid out in perm_b.  Used as the exact reference for the
    transpose kernels."""
    # axis i of the result is natural axis perm_b[i], found at position
    # perm_a.index(perm_b[i]) of the input
    src_axes = [list(perm_a).index(a) for a in perm_b]
    return np.ascontiguousarray(np.transpose(x, src_axes))

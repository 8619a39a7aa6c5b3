"""The 1-D FFT of a row split over processes, executed the binary-exchange way.

TEST INFRASTRUCTURE ONLY: imported by tests, never by the product path.

At level M of Eq. (13) the ranges of Eqs. (14)-(15) cut the rows along the
FFT axis, and the paper does not say how such a row is transformed.  The
reading the library's staged plans follow, and that ``decomp.split_row_volume``
counts, is the textbook binary exchange: the c processes that share a row
(b consecutive points each, in process order) run the first log2 c stages of a
radix-2 decimation-in-frequency FFT across processes, then each transforms its
own b points.  This module runs that algorithm on explicit per-process arrays
and counts the points the processes send each other, so that the count can be
checked against the closed form and the result against the DFT of Eq. (1).

Decimation in frequency, one stage of half-span h: inside every span of 2h
points, the lower half keeps a + b and the upper half (a - b) w_{2h}^n for the
pair a = x[n], b = x[n + h], n the offset in the lower half.  After s stages
the row is 2^s independent sequences whose DFTs give the outputs with index
congruent to the bit-reversed sequence number modulo 2^s.
"""
from __future__ import annotations

import numpy as np

from .dft import dft_bruteforce


def binary_exchange_row(blocks, sign: int = -1):
    """The DFT of one row of N = c b points held by c processes, ``blocks[i]``
    being process i's b consecutive points.  c must be a power of two.

    Every stage pairs each process with the one whose block sits half a span
    away; the two send each other their whole blocks (b points each way) and
    each keeps its half of the butterflies.  Returns (X, sent): X the row's DFT
    in natural order (assembled from the processes' pieces), sent the number
    of points that crossed from one process to another.
    """
    c = len(blocks)
    s = c.bit_length() - 1
    if c < 1 or (1 << s) != c:
        raise ValueError("the binary exchange needs a power-of-two number of processes")
    cur = [np.asarray(x, dtype=np.complex128).copy() for x in blocks]
    b = cur[0].size
    if any(x.size != b for x in cur):
        raise ValueError("every process must hold the same number of points")
    N = c * b
    sent = 0
    for st in range(s):
        h = N >> (st + 1)                 # half-span, in points (a multiple of b)
        nxt = []
        for i in range(c):
            partner = i ^ (h // b)
            sent += b                     # the partner's whole block arrives at i
            pos = i * b + np.arange(b)    # positions of i's points in the row
            if (i * b // h) % 2 == 0:     # i holds the lower half of its span
                nxt.append(cur[i] + cur[partner])
            else:
                n = pos % h
                nxt.append((cur[partner] - cur[i]) * np.exp(sign * 2j * np.pi * n / (2 * h)))
        cur = nxt
    X = np.empty(N, dtype=np.complex128)
    for i in range(c):
        rev = int(format(i, f"0{s}b")[::-1], 2) if s else 0
        X[rev + c * np.arange(b)] = dft_bruteforce(cur[i], sign)
    return X, sent

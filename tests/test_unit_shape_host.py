"""Host tests of the fused FFT + transpose unit's shape rule (fft_fused_unit_shape):
the limits every shape must respect, the run-length classes it picks from, and
that it never makes more units than a power-of-two rule within the same
limits would (the rule it replaced).  No device needed."""
import math

import pytest

from paper_1302_6189_amd import fftrw, inputs

THREADS = 256
ITEMS = 16  # values per thread a unit may hold


def pitch(N, esz):
    return N + 2 if esz == 8 and N % 2 == 0 else N + 1


def lanes(rows):
    lanes = 1
    while lanes * 2 * rows <= THREADS:
        lanes *= 2
    return lanes


def pow2_units(N, esz, Nv, ns):
    # rows per slice and slices as powers of two, each doubled while the unit
    # stays within the budget and the doubled count stays below twice the extent
    budget = min(4096 if esz == 8 else 2048, ITEMS * THREADS)
    P, r = pitch(N, esz), 1
    while r * 2 <= THREADS and r * 2 * P <= budget and r * 2 <= 2 * Nv - 1:
        r *= 2
    g = 1
    while g * 2 * r <= THREADS and g * 2 * r * P <= budget and g * 2 <= 2 * ns - 1:
        g *= 2
    return math.ceil(Nv / r) * math.ceil(ns / g)


SIZES = [int(v) for v in inputs.SMOOTH_SIZES] + [2, 3, 5, 8, 256, 300, 480, 512, 1000, 2048, 4000]


@pytest.mark.parametrize("esz", [8, 16])
def test_unit_shape_limits_and_run_classes(esz):
    budget = 4096 if esz == 8 else 2048
    for N in SIZES:
        if N * esz > 16 * 4096 or (esz == 16 and N > 2047):
            continue
        for Nv in [1, 2, 3, 12, 15, 16, 45, 96, 160, 192, 255, 512]:
            for ns in [1, 3, 7, 144, 1000]:
                rw, G = fftrw.fft_fused_unit_shape(N, Nv, ns, esz)
                rows = rw * G
                assert 1 <= rw <= Nv and 1 <= G <= ns, (N, Nv, ns, rw, G)
                assert rows <= THREADS
                assert rows == 1 or rows * pitch(N, esz) <= budget
                assert N <= 16 * lanes(rows), (N, rows)
                # whole v extent, whole 128-byte runs, or a power of two
                assert rw == Nv or rw % 16 == 0 or (rw & (rw - 1)) == 0, (N, Nv, ns, rw)
                assert pow2_units(N, esz, Nv, ns) >= math.ceil(Nv / rw) * math.ceil(ns / G), (N, Nv, ns, rw, G)


def test_unit_shape_batch_items_fewer_units():
    # the batched workload's steps: every (N, Nv, slices) of every item's axes
    old = new = 0
    for dims, _ in inputs.batch_items(256, seed=5):
        T = math.prod(dims)
        for N in set(dims):
            for Nv in set(dims):
                ns = T // (N * Nv)
                rw, G = fftrw.fft_fused_unit_shape(N, Nv, ns)
                new += math.ceil(Nv / rw) * math.ceil(ns / G)
                old += pow2_units(N, 8, Nv, ns)
    assert new < old


def test_unit_shape_refuses_bad_arguments():
    for args in [(1, 4, 4, 8), (16, 0, 4, 8), (16, 4, 0, 8), (16, 4, 4, 4)]:
        with pytest.raises(fftrw.FftrwError):
            fftrw.fft_fused_unit_shape(args[0], args[1], args[2], args[3])

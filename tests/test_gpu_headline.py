"""GPU parity of the benchmarked path: 512-point rows fused with their
transposes (the 512-thread work-group variant of the fused kernel), compared
element by element with the FP64 oracle (Eq. (2) computed axis by axis on the
same FP32-rounded input).

* 512^3 complex64 at full size, in the plans the benchmark times (fused,
  device counting), forward and inverse: N_p = 4096 best order, N_p = 8 best
  order, N_p = 4096 worst order.
* Small shapes (at most 2^24 points) that put 512-point rows and odd or short
  next-layout axes into the fused kernels, over several orders and ragged N_p.

Tolerance: rel-L2 <= 1e-5 (FP32 path), and max|y - ref| / max|ref| <= 1e-5.
"""
import math

import numpy as np
import pytest

from oracle import decomp, dft, orders
from paper_1302_6189_amd import fftrw, inputs
from tests.gpu_util import empty_dev, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def cube512():
    """The 512^3 input (seed 13026189 + 2, as benchmarked) and the oracle's
    forward and inverse transforms of it, computed once."""
    dims = (512, 512, 512)
    x = inputs.uniform(dims, 2, np.complex64)
    fwd = dft.fftn_direct(x)
    inv = dft.ifftn_direct(x)
    return dims, x, fwd, inv


def _compare(y, ref, what):
    err = dft.rel_l2(y, ref)
    mrel = dft.max_abs_rel(y, ref)
    print(f"{what}: rel-L2 {err:.3e} max-abs {dft.max_abs(y, ref):.3e} max-abs/max|ref| {mrel:.3e}", flush=True)
    assert err <= TOL and mrel <= TOL, (what, err, mrel)


@pytest.mark.parametrize("P,which", [(4096, "best"), (8, "best"), (4096, "worst")])
def test_512cube_bench_plans_against_oracle(gpu_lib, cube512, P, which):
    dims, x, ref_fwd, ref_inv = cube512
    r = fftrw.fft_order_search(dims, P)
    order = r["best_order"] if which == "best" else r["worst_order"]
    print(f"512^3 P={P} {which} order {fftrw.order_to_str(order)}", flush=True)
    plan = fftrw.Plan(dims, P, order, flags=fftrw.FLAG_COUNT_MOVED | fftrw.FLAG_FUSED_FFT)
    desc = plan.describe()[1]
    assert desc.startswith("fused|"), desc
    xd = to_dev(x)
    yd = empty_dev(dims, np.complex64)
    plan.exec_fwd(xd, yd)
    _compare(to_host(yd), ref_fwd, f"forward P={P} {which}")
    analytic, moved = plan.stats()
    assert moved == analytic
    assert sum(analytic[:2]) == r["best_volume" if which == "best" else "worst_volume"]
    plan.exec_inv(xd, yd)
    _compare(to_host(yd), ref_inv, f"inverse P={P} {which}")
    _, moved = plan.stats()
    assert moved == analytic  # the inverse runs the same order
    assert np.array_equal(to_host(xd), x)  # the input is left untouched
    del xd, yd
    plan.destroy()


# (dims, P values, canonical order indices): every shape has a 512-point FFT
# axis and every step of these orders fuses; (512, 64, 45) ends with
# 512-point rows fused into a v axis of odd length 45, (512, 75, 64) starts
# with 64-point rows into v = 75 (odd)
SMALL = [((512, 64, 64), (7, 100, 3000), range(8)),
         ((64, 128, 512), (5, 48, 1000), range(8)),
         ((512, 64, 45), (3, 64, 500), (0, 1, 4, 5)),
         ((512, 75, 64), (9, 128), (0, 3, 6)),
         ((96, 512, 80, 3), (6, 300), (0, 401, 1295)),
         ((512, 12, 64, 20), (48,), (72, 1211))]


def _small_cases():
    out = []
    for dims, Ps, idxs in SMALL:
        for P in Ps:
            for i in idxs:
                out.append((dims, P, i))
    return out


@pytest.mark.parametrize("dims,P,oidx", _small_cases())
def test_512_rows_fused_against_oracle(gpu_lib, dims, P, oidx):
    M = len(dims)
    order = fftrw.fft_order_at(M, oidx)
    plan = fftrw.Plan(dims, P, order, flags=fftrw.FLAG_COUNT_MOVED)
    desc = plan.describe()[1]
    print(dims, P, fftrw.order_to_str(order), desc, flush=True)
    assert desc.startswith("fused|"), desc
    assert "8x8x8" in desc  # a 512-point step runs in the compile-time fused kernel
    x = inputs.uniform(dims, 60 + oidx, np.complex64)
    xd = to_dev(x)
    yd = empty_dev(dims, np.complex64)
    plan.exec_fwd(xd, yd)
    ref = dft.fftn_direct(x, orders.fft_axis_sequence(order))
    _compare(to_host(yd), ref, "forward")
    analytic, moved = plan.stats()
    steps, ret = decomp.order_volumes(dims, P, order) if math.prod(dims) <= 1 << 21 else \
        (fftrw.fft_comm_volume(dims, P, order)[0], fftrw.fft_comm_volume(dims, P, order)[2])
    assert analytic == list(steps) + [ret]
    assert moved == analytic
    zd = empty_dev(dims, np.complex64)
    plan.exec_inv(yd, zd)
    _compare(to_host(zd), x, "round trip")
    # bit-identical to separate FFT and transpose kernels
    sep = fftrw.Plan(dims, P, order, flags=fftrw.FLAG_SEPARATE)
    assert not sep.describe()[1].startswith("fused|")
    sep.exec_fwd(xd, zd)
    assert np.array_equal(to_host(zd), to_host(yd))

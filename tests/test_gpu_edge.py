"""Degenerate shapes on the GPU: single points, size-1 axes everywhere,
one process per point, rows of the longest supported length, and the
largest process counts; every mode that accepts the shape, both precisions,
against the oracle's values and point-by-point amounts."""
import math

import numpy as np
import pytest

from oracle import decomp, dft, orders
from paper_1302_6189_amd import fftrw, inputs
from tests.gpu_util import empty_dev, to_dev, to_host

pytestmark = pytest.mark.gpu

MODES = {"fused": fftrw.FLAG_FUSED_FFT, "separate": fftrw.FLAG_SEPARATE, "staged": fftrw.FLAG_STAGED}
TOL = {np.complex64: 1e-5, np.complex128: 1e-12}
DT = {np.complex64: fftrw.C64, np.complex128: fftrw.C128}

CASES = [((1, 1, 1), 1, 0), ((1, 1, 2), 1, 3), ((2, 1, 1), 2, 5), ((1, 64, 1), 64, 2), ((3, 1, 5), 15, 1),
         ((1, 1, 1, 1), 1, 7), ((2, 1, 2, 1, 2), 8, 1000), ((4096, 2, 2), 3, 0), ((2, 4096, 2), 8192, 4),
         ((5, 6, 4), 120, 6)]


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("dtype", [np.complex64, np.complex128])
@pytest.mark.parametrize("dims,P,oidx", CASES)
def test_degenerate_shapes(gpu_lib, dims, P, oidx, dtype, mode):
    M = len(dims)
    order = fftrw.fft_order_at(M, oidx % fftrw.fft_order_count(M))
    print(dims, P, orders.order_to_str(order), np.dtype(dtype).name, mode, flush=True)
    split = any(decomp.level([dims[a] for a in p], P) >= M for p in order)
    try:
        plan = fftrw.Plan(dims, P, order, dtype=DT[dtype], flags=MODES[mode] | fftrw.FLAG_COUNT_MOVED)
    except fftrw.FftrwError as e:
        # only staged transposes refuse, and only at level M
        assert mode == "staged" and split and e.code == fftrw.E_ROWSPLIT
        return
    x = inputs.uniform(dims, 9, dtype)
    xd = to_dev(x)
    yd = empty_dev(dims, dtype)
    plan.exec_fwd(xd, yd)
    ref = dft.fftn_direct(x, orders.fft_axis_sequence(order))
    assert dft.rel_l2(to_host(yd), ref) < TOL[dtype]
    analytic, moved = plan.stats()
    steps, ret = decomp.order_volumes(dims, P, order)
    assert analytic == steps + [ret] and moved == analytic
    zd = empty_dev(dims, dtype)
    plan.exec_inv(yd, zd)
    assert dft.rel_l2(to_host(zd), x) < TOL[dtype]
    if math.prod(dims) == 1:
        assert np.array_equal(to_host(yd), x) and moved == [0] * M

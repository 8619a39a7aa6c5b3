"""Seeded random sweep of the plan paths against the oracle: M = 3..5, small
2,3,5-smooth sizes (1 and 2 included), ragged N_p, random orders, fused /
separate / staged execution and both precisions.  Each case checks the
transform against the FP64 oracle and the device counts against the oracle's
point-by-point amounts."""
import math

import numpy as np
import pytest

from oracle import decomp, dft, orders
from paper_1302_6189_amd import fftrw, inputs
from tests.gpu_util import empty_dev, to_dev, to_host

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 3, 4, 5, 6, 8, 9, 10, 12, 15, 16, 18, 20, 24, 25, 27, 30, 32, 36, 40, 45, 48, 64]
MODES = {"fused": fftrw.FLAG_FUSED_FFT, "separate": fftrw.FLAG_SEPARATE, "staged": fftrw.FLAG_STAGED}
TOL = {np.complex64: 1e-5, np.complex128: 1e-12}


def _cases(n=120, seed=13026189 + 7):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        M = int(rng.integers(3, 6))
        dims = tuple(int(rng.choice(SIZES)) for _ in range(M))
        T = math.prod(dims)
        if T > 60000 or T < 8:
            continue
        # mostly below the row-split regime (N_p <= T / largest size); one case
        # in five anywhere up to T
        cap = T if len(out) % 5 == 4 else max(1, T // max(dims))
        P = int(rng.integers(1, min(cap, 1500) + 1))
        idx = int(rng.integers(0, fftrw.fft_order_count(M)))
        mode = list(MODES)[len(out) % 3]
        dtype = np.complex64 if len(out) % 4 else np.complex128
        out.append((dims, P, idx, mode, dtype))
    return out


@pytest.mark.parametrize("dims,P,idx,mode,dtype", _cases())
def test_random_plans(gpu_lib, dims, P, idx, mode, dtype):
    M = len(dims)
    order = fftrw.fft_order_at(M, idx)
    print(dims, P, orders.order_to_str(order), mode, np.dtype(dtype).name, flush=True)
    try:
        plan = fftrw.Plan(dims, P, order, dtype=fftrw.C64 if dtype == np.complex64 else fftrw.C128,
                          flags=MODES[mode] | fftrw.FLAG_COUNT_MOVED)
    except fftrw.FftrwError as e:
        # staged transposes refuse the row-split regime (level M), exactly
        # when the oracle says it occurs; the other paths run it
        assert e.code == fftrw.E_ROWSPLIT and mode == "staged"
        assert any(decomp.level([dims[a] for a in p], P) >= M for p in order)
        return
    x = inputs.uniform(dims, 2 + idx % 97, dtype)
    xd = to_dev(x)
    yd = empty_dev(dims, dtype)
    plan.exec_fwd(xd, yd)
    ref = dft.fftn_direct(x, orders.fft_axis_sequence(order))
    assert dft.rel_l2(to_host(yd), ref) < TOL[dtype]
    analytic, moved = plan.stats()
    steps, ret = decomp.order_volumes(dims, P, order)
    assert analytic == steps + [ret]
    assert moved == analytic
    zd = empty_dev(dims, dtype)
    plan.exec_inv(yd, zd)
    assert dft.rel_l2(to_host(zd), x) < TOL[dtype]


@pytest.mark.parametrize("dims,P,idx,mode,dtype", _cases(30, seed=13026189 + 8))
def test_random_plans_matched(gpu_lib, dims, P, idx, mode, dtype):
    M = len(dims)
    order = fftrw.fft_order_at(M, idx)
    try:
        plan = fftrw.Plan(dims, P, order, flags=MODES[mode] | fftrw.FLAG_COUNT_MOVED | fftrw.FLAG_OWN_MATCHED)
    except fftrw.FftrwError as e:
        if e.code == fftrw.E_ROWSPLIT:
            # staged transposes need whole rows, exactly as under the literal reading
            assert mode == "staged"
            assert any(decomp.level([dims[a] for a in p], P) >= M for p in order)
        else:
            raise
        return
    x = inputs.uniform(dims, 3, np.complex64)
    xd = to_dev(x)
    yd = empty_dev(dims, np.complex64)
    plan.exec_fwd(xd, yd)
    analytic, moved = plan.stats()
    steps, ret = decomp.order_volumes(dims, P, order, ownership="matched")
    assert analytic == steps + [ret] and moved == analytic

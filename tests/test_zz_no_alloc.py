"""fft_exec_noalloc through the C ABI: the whole pipeline with its workspace in
the library's fixed device array, against fft_plan + fft_exec_fwd/inv with
the same arguments (the same kernels, so bit for bit), on calls in a row
whose sizes shrink, grow to the limit and shrink again (the array keeps the
last call's contents)."""
import numpy as np
import pytest

from oracle import dft, orders
from paper_1302_6189_amd import fftrw, inputs
from tests.gpu_util import empty_dev, layout_shape, to_dev, to_host

pytestmark = pytest.mark.gpu

C64, C128 = fftrw.C64, fftrw.C128
NP = {C64: np.complex64, C128: np.complex128}

# (dims, P, canonical order index or None for the best order, dtype, flags)
SEQUENCE = [((64, 96, 128), 48, None, C64, 0),                       # fused
            ((24, 20, 16, 12), 30, 777, C64, 0),                     # smaller, 4-D, smooth rows
            ((256, 256, 128), 4096, 0, C64, 0),                      # the limit: 2^23 points, 64 MiB
            ((12, 10, 9), 7, 3, C64, fftrw.FLAG_SEPARATE),           # much smaller, separate kernels
            ((32, 16, 32, 32, 8), 100, 123457, C128, 0),             # 5-D complex128, 64 MiB
            ((16, 16, 16), 300, 5, C64, fftrw.FLAG_LEAVE_PERMUTED)]  # output left in the last layout


def _order(dims, oidx):
    return None if oidx is None else fftrw.fft_order_at(len(dims), oidx)


@pytest.mark.parametrize("direction", [-1, 1])
def test_noalloc_matches_plan_exec(gpu_lib, direction):
    for k, (dims, P, oidx, dtype, flags) in enumerate(SEQUENCE):
        order = _order(dims, oidx)
        npdt = NP[dtype]
        print("call", k, dims, P, oidx, np.dtype(npdt).name, flags, "direction", direction, flush=True)
        x = inputs.uniform(dims, 200 + k, npdt)
        xd = to_dev(x)
        plan = fftrw.Plan(dims, P, order, dtype=dtype, flags=flags)
        used_order = plan.describe()[0]
        out_shape = layout_shape(dims, used_order[-1]) if flags & fftrw.FLAG_LEAVE_PERMUTED else dims
        want = empty_dev(out_shape, npdt)
        (plan.exec_fwd if direction < 0 else plan.exec_inv)(xd, want)
        got = empty_dev(out_shape, npdt)
        got.fill_(float("nan"))
        fftrw.fft_exec_noalloc(dims, P, order, direction, xd, got, dtype=dtype, flags=flags)
        g, w = to_host(got), to_host(want)
        assert np.array_equal(g, w), k
        assert np.array_equal(to_host(xd), x)  # in != out: the input is left untouched
        if not flags & fftrw.FLAG_LEAVE_PERMUTED:
            seq = orders.fft_axis_sequence(used_order)
            ref = dft.fftn_direct(x, seq) if direction < 0 else dft.ifftn_direct(x, seq)
            assert dft.rel_l2(g, ref) < (1e-5 if dtype == C64 else 1e-12), k
        plan.destroy()
        del xd, want, got


def test_noalloc_in_place(gpu_lib):
    dims, P = (48, 40, 36), 20
    x = inputs.gaussian(dims, 9, np.complex64)
    plan = fftrw.Plan(dims, P, None)
    want = empty_dev(dims, np.complex64)
    xd = to_dev(x)
    plan.exec_fwd(xd, want)
    fftrw.fft_exec_noalloc(dims, P, None, -1, xd, xd)
    assert np.array_equal(to_host(xd), to_host(want))


def test_noalloc_refusals(gpu_lib):
    xd = to_dev(inputs.uniform((8, 8, 8), 0, np.complex64))
    # one point past the 64 MiB workspace
    with pytest.raises(fftrw.FftrwError) as e:
        fftrw.fft_exec_noalloc((257, 256, 128), 64, None, -1, xd, xd)
    assert e.value.code == fftrw.E_SIZE and "at most 8388608 points" in str(e.value)
    with pytest.raises(fftrw.FftrwError) as e:
        fftrw.fft_exec_noalloc((256, 256, 128), 64, None, -1, xd, xd, dtype=C128)
    assert e.value.code == fftrw.E_SIZE
    for flags in (fftrw.FLAG_STAGED, fftrw.FLAG_COUNT_MOVED, fftrw.FLAG_OWN_MATCHED):
        with pytest.raises(fftrw.FftrwError) as e:
            fftrw.fft_exec_noalloc((8, 8, 8), 4, None, -1, xd, xd, flags=flags)
        assert e.value.code == fftrw.E_UNSUPPORTED
    with pytest.raises(fftrw.FftrwError) as e:
        fftrw.fft_exec_noalloc((8, 8, 8), 4, None, 0, xd, xd)
    assert e.value.code == fftrw.E_ARG
    # the refusals left the entry point usable
    y = empty_dev((8, 8, 8), np.complex64)
    fftrw.fft_exec_noalloc((8, 8, 8), 4, None, -1, xd, y)
    ref = dft.fftn_direct(inputs.uniform((8, 8, 8), 0, np.complex64),
                          orders.fft_axis_sequence(fftrw.fft_order_search((8, 8, 8), 4)["best_order"]))
    assert dft.rel_l2(to_host(y), ref) < 1e-5

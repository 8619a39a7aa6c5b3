"""GPU parity in the row-split regime (level M of Eq. (13): more processes than
rows along some FFT axis).  A split row is transformed whole (its processes
share the device's memory); the transposes are counted exactly as at any
other level.  Values against the FP64 oracle, device counts against the
oracle's point-by-point amounts, transposes bit for bit."""
import math

import numpy as np
import pytest

from oracle import decomp, dft, orders, pipeline
from paper_1302_6189_amd import fftrw, inputs
from tests.gpu_util import empty_dev, to_dev, to_host

pytestmark = pytest.mark.gpu

DT = {np.complex64: fftrw.C64, np.complex128: fftrw.C128}
TOL = {np.complex64: 1e-5, np.complex128: 1e-12}
MODES = {"separate": fftrw.FLAG_SEPARATE, "fused": fftrw.FLAG_FUSED_FFT}

CASES = [((32, 32, 32), 2048, 3), ((64, 64, 64), 8192, 0), ((16, 8, 4), 100, 5), ((8, 8, 8), 512, 2),
         ((8, 8, 8, 8), 1000, 700), ((4, 4, 4, 4, 4), 300, 4000000), ((12, 10, 9), 500, 1),
         ((256, 256, 256), 70000, 4), ((60, 48, 36), 3000, 6)]


def _split_steps(dims, P, order):
    M = len(dims)
    return [t for t, p in enumerate(order) if decomp.level([dims[a] for a in p], P) == M]


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("dtype", [np.complex64, np.complex128])
@pytest.mark.parametrize("dims,P,oidx", CASES)
def test_row_split_plans(gpu_lib, dims, P, oidx, dtype, mode):
    M = len(dims)
    T = math.prod(dims)
    if dtype == np.complex128 and T > 1 << 20:
        pytest.skip("large FP64 case covered by complex64")
    order = fftrw.fft_order_at(M, oidx)
    print(dims, P, orders.order_to_str(order), np.dtype(dtype).name, mode, flush=True)
    assert _split_steps(dims, P, order)
    plan = fftrw.Plan(dims, P, order, dtype=DT[dtype], flags=MODES[mode] | fftrw.FLAG_COUNT_MOVED)
    x = inputs.uniform(dims, 23, dtype)
    xd = to_dev(x)
    yd = empty_dev(dims, dtype)
    plan.exec_fwd(xd, yd)
    analytic, moved = plan.stats()
    assert moved == analytic
    if T <= 1 << 20:
        steps, ret = decomp.order_volumes(dims, P, order)
        assert analytic == steps + [ret]
        ref = dft.fftn_direct(x, orders.fft_axis_sequence(order))
        assert dft.rel_l2(to_host(yd), ref) < TOL[dtype]
    else:
        # large: the library's analytic amounts, and values bit-identical to a
        # plan of the same order at N_p = 8 (N_p changes no arithmetic)
        steps, _, ret = fftrw.fft_comm_volume(dims, P, order, allow_rowsplit=True)
        assert analytic == steps + [ret]
        plain = fftrw.Plan(dims, 8, order, dtype=DT[dtype], flags=fftrw.FLAG_SEPARATE)
        zd = empty_dev(dims, dtype)
        plain.exec_fwd(xd, zd)
        assert np.array_equal(to_host(yd), to_host(zd))
        del zd
    zd = empty_dev(dims, dtype)
    plan.exec_inv(yd, zd)
    assert dft.rel_l2(to_host(zd), x) < TOL[dtype]
    if mode == "fused" and dims in ((64, 64, 64), (256, 256, 256), (12, 10, 9), (60, 48, 36)):
        assert plan.describe()[1].startswith("fused|")


@pytest.mark.parametrize("dims,P,oidx", [((16, 8, 4), 100, 5), ((8, 8, 8, 8), 1000, 700),
                                         ((4, 4, 4, 4, 4), 1024, 123456), ((8, 6, 10), 480, 3)])
def test_row_split_transposes_bit_exact(gpu_lib, dims, P, oidx):
    # every transpose of the order on its own, including the return
    M = len(dims)
    order = fftrw.fft_order_at(M, oidx)
    plan = fftrw.Plan(dims, P, order, flags=fftrw.FLAG_COUNT_MOVED)
    ident = tuple(range(M))
    seq = list(order) + [ident]
    for t in range(M):
        a, b = seq[t], seq[t + 1]
        nat = inputs.uniform(dims, 31 + t, np.complex64)
        xd = to_dev(pipeline.permute_layout(nat, ident, a))
        yd = empty_dev(tuple(dims[i] for i in b), np.complex64)
        plan.exec_transpose(t, xd, yd)
        assert np.array_equal(to_host(yd), pipeline.permute_layout(nat, ident, b)), t
        _, moved = plan.stats()
        assert moved[t] == decomp.pair_volume(dims, P, a, b), t


def test_one_point_per_process(gpu_lib):
    # N_p = T: every point is its own process, so exactly the points whose
    # position changes between two layouts move
    dims = (8, 4, 6)
    T = math.prod(dims)
    order = fftrw.fft_order_at(3, 6)
    plan = fftrw.Plan(dims, T, order, flags=fftrw.FLAG_FUSED_FFT | fftrw.FLAG_COUNT_MOVED)
    x = inputs.uniform(dims, 3, np.complex64)
    xd = to_dev(x)
    yd = empty_dev(dims, np.complex64)
    plan.exec_fwd(xd, yd)
    _, moved = plan.stats()
    seq = list(order) + [(0, 1, 2)]
    nat = np.arange(T).reshape(dims)
    for t in range(3):
        pa = np.empty(T, dtype=np.int64)
        pb = np.empty(T, dtype=np.int64)
        pa[np.transpose(nat, seq[t]).reshape(-1)] = np.arange(T)
        pb[np.transpose(nat, seq[t + 1]).reshape(-1)] = np.arange(T)
        assert moved[t] == int(np.count_nonzero(pa != pb)), t
    assert dft.rel_l2(to_host(yd), dft.fftn_direct(x, orders.fft_axis_sequence(order))) < 1e-5


@pytest.mark.parametrize("fused", [False, True])
def test_row_split_matched_ownership(gpu_lib, fused):
    dims, P = (8, 8, 8), 100
    order = fftrw.fft_order_at(3, 5)
    flags = fftrw.FLAG_COUNT_MOVED | fftrw.FLAG_OWN_MATCHED | (fftrw.FLAG_FUSED_FFT if fused else 0)
    plan = fftrw.Plan(dims, P, order, flags=flags)
    x = inputs.uniform(dims, 41, np.complex64)
    xd = to_dev(x)
    yd = empty_dev(dims, np.complex64)
    plan.exec_fwd(xd, yd)
    analytic, moved = plan.stats()
    steps, ret = decomp.order_volumes(dims, P, order, ownership="matched")
    assert analytic == steps + [ret] and moved == analytic
    assert dft.rel_l2(to_host(yd), dft.fftn_direct(x, orders.fft_axis_sequence(order))) < 1e-5


@pytest.mark.parametrize("flags", [0, fftrw.FLAG_BATCH_NO_FUSE])
def test_row_split_items_in_a_batch(gpu_lib, flags):
    items = [((16, 8, 4), 100), ((12, 10, 9), 500), ((8, 8, 8), 512), ((20, 18, 24, 6), 7),
             ((6, 5, 8, 4, 3), 2000)]
    xs = [inputs.uniform(d, 60 + i, np.complex64) for i, (d, _) in enumerate(items)]
    b = fftrw.Batch(items, flags=flags | fftrw.FLAG_COUNT_MOVED)
    ins = [to_dev(x) for x in xs]
    outs = [empty_dev(x.shape, np.complex64) for x in xs]
    b.exec_fwd(ins, outs)
    st = b.stats()
    assert st["error"] == 0
    for i, (dims, P) in enumerate(items):
        order = fftrw.fft_order_search(dims, P)["best_order"]
        ref = dft.fftn_direct(xs[i], orders.fft_axis_sequence(order))
        assert dft.rel_l2(to_host(outs[i]), ref) < 1e-5, (i, dims, P)
        steps, ret = decomp.order_volumes(dims, P, order)
        assert st["analytic"][i] == steps + [ret]
        assert st["moved"][i] == st["analytic"][i], i


# Staged plans at level M: the split rows' FFT runs as a binary exchange among
# the processes sharing each row (every range b = T / N_p points, c = N / b a
# power of two per row); transposes touching a level-M decomposition run as
# the counted fused permutation, the others through pack -> exchange -> unpack.
STAGED_SPLIT = [((64, 64, 64), 8192, 0),       # b = 32, c = 2 on every step
                ((64, 64, 64), 16384, 5),      # b = 16, c = 4
                ((16, 16, 16), 4096, 3),       # b = 1, c = 16: every point its own process
                ((12, 24, 48), 4608, 6),       # b = 3 (3-point block DFTs), c = 4, 8, 16
                ((64, 64, 16), 2048, 1),       # only the steps along a 64-point axis split (b = 32)
                ((8, 8, 8, 8), 1024, 700),     # 4-D, b = 4, c = 2
                ((8, 8, 8, 8, 8), 8192, 4000000)]  # 5-D, b = 4, c = 2


@pytest.mark.parametrize("dtype", [np.complex64, np.complex128])
@pytest.mark.parametrize("dims,P,oidx", STAGED_SPLIT)
def test_staged_split_rows_binary_exchange(gpu_lib, dims, P, oidx, dtype):
    M = len(dims)
    order = fftrw.fft_order_at(M, oidx)
    plan = fftrw.Plan(dims, P, order, dtype=DT[dtype], flags=fftrw.FLAG_STAGED)
    x = inputs.uniform(dims, 71 + oidx, dtype)
    xd = to_dev(x)
    yd = empty_dev(dims, dtype)
    plan.exec_fwd(xd, yd)
    ref = dft.fftn_direct(x, orders.fft_axis_sequence(order))
    err = dft.rel_l2(to_host(yd), ref)
    split_want = decomp.order_split_volumes(dims, P, order)
    split_analytic, split_moved = plan.rowsplit_stats()
    print(dims, P, orders.order_to_str(order), np.dtype(dtype).name, "rel-L2", err, "split", split_moved,
          flush=True)
    assert err < TOL[dtype]
    # the split rows' exchange: N log2 c points per split row, counted as copied
    assert split_analytic == split_want
    assert split_moved == split_want
    assert sum(split_want) > 0
    # the transposes: owner changes, counted on the device, equal the oracle's
    analytic, moved = plan.stats()
    steps, ret = decomp.order_volumes(dims, P, order)
    assert analytic == steps + [ret] and moved == analytic
    # messages: staged transposes only (whole rows on both sides)
    msgs = plan.messages()
    seq = list(order) + [tuple(range(M))]
    for t in range(M):
        split_t = any(decomp.level([dims[a] for a in p], P) >= M for p in (seq[t], seq[t + 1]))
        assert (msgs[t] == -1) == split_t, t
    zd = empty_dev(dims, dtype)
    plan.exec_inv(yd, zd)
    assert dft.rel_l2(to_host(zd), x) < TOL[dtype]
    assert plan.rowsplit_stats()[1] == split_want  # the inverse exchanges as much


def test_staged_split_rows_refusals(gpu_lib):
    # ranges that are not T / N_p points each, or rows that are not a power of
    # two of them, have no binary exchange: staged plans refuse
    for dims, P in [((8, 8, 8), 65), ((12, 10, 9), 500), ((20, 18, 24), 2880)]:
        with pytest.raises(fftrw.FftrwError) as e:
            fftrw.Plan(dims, P, fftrw.fft_order_at(3, 0), flags=fftrw.FLAG_STAGED)
        assert e.value.code == fftrw.E_ROWSPLIT, (dims, P)
    # below level M nothing changes
    p = fftrw.Plan((16, 16, 16), 16, fftrw.fft_order_at(3, 0), flags=fftrw.FLAG_STAGED)
    assert p.rowsplit_stats()[0] == [0, 0, 0]

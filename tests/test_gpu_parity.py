"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances (relative L2 against FP64): 1e-5 for the FP32 path, 1e-12 for the
FP64 path; transposes and counters are compared bit for bit.
"""
import itertools

import numpy as np
import pytest

from oracle import decomp, dft, orders, pipeline
from paper_1302_6189_amd import fftrw, inputs
from tests.gpu_util import bits_equal, empty_dev, layout_shape, sampled_dft, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL = {np.complex64: 1e-5, np.complex128: 1e-12}
DT = {np.complex64: fftrw.C64, np.complex128: fftrw.C128}


def _cases_rows():
    # row lengths: powers of two, smooth mixed radices, ragged row counts
    # (every axis is transformed by some step, so row counts are 2,3,5-smooth
    # too; odd counts leave a partial last work-group)
    return [(16, 1125), (32, 375), (64, 4096), (128, 75), (256, 2025), (512, 1215), (1024, 45), (2048, 9),
            (4096, 5), (12, 1000), (15, 100), (18, 50), (45, 75), (100, 40), (192, 135), (243, 27),
            (375, 8), (1000, 3), (3, 1024), (2, 4096), (1, 10)]


@pytest.mark.parametrize("dtype", [np.complex64, np.complex128])
@pytest.mark.parametrize("n,rows", _cases_rows())
def test_fft_step_rows(gpu_lib, n, rows, dtype):
    dims = (rows, n)
    x = inputs.uniform(dims, 101 + n, dtype)
    plan = fftrw.Plan(dims, 1, "ab->ba", dtype=DT[dtype])
    xd = to_dev(x)
    for direction in (-1, 1):
        yd = empty_dev(dims, dtype)
        plan.exec_fft_step(0, direction, xd, yd)
        y = to_host(yd)
        ref = dft.fft1d_rows(x, sign=direction)
        assert dft.rel_l2(y, ref) < TOL[dtype], (n, rows, direction)
    # in place
    plan.exec_fft_step(0, -1, xd, xd)
    assert dft.rel_l2(to_host(xd), dft.fft1d_rows(x)) < TOL[dtype]


def _transpose_cases():
    out = []
    for dims, P in [((8, 8, 8), 4), ((16, 12, 10), 7), ((64, 64, 64), 48), ((5, 6, 9), 3),
                    ((1, 8, 8), 1), ((32, 32, 32), 1000)]:
        for o in list(orders.all_orders(3))[::3]:
            out.append((dims, P, o))
    for dims, P in [((6, 10, 12, 4), 48), ((16, 16, 16, 16), 256), ((8, 8, 8, 8), 500)]:
        for idx in (0, 17, 300, 1295):
            out.append((dims, P, orders_at(4, idx)))
    for dims, P in [((4, 6, 4, 5, 8), 48), ((8, 8, 8, 8, 4), 1000), ((4, 4, 4, 4, 4), 256)]:
        for idx in (0, 123456, 7962623):
            out.append((dims, P, orders_at(5, idx)))
    return out


def orders_at(M, idx):
    return fftrw.fft_order_at(M, idx)


@pytest.mark.parametrize("staged", [False, True])
@pytest.mark.parametrize("dtype", [np.complex64, np.complex128])
@pytest.mark.parametrize("dims,P,order", _transpose_cases())
def test_transpose_bit_exact_and_counted(gpu_lib, dims, P, order, dtype, staged):
    M = len(dims)
    flags = fftrw.FLAG_COUNT_MOVED | (fftrw.FLAG_STAGED if staged else 0)
    plan = fftrw.Plan(dims, P, order, dtype=DT[dtype], flags=flags)
    ident = tuple(range(M))
    seq = list(order) + [ident]
    analytic, _ = plan.stats()
    for t in range(M):
        a, b = seq[t], seq[t + 1]
        nat = inputs.uniform(dims, 7 + t, dtype)
        xa = pipeline.permute_layout(nat, ident, a)
        xd = to_dev(xa)
        yd = empty_dev(layout_shape(dims, b), dtype)
        plan.exec_transpose(t, xd, yd)
        y = to_host(yd)
        assert bits_equal(y, pipeline.permute_layout(nat, ident, b)), (t, a, b)
        _, moved = plan.stats()
        want = decomp.pair_volume(dims, P, a, b)
        assert analytic[t] == want
        assert moved[t] == want, (t, moved[t], want)
        if staged and P <= 256:
            # messages of the all-to-all: off-diagonal pairs that share points
            C = decomp.pair_matrix(dims, P, a, b)
            np.fill_diagonal(C, 0)
            assert plan.messages()[t] == int(np.count_nonzero(C)), t


@pytest.mark.parametrize("dtype", [np.complex128, np.complex64])
@pytest.mark.parametrize("oidx", range(8))
def test_32cube_all_orders(gpu_lib, oidx, dtype):
    # 32^3, P = 4, every 3-D order; the oracle consumes exactly the GPU's input
    dims, P = (32, 32, 32), 4
    order = list(orders.all_orders(3))[oidx]
    x = inputs.uniform(dims, 1, np.complex128).astype(dtype)
    ref = dft.fftn_direct(x, orders.fft_axis_sequence(order))
    plan = fftrw.Plan(dims, P, order, dtype=DT[dtype], flags=fftrw.FLAG_COUNT_MOVED)
    xd = to_dev(x)
    yd = empty_dev(dims, dtype)
    plan.exec_fwd(xd, yd)
    y = to_host(yd)
    assert dft.rel_l2(y, ref) < TOL[dtype]
    analytic, moved = plan.stats()
    steps, ret = decomp.order_volumes(dims, P, order)
    assert analytic == steps + [ret] and moved == analytic
    # inverse round trip
    zd = empty_dev(dims, dtype)
    plan.exec_inv(yd, zd)
    assert dft.rel_l2(to_host(zd), x) < TOL[dtype]
    # the decomposed oracle pipeline gives the same counts
    _, st, rt = pipeline.fftn_decomposed(x, P, order)
    assert st + [rt] == moved


@pytest.mark.parametrize("staged", [False, True])
def test_in_place_and_leave_permuted(gpu_lib, staged):
    dims, P = (24, 20, 16, 12), 30
    order = orders_at(4, 777)
    x = inputs.gaussian(dims, 3, np.complex64)
    ref = dft.fftn_direct(x, orders.fft_axis_sequence(order))
    extra = fftrw.FLAG_STAGED if staged else 0
    plan = fftrw.Plan(dims, P, order, flags=fftrw.FLAG_COUNT_MOVED | extra)
    xd = to_dev(x)
    plan.exec_fwd(xd, xd)
    assert dft.rel_l2(to_host(xd), ref) < 1e-5
    plan2 = fftrw.Plan(dims, P, order, flags=fftrw.FLAG_LEAVE_PERMUTED | extra)
    xd = to_dev(x)
    yd = empty_dev(layout_shape(dims, order[-1]), np.complex64)
    plan2.exec_fwd(xd, yd)
    want = pipeline.permute_layout(ref, tuple(range(4)), order[-1])
    assert dft.rel_l2(to_host(yd), want) < 1e-5
    assert bits_equal(to_host(xd), x)  # input untouched when in != out


@pytest.mark.parametrize("dims,P,oidx", [((64, 64, 64, 64), 48, 0), ((64, 64, 64, 64), 256, 401),
                                         ((64, 64, 64, 64), 1000, 1295),
                                         ((32, 32, 32, 32, 16), 48, 0), ((32, 32, 32, 32, 16), 256, 3333333),
                                         ((32, 32, 32, 32, 16), 1000, 7962623)])
@pytest.mark.parametrize("staged", [False, True])
def test_64pow4_and_32pow4x16_orders(gpu_lib, dims, P, oidx, staged):
    M = len(dims)
    order = fftrw.fft_order_at(M, oidx)
    extra = fftrw.FLAG_STAGED if staged else 0
    try:
        plan = fftrw.Plan(dims, P, order, flags=fftrw.FLAG_COUNT_MOVED | extra)
    except fftrw.FftrwError as e:
        assert e.code == fftrw.E_ROWSPLIT and staged
        pytest.skip("staged transposes need whole rows")
    x = inputs.gaussian(dims, 3 if M == 4 else 30, np.complex64)
    xd = to_dev(x)
    yd = empty_dev(dims, np.complex64)
    plan.exec_fwd(xd, yd)
    y = to_host(yd)
    ref = dft.fftn_direct(x, orders.fft_axis_sequence(order))
    assert dft.rel_l2(y, ref) < 1e-5
    analytic, moved = plan.stats()
    steps, tot, ret = fftrw.fft_comm_volume(dims, P, order)
    assert analytic == steps + [ret] and moved == analytic


@pytest.mark.parametrize("P,which", [(8, "best"), (4096, "best"), (4096, "worst"), (512, "worst")])
def test_512cube_full_size_sampled(gpu_lib, P, which):
    # 512^3 complex64 at full size: points of Eq. (2) computed one by one in
    # FP64, Parseval over the whole output, exact device counts
    dims = (512, 512, 512)
    r = fftrw.fft_order_search(dims, P)
    order = r["best_order"] if which == "best" else r["worst_order"]
    x = inputs.uniform(dims, 2, np.complex64)
    plan = fftrw.Plan(dims, P, order, flags=fftrw.FLAG_COUNT_MOVED)
    xd = to_dev(x)
    yd = empty_dev(dims, np.complex64)
    plan.exec_fwd(xd, yd)
    y = to_host(yd)
    rng = np.random.default_rng(P)
    pts = [tuple(int(v) for v in rng.integers(0, 512, 3)) for _ in range(6)] + [(0, 0, 0), (511, 1, 256)]
    want = sampled_dft(x, pts)
    got = np.array([y[p] for p in pts])
    scale = np.sqrt(np.mean(np.abs(want) ** 2))
    assert np.max(np.abs(got - want)) / scale < 1e-4
    T = x.size
    e_in = np.sum(np.abs(x.astype(np.complex128)) ** 2)
    e_out = np.sum(np.abs(y.astype(np.complex128)) ** 2)
    assert abs(e_out - T * e_in) / (T * e_in) < 1e-5
    analytic, moved = plan.stats()
    assert moved == analytic
    assert sum(analytic[:2]) == r["best_volume" if which == "best" else "worst_volume"]
    del xd, yd


def test_plan_errors_on_device(gpu_lib):
    with pytest.raises(fftrw.FftrwError) as e:
        fftrw.Plan((7, 8, 8), 2, "abc->acb->bca")
    assert e.value.code == fftrw.E_SIZE
    with pytest.raises(fftrw.FftrwError) as e:
        fftrw.Plan((4,) * 6, 2, None)  # 6-D: host model only
    assert e.value.code == fftrw.E_SIZE
    with pytest.raises(fftrw.FftrwError) as e:
        fftrw.Plan((4096, 4096, 4096), 8, None, dtype=fftrw.C128)  # a 1.1 TB workspace
    assert e.value.code == fftrw.E_NOMEM
    with pytest.raises(fftrw.FftrwError) as e:
        fftrw.Plan((8, 8, 8), 513, "abc->acb->bca")  # more processes than points
    assert e.value.code == fftrw.E_ROWSPLIT
    with pytest.raises(fftrw.FftrwError) as e:
        fftrw.Plan((8, 8, 8), 65, "abc->acb->bca", flags=fftrw.FLAG_STAGED)  # level M, staged
    assert e.value.code == fftrw.E_ROWSPLIT
    with pytest.raises(fftrw.FftrwError) as e:
        fftrw.Plan((8, 8, 8), 4, "abc->acb->bca", dtype=3)
    assert e.value.code == fftrw.E_ARG
    p = fftrw.Plan((8, 8, 8), 4, "abc->acb->bca")
    xd = to_dev(inputs.uniform((8, 8, 8), 0))
    with pytest.raises(fftrw.FftrwError) as e:
        p.exec_transpose(0, xd, xd)
    assert e.value.code == fftrw.E_ARG
    with pytest.raises(fftrw.FftrwError) as e:
        p.exec_fft_step(3, -1, xd, xd)
    assert e.value.code == fftrw.E_ARG


def test_default_order_is_best(gpu_lib):
    dims, P = (16, 16, 16, 16), 300
    p = fftrw.Plan(dims, P, None)
    o, _ = p.describe()
    assert o == fftrw.fft_order_search(dims, P)["best_order"]


@pytest.mark.parametrize("dims,P,oidx", [((64, 64, 64), 48, 0), ((64, 64, 64), 1000, 3), ((128, 32, 64), 7, 5),
                                         ((512, 512, 512), 4096, 0), ((16, 32, 64, 128), 300, 777),
                                         ((32, 16, 64, 32, 16), 100, 123457), ((256, 256, 256), 64, 6),
                                         ((60, 48, 36), 20, 3), ((45, 50, 27, 12), 50, 400),
                                         ((96, 80, 64), 7, 1), ((12, 15, 20, 6, 9), 64, 5000000),
                                         ((250, 243, 6), 1000, 2)])
@pytest.mark.parametrize("dtype", [np.complex64, np.complex128])
def test_fused_fft_transpose(gpu_lib, dims, P, oidx, dtype):
    if dtype == np.complex128 and np.prod(dims) > 1 << 24:
        pytest.skip("large FP64 case covered by complex64")
    M = len(dims)
    order = fftrw.fft_order_at(M, oidx)
    plan = fftrw.Plan(dims, P, order, dtype=DT[dtype], flags=fftrw.FLAG_FUSED_FFT | fftrw.FLAG_COUNT_MOVED)
    fused = plan.describe()[1].startswith("fused|")
    x = inputs.uniform(dims, 11, dtype)
    xd = to_dev(x)
    yd = empty_dev(dims, dtype)
    plan.exec_fwd(xd, yd)
    analytic, moved = plan.stats()
    assert moved == analytic
    if np.prod(dims) <= 1 << 24:
        ref = dft.fftn_direct(x, orders.fft_axis_sequence(order))
        assert dft.rel_l2(to_host(yd), ref) < TOL[dtype]
    else:
        # full size: against the unfused pipeline (same kernels' arithmetic per row)
        plain = fftrw.Plan(dims, P, order, dtype=DT[dtype], flags=fftrw.FLAG_SEPARATE)
        zd = empty_dev(dims, dtype)
        plain.exec_fwd(xd, zd)
        assert np.array_equal(to_host(yd), to_host(zd))
        del zd
    zd = empty_dev(dims, dtype)
    plan.exec_inv(yd, zd)
    assert dft.rel_l2(to_host(zd), x) < TOL[dtype]
    # which shapes fuse: rows 16..512 (FP32) / ..256 (FP64) with runs >= 8 along v
    print("fused" if fused else "unfused", dims, flush=True)
    if dims in ((64, 64, 64), (512, 512, 512), (256, 256, 256)) and dtype == np.complex64:
        assert fused
    if dims in ((60, 48, 36), (45, 50, 27, 12), (12, 15, 20, 6, 9), (250, 243, 6)):
        assert fused  # every step has 2,3,5-smooth rows: the generic fused unit


def test_fused_leave_permuted_and_in_place(gpu_lib):
    dims, P = (64, 32, 128, 16), 40
    order = fftrw.fft_order_at(4, 999)
    x = inputs.gaussian(dims, 12, np.complex64)
    ref = dft.fftn_direct(x, orders.fft_axis_sequence(order))
    plan = fftrw.Plan(dims, P, order, flags=fftrw.FLAG_FUSED_FFT | fftrw.FLAG_LEAVE_PERMUTED | fftrw.FLAG_COUNT_MOVED)
    xd = to_dev(x)
    yd = empty_dev(layout_shape(dims, order[-1]), np.complex64)
    plan.exec_fwd(xd, yd)
    assert dft.rel_l2(to_host(yd), pipeline.permute_layout(ref, tuple(range(4)), order[-1])) < 1e-5
    a, m = plan.stats()
    assert m[:-1] == a[:-1] and m[-1] == -1
    # in == out falls back to the unfused pipeline and stays correct
    plan2 = fftrw.Plan(dims, P, order, flags=fftrw.FLAG_FUSED_FFT)
    xd = to_dev(x)
    plan2.exec_fwd(xd, xd)
    assert dft.rel_l2(to_host(xd), ref) < 1e-5


@pytest.mark.parametrize("fused", [False, True])
@pytest.mark.parametrize("dims,P,oidx", [((16, 16, 16), 48, 3), ((32, 32, 32), 100, 5), ((32, 16, 64), 7, 1),
                                         ((8, 8, 16, 16), 20, 700), ((16, 16, 16, 16), 300, 1295)])
def test_matched_ownership_device_counts(gpu_lib, dims, P, oidx, fused):
    # the relabelled ranges of the matched reading, counted on the device
    M = len(dims)
    order = fftrw.fft_order_at(M, oidx)
    flags = fftrw.FLAG_COUNT_MOVED | fftrw.FLAG_OWN_MATCHED | (fftrw.FLAG_FUSED_FFT if fused else 0)
    plan = fftrw.Plan(dims, P, order, flags=flags)
    x = inputs.uniform(dims, 17, np.complex64)
    xd = to_dev(x)
    yd = empty_dev(dims, np.complex64)
    plan.exec_fwd(xd, yd)
    analytic, moved = plan.stats()
    steps, ret = decomp.order_volumes(dims, P, order, ownership="matched")
    assert analytic == steps + [ret]
    assert moved == analytic
    ref = dft.fftn_direct(x, orders.fft_axis_sequence(order))
    assert dft.rel_l2(to_host(yd), ref) < 1e-5


def test_plan_log_line(gpu_lib):
    # FFTRW_LOG=1: one line per plan created, naming its order and kernels
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("from paper_1302_6189_amd import fftrw\n"
            "p = fftrw.Plan((8, 8, 8), 4, 'abc->acb->bca', flags=fftrw.FLAG_FUSED_FFT)\n")
    env = dict(os.environ, FFTRW_LOG="1")
    r = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, stdout=subprocess.PIPE,
                       stderr=subprocess.PIPE, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    lines = [l for l in r.stderr.splitlines() if l.startswith("fftrw: plan ")]
    assert len(lines) == 1 and "8x8x8 P=4 order abc->acb->bca kernels" in lines[0], r.stderr

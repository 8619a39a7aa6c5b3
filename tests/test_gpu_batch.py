"""GPU parity of the batched form: many uneven transforms in one persistent,
graph-replayed launch, against the FP64 oracle and the per-item path."""
import numpy as np
import pytest

from oracle import dft, orders
from paper_1302_6189_amd import fftrw, inputs
from tests.gpu_util import empty_dev, to_dev, to_host

pytestmark = pytest.mark.gpu

SMALL = [((12, 15, 16), 5), ((20, 18, 24, 6), 7), ((16, 16, 16), 1), ((27, 25, 12), 64),
         ((8, 12, 10, 6, 5), 9), ((32, 30, 18), 33), ((45, 6, 50), 2), ((64, 48, 40), 48),
         ((10, 12, 9, 8), 100), ((6, 5, 8, 4, 3), 30), ((192, 12, 20), 17), ((81, 16, 15), 12)]


def _run(batch, xs, fwd=True):
    ins = [to_dev(x) for x in xs]
    outs = [empty_dev(x.shape, np.complex64) for x in xs]
    (batch.exec_fwd if fwd else batch.exec_inv)(ins, outs)
    return ins, outs


def test_small_batch_against_oracle(gpu_lib):
    xs = [inputs.uniform(d, 50 + i, np.complex64) for i, (d, _) in enumerate(SMALL)]
    b = fftrw.Batch(SMALL, flags=fftrw.FLAG_COUNT_MOVED)
    ins, outs = _run(b, xs)
    st = b.stats()
    assert st["error"] == 0
    for i, (dims, P) in enumerate(SMALL):
        order = fftrw.fft_order_search(dims, P)["best_order"]
        ref = dft.fftn_direct(xs[i], orders.fft_axis_sequence(order))
        err = dft.rel_l2(to_host(outs[i]), ref)
        assert err < 1e-5, (i, dims, P, err)
        steps, _, ret = fftrw.fft_comm_volume(dims, P, order)
        assert st["analytic"][i] == steps + [ret]
        assert st["moved"][i] == st["analytic"][i], (i, st["moved"][i])
    # inverse round trip through the batch
    back = [empty_dev(x.shape, np.complex64) for x in xs]
    b.exec_inv(outs, back)
    for i, x in enumerate(xs):
        assert dft.rel_l2(to_host(back[i]), x) < 1e-5
    assert b.stats()["error"] == 0


def test_graph_replays_match_eager(gpu_lib):
    import torch
    xs = [inputs.gaussian(d, 70 + i, np.complex64) for i, (d, _) in enumerate(SMALL)]
    eager = fftrw.Batch(SMALL, flags=fftrw.FLAG_BATCH_NO_GRAPH | fftrw.FLAG_COUNT_MOVED)
    ins, ref_outs = _run(eager, xs)
    ref = [to_host(o) for o in ref_outs]
    ref_moved = eager.stats()["moved"]
    g = fftrw.Batch(SMALL, flags=fftrw.FLAG_COUNT_MOVED)
    outs = [empty_dev(x.shape, np.complex64) for x in xs]
    for rep in range(4):
        for o in outs:
            o.zero_()
        g.exec_fwd(ins, outs)
        torch.cuda.synchronize()
        # the program's own eager work between replays
        junk = torch.randn(1 << 20, device="cuda").sum().item()
        assert np.isfinite(junk)
        for i in range(len(xs)):
            assert np.array_equal(to_host(outs[i]), ref[i]), (rep, i)
        st = g.stats()
        assert st["error"] == 0 and st["moved"] == ref_moved


def test_batch_matches_per_item_plans(gpu_lib):
    items = inputs.batch_items(24, seed=5)
    xs = [inputs.uniform(d, 90 + i, np.complex64) for i, (d, _) in enumerate(items)]
    b = fftrw.Batch(items, flags=fftrw.FLAG_COUNT_MOVED)
    ins, outs = _run(b, xs)
    st = b.stats()
    assert st["error"] == 0
    for i, (dims, P) in enumerate(items):
        p = fftrw.Plan(dims, P, None)
        y = empty_dev(dims, np.complex64)
        p.exec_fwd(ins[i], y)
        assert dft.rel_l2(to_host(outs[i]), to_host(y)) < 2e-6, (i, dims)
        assert st["moved"][i] == st["analytic"][i]


@pytest.fixture(scope="module")
def batch256():
    """The 256-item batched workload (seed 13026189 + 5) run once in each
    schedule: fused stages (the default) and separate FFT / transpose stages."""
    items = inputs.batch_items(256, seed=5)
    xs = [inputs.uniform(d, 1000 + i, np.complex64) for i, (d, _) in enumerate(items)]
    runs = {}
    for name, extra in (("fused", 0), ("separate", fftrw.FLAG_BATCH_NO_FUSE)):
        b = fftrw.Batch(items, flags=fftrw.FLAG_COUNT_MOVED | extra)
        ins, outs = _run(b, xs)
        st = b.stats()
        runs[name] = ([to_host(o) for o in outs], st)
        del ins, outs
        b.destroy()
    return items, xs, runs


@pytest.mark.parametrize("chunk", range(8))
def test_full_256_item_batch_against_oracle(gpu_lib, batch256, chunk):
    # every item of the workload, both schedules: values against the FP64
    # oracle element by element, device counts against the analytic amounts
    items, xs, runs = batch256
    for i in range(32 * chunk, 32 * chunk + 32):
        dims, P = items[i]
        order = fftrw.fft_order_search(dims, P)["best_order"]
        ref = dft.fftn_direct(xs[i], orders.fft_axis_sequence(order))
        steps, _, ret = fftrw.fft_comm_volume(dims, P, order)
        for name, (ys, st) in runs.items():
            assert st["error"] == 0
            y = ys[i]
            err, mrel = dft.rel_l2(y, ref), dft.max_abs_rel(y, ref)
            assert err < 1e-5 and mrel < 1e-5, (name, i, dims, P, err, mrel)
            assert st["analytic"][i] == steps + [ret], (name, i)
            assert st["moved"][i] == st["analytic"][i], (name, i, st["moved"][i])
        assert np.array_equal(runs["fused"][0][i], runs["separate"][0][i]), i


def test_autotuned_batch(gpu_lib, tmp_path):
    import json
    items = inputs.batch_items(32, seed=5)
    cache = str(tmp_path / "tune.json")
    fftrw.fft_autotune(items, cache)
    with open(cache) as f:
        rec = json.load(f)
    assert rec["device"].startswith("gfx950") and rec["version"].startswith("fftrw")
    lengths = {d[a] for d, _ in items for a in range(len(d))}
    assert {r["n"] for r in rec["rows"]} == lengths
    for r in rec["rows"]:
        assert np.prod(r["radix"]) == r["n"]
    # radix orders timed in the fused FFT step + transpose, per (N, N_v) pair
    assert rec["fused"]
    assert {r["n"] for r in rec["fused"]} == lengths
    for r in rec["fused"]:
        assert np.prod(r["radix"]) == r["n"]
    xs = [inputs.uniform(d, 300 + i, np.complex64) for i, (d, _) in enumerate(items)]
    b = fftrw.Batch(items, flags=fftrw.FLAG_COUNT_MOVED, tune_cache=cache)
    ins, outs = _run(b, xs)
    st = b.stats()
    assert st["error"] == 0 and st["moved"] == st["analytic"]
    for i in (0, 5, 17, 31):
        dims, P = items[i]
        order = fftrw.fft_order_search(dims, P)["best_order"]
        ref = dft.fftn_direct(xs[i], orders.fft_axis_sequence(order))
        assert dft.rel_l2(to_host(outs[i]), ref) < 1e-5
    # a cache for another device is ignored (same results as no cache)
    rec["device"] = "other"
    with open(cache, "w") as f:
        json.dump(rec, f)
    b2 = fftrw.Batch(items, tune_cache=cache)
    ins2, outs2 = _run(b2, xs)
    plain = fftrw.Batch(items)
    ins3, outs3 = _run(plain, xs)
    for i in range(len(items)):
        assert np.array_equal(to_host(outs2[i]), to_host(outs3[i]))


def test_fused_radix_cache_entries(gpu_lib, tmp_path):
    # the fused stages take the cache's per-(N, N_v) radix orders only when
    # they are valid (radices of the kernel, product N); otherwise the batch
    # keeps its built-in orders and computes bit for bit what an untuned
    # batch does
    import json
    items = inputs.batch_items(12, seed=9)
    xs = [inputs.uniform(d, 500 + i, np.complex64) for i, (d, _) in enumerate(items)]
    cache = str(tmp_path / "tune.json")
    fftrw.fft_autotune(items, cache)
    with open(cache) as f:
        rec = json.load(f)
    rec["rows"], rec["tiles"] = [], []
    plain = fftrw.Batch(items)
    _, ref_outs = _run(plain, xs)
    bad = dict(rec, fused=[dict(r, radix=[7] if i % 2 else r["radix"] + [2]) for i, r in enumerate(rec["fused"])])
    with open(cache, "w") as f:
        json.dump(bad, f)
    b = fftrw.Batch(items, tune_cache=cache)
    _, outs = _run(b, xs)
    for i in range(len(items)):
        assert np.array_equal(to_host(outs[i]), to_host(ref_outs[i])), i
    # valid orders (every order reversed: still the product N) are applied
    good = dict(rec, fused=[dict(r, radix=r["radix"][::-1]) for r in rec["fused"]])
    with open(cache, "w") as f:
        json.dump(good, f)
    b2 = fftrw.Batch(items, flags=fftrw.FLAG_COUNT_MOVED, tune_cache=cache)
    _, outs2 = _run(b2, xs)
    st = b2.stats()
    assert st["error"] == 0 and st["moved"] == st["analytic"]
    differs = False
    for i, (dims, P) in enumerate(items):
        order = fftrw.fft_order_search(dims, P)["best_order"]
        ref = dft.fftn_direct(xs[i], orders.fft_axis_sequence(order))
        y = to_host(outs2[i])
        assert dft.rel_l2(y, ref) < 1e-5, i
        differs = differs or not np.array_equal(y, to_host(ref_outs[i]))
    assert differs  # some reversed order changed the arithmetic


@pytest.mark.parametrize("leave", [False, True])
def test_fused_schedule_matches_separate_stages(gpu_lib, leave):
    # FFT steps fused with their transposes run the same passes on the same data
    items = inputs.batch_items(24, seed=5)
    xs = [inputs.uniform(d, 500 + i, np.complex64) for i, (d, _) in enumerate(items)]
    extra = fftrw.FLAG_LEAVE_PERMUTED if leave else 0
    fused = fftrw.Batch(items, flags=fftrw.FLAG_COUNT_MOVED | extra)
    plain = fftrw.Batch(items, flags=fftrw.FLAG_COUNT_MOVED | fftrw.FLAG_BATCH_NO_FUSE | extra)
    for fwd in (True, False):
        _, a = _run(fused, xs, fwd)
        _, b = _run(plain, xs, fwd)
        for i in range(len(items)):
            assert np.array_equal(to_host(a[i]), to_host(b[i])), (i, fwd)
    sa, sb = fused.stats(), plain.stats()
    assert sa["error"] == 0 and sb["error"] == 0
    assert sa["moved"] == sb["moved"]
    for mi, ai in zip(sa["moved"], sa["analytic"]):
        assert all(m == -1 or m == a_ for m, a_ in zip(mi, ai))
        assert (mi[-1] == -1) == leave


def test_in_place_needs_the_separate_schedule(gpu_lib):
    items = [((12, 16, 20), 5), ((16, 16, 16, 16), 30)]
    xs = [inputs.uniform(d, 70 + i, np.complex64) for i, (d, _) in enumerate(items)]
    ins = [to_dev(x) for x in xs]
    with pytest.raises(fftrw.FftrwError) as e:
        fftrw.Batch(items).exec_fwd(ins, ins)
    assert e.value.code == fftrw.E_ARG
    b = fftrw.Batch(items, flags=fftrw.FLAG_BATCH_NO_FUSE)
    b.exec_fwd(ins, ins)
    for i, (d, P) in enumerate(items):
        order = fftrw.fft_order_search(d, P)["best_order"]
        ref = dft.fftn_direct(xs[i], orders.fft_axis_sequence(order))
        assert dft.rel_l2(to_host(ins[i]), ref) < 1e-5


@pytest.mark.parametrize("flags", [0, fftrw.FLAG_BATCH_NO_FUSE])
def test_long_rows_in_a_batch(gpu_lib, flags):
    # a row longer than 2047 points switches the batch to 16 values per lane
    items = [((2560, 3, 2), 3), ((12, 15, 16), 5), ((4096, 2, 2), 2)]
    xs = [inputs.uniform(d, 80 + i, np.complex64) for i, (d, _) in enumerate(items)]
    b = fftrw.Batch(items, flags=flags | fftrw.FLAG_COUNT_MOVED)
    ins, outs = _run(b, xs)
    st = b.stats()
    assert st["error"] == 0
    for i, (dims, P) in enumerate(items):
        order = fftrw.fft_order_search(dims, P)["best_order"]
        ref = dft.fftn_direct(xs[i], orders.fft_axis_sequence(order))
        assert dft.rel_l2(to_host(outs[i]), ref) < 1e-5, (i, dims)
        assert st["moved"][i] == st["analytic"][i]


def test_barrier_timeout_is_reported(gpu_lib, monkeypatch):
    # force the time-out path from the host: a level wait bounded by 0 ticks
    # ends at once, so the batch's results are not reliable -- the sticky
    # count says so, stats fails with E_DEVICE and the batch refuses to run
    # again; a batch planned without the hook is unaffected
    items = [((16, 12, 10, 8), 20), ((20, 18, 24, 6), 7), ((12, 15, 16), 5)] * 8
    xs = [inputs.uniform(d, 40 + i, np.complex64) for i, (d, _) in enumerate(items)]
    monkeypatch.setenv("FFTRW_BATCH_WAIT_TICKS", "0")
    b = fftrw.Batch(items, flags=fftrw.FLAG_COUNT_MOVED)
    monkeypatch.delenv("FFTRW_BATCH_WAIT_TICKS")
    ins, outs = _run(b, xs)
    with pytest.raises(fftrw.FftrwError) as e:
        b.stats()
    assert e.value.code == fftrw.E_DEVICE and "timed out" in str(e.value)
    with pytest.raises(fftrw.FftrwError) as e:
        b.exec_fwd(ins, outs)
    assert e.value.code == fftrw.E_DEVICE
    ok = fftrw.Batch(items, flags=fftrw.FLAG_COUNT_MOVED)
    _, outs2 = _run(ok, xs)
    assert ok.stats()["error"] == 0
    for i, (dims, P) in enumerate(items[:3]):
        order = fftrw.fft_order_search(dims, P)["best_order"]
        ref = dft.fftn_direct(xs[i], orders.fft_axis_sequence(order))
        assert dft.rel_l2(to_host(outs2[i]), ref) < 1e-5

#!/usr/bin/env python3
"""Benchmark of the row-wise decomposed 3-D FFT on one MI355X.

Workload: 3-D complex64 FFT of 512 x 512 x 512 points over P = 4096 virtual
processes (two-level decomposition) with the best transpose order, FP32 math,
inputs re/im i.i.d. U[-1, 1) resident in HBM.  One step = one forward and one
inverse transform (natural-order input and output), each the whole Fig. 4
pipeline: 3 FFT passes, 2 order transposes and the return transpose, with
the owner changes of every transpose counted on the device.

Prints one JSON line: effective GFLOP/s (5 T log2 T per transform), the
per-kernel HBM roofline of the dominant kernel from HIP events recorded on
the exec stream, and the FP64 oracle timed on a bounded sample on the host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "effective GFLOP/s (5N·log2N) + HBM GB/s % peak, 512^3 c64 FP32 vs MFMA vs batched"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_512cube.json")
KERNEL_SOURCES = ["paper_1302_6189_amd/csrc/fft_pow2.hip", "paper_1302_6189_amd/csrc/xpose_tile.hpp",
                  "paper_1302_6189_amd/csrc/cplx.hpp", "paper_1302_6189_amd/csrc/kernels.hpp"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None if the kernel sources changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def progress(what):
    """One line on stderr as each leg of the run ends (the JSON line goes to stdout)."""
    print(f"bench: {what}", file=sys.stderr, flush=True)


def cpu_baseline(dims, x_host, P, order):
    """The FP64 oracle, as it stands, on a bounded sample: every axis's 1-D FFT
    pass over a quarter of the array (whole rows), scaled to one transform; then
    the same on one thread over a sixteenth of the array; and the oracle's
    point-by-point owner counting of one order's amounts (the order search
    repeats it for every order) beside the library's whole search."""
    import numpy as np

    from oracle import dft
    T = math.prod(dims)

    def passes(S):
        t0 = time.perf_counter()
        dft.fft_along_axis(x_host[0:S].astype(np.complex128), 2)
        dft.fft_along_axis(x_host[0:S].astype(np.complex128), 1)
        dft.fft_along_axis(x_host[:, 0:S].astype(np.complex128), 0)
        return time.perf_counter() - t0

    threads = dft.num_threads()
    S = dims[0] // 4
    sec = passes(S)
    full = sec * dims[0] / S
    dft.set_threads(1)
    S1 = dims[0] // 16
    sec1 = passes(S1)
    dft.set_threads(threads)
    full1 = sec1 * dims[0] / S1
    return {"value": round(5 * T * math.log2(T) / full / 1e9, 3), "unit": "GFLOP/s",
            "cores": threads, "kind": "oracle",
            "sample": f"FP64 recursive-FFT oracle, each axis's pass over 1/4 of the 512^3 array "
                      f"({sec:.2f} s measured, x{dims[0] // S} to one transform)",
            "one_thread": {"value": round(5 * T * math.log2(T) / full1 / 1e9, 3), "unit": "GFLOP/s",
                           "sample": f"each axis's pass over 1/16 of the array on one thread ({sec1:.2f} s, "
                                     f"x{dims[0] // S1})"},
            "order_amounts": order_amounts(dims, P, order),
            "cpu_model": cpu_model(), "nproc": os.cpu_count()}


def order_amounts(dims, P, order):
    """Seconds for the oracle's amounts of one transpose order (its transposes
    and the return, from per-process owner counts) and for the library's exact
    search over all orders."""
    from oracle import decomp
    from paper_1302_6189_amd import fftrw
    M = len(dims)
    t0 = time.perf_counter()
    steps, ret = decomp.order_volumes(dims, P, order)
    sec = time.perf_counter() - t0
    t0 = time.perf_counter()
    search = fftrw.fft_order_search(dims, P)
    lib_sec = time.perf_counter() - t0
    lib_steps, _, lib_ret = fftrw.fft_comm_volume(dims, P, order)
    n = fftrw.fft_order_count(M)
    return {"oracle_s_per_order": round(sec, 2), "orders": n,
            "oracle_s_all_orders": round(sec * n, 1), "library_search_s": round(lib_sec, 4),
            "amounts_equal": [int(v) for v in steps] == list(lib_steps) and int(ret) == lib_ret,
            "best_order": fftrw.order_to_str(search["best_order"]),
            "sample": f"the oracle's literal amounts of order {fftrw.order_to_str(order)} at N_p = {P} "
                      f"(x{n} for every order)"}


def time_fwd(plan, x, y, stream, reps, warm=3):
    """Average milliseconds of one forward transform (HIP events on the exec stream)."""
    import torch
    for _ in range(warm):
        plan.exec_fwd(x, y, stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        plan.exec_fwd(x, y, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def precision_forms(reps, dims=(256, 256, 256), P=64):
    """A 3-D complex64 transform (256^3 at P = 64, or 512^3 at P = 4096; best
    order): FP32 Stockham against the split FP16 / BF16 / BF16x3 MFMA forms
    (256-point rows as two radix-16 contractions, 512-point rows as two such
    halves and a radix-2 combination); time per transform and errors against
    the FP64 oracle on uniform and log-uniform inputs.  Errors are computed first;
    the timings follow back to back (the host-side error checks leave the GPU
    idle for seconds, and a short timed run right after them would include the
    clock ramp), each form timed three times, interleaved, median reported."""
    import numpy as np
    import torch

    from oracle import dft, orders
    from paper_1302_6189_amd import fftrw, inputs
    T = math.prod(dims)
    order = fftrw.fft_order_search(dims, P)["best_order"]
    seq = orders.fft_axis_sequence(order)
    data = {}
    for kind, seed in (("uniform", 4), ("log_uniform", 40)):
        x = getattr(inputs, kind)(dims, seed, np.complex64)
        data[kind] = (x, dft.fftn_direct(x, seq))
    stream = torch.cuda.current_stream()
    forms = (("fp32", fftrw.PREC_NATIVE), ("split_f16", fftrw.PREC_SPLIT_F16),
             ("split_bf16", fftrw.PREC_SPLIT_BF16), ("split_bf16x3", fftrw.PREC_SPLIT_BF16X3))
    xd = torch.from_numpy(data["uniform"][0]).cuda()
    yd = torch.empty_like(xd)
    res, plans = {}, {}
    for name, prec in forms:
        plan = fftrw.Plan(dims, P, order, precision=prec, flags=fftrw.FLAG_SEPARATE)
        fplan = fftrw.Plan(dims, P, order, precision=prec, flags=fftrw.FLAG_FUSED_FFT)
        plans[name] = (plan, fplan)
        entry = {}
        for kind, (x, ref) in data.items():
            xk = torch.from_numpy(x).cuda()
            yk = torch.empty_like(xk)
            plan.exec_fwd(xk, yk, stream)
            torch.cuda.synchronize()
            y = yk.cpu().numpy()
            entry[kind] = {"rel_l2": float(f"{dft.rel_l2(y, ref):.3e}"),
                           "max_abs": float(f"{dft.max_abs(y, ref):.3e}"),
                           "max_abs_over_max_ref": float(f"{dft.max_abs_rel(y, ref):.3e}")}
            del xk, yk
        res[name] = entry
    n = max(reps, 50)
    times = {name: ([], []) for name, _ in forms}
    for _ in range(3):
        for name, _ in forms:
            plan, fplan = plans[name]
            times[name][0].append(time_fwd(plan, xd, yd, stream, n, warm=20))
            times[name][1].append(time_fwd(fplan, xd, yd, stream, n, warm=20))
    for name, _ in forms:
        plan, fplan = plans[name]
        entry = res[name]
        ms = float(np.median(times[name][0]))
        entry["ms_per_transform"] = round(ms, 4)
        entry["GFLOPs"] = round(5 * T * math.log2(T) / (ms * 1e-3) / 1e9, 1)
        plan.set_timing(True)
        plan.exec_fwd(xd, yd, stream)
        st = plan.timings()
        plan.set_timing(False)
        entry["fft_pass_ms"] = round(sum(st[0::2]) / 3, 4)
        entry["fft_pass_GBs"] = round(2 * T * 8 / (entry["fft_pass_ms"] * 1e-3) / 1e9, 1)
        # the same arithmetic with each FFT step fused with its transpose
        fms = float(np.median(times[name][1]))
        fplan.set_timing(True)
        fplan.exec_fwd(xd, yd, stream)
        fst = fplan.timings()
        fplan.set_timing(False)
        entry["fused"] = {"ms_per_transform": round(fms, 4),
                          "GFLOPs": round(5 * T * math.log2(T) / (fms * 1e-3) / 1e9, 1),
                          "step_ms": round(sum(fst) / len(fst), 4),
                          "step_GBs": round(2 * T * 8 / (sum(fst) / len(fst) * 1e-3) / 1e9, 1),
                          "kernels": fplan.describe()[1]}
        plan.destroy()
        fplan.destroy()
    del xd, yd
    res["timing"] = f"median of 3 interleaved runs of {n} transforms after 20 warm-up transforms"
    res["workload"] = (f"3-D complex64 FFT {'x'.join(map(str, dims))}, P={P}, order "
                       + fftrw.order_to_str(order))
    return res


def batched_form(reps):
    """256 uneven 3-D/4-D/5-D complex64 items (sizes 2^a 3^b 5^c in [12, 192],
    T <= 2^22, N_p in [1, 64], best orders): one persistent graph-replayed
    launch against loops launching each item's own plan, once with fused
    steps (the same per-step work as the batch's fused stages: like for like)
    and once with separate FFT and transpose kernels."""
    import numpy as np
    import torch

    from paper_1302_6189_amd import fftrw, inputs
    items = inputs.batch_items(256, seed=5)
    xs = [torch.from_numpy(inputs.uniform(d, 1000 + i, np.complex64)).cuda() for i, (d, _) in enumerate(items)]
    ys = [torch.empty_like(x) for x in xs]
    stream = torch.cuda.current_stream()
    Ts = [math.prod(d) for d, _ in items]
    flops = sum(5 * T * math.log2(T) for T in Ts)
    alg_bytes = sum(4 * 8 * len(d) * T for (d, _), T in zip(items, Ts))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def run_batch(cache):
        batch = fftrw.Batch(items, flags=fftrw.FLAG_COUNT_MOVED, tune_cache=cache)
        for _ in range(3):
            batch.exec_fwd(xs, ys, stream)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            batch.exec_fwd(xs, ys, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        st = batch.stats()
        batch.destroy()
        return ms, st

    import tempfile
    cache = os.path.join(tempfile.gettempdir(), "fftrw_tune_batch256.json")
    t0 = time.perf_counter()
    fftrw.fft_autotune(items, cache)
    tune_s = time.perf_counter() - t0
    ms_untuned, _ = run_batch(None)
    ms_batch, st = run_batch(cache)
    counts_ok = all(m == a for m, a in zip(st["moved"], st["analytic"]))

    def run_loop(flags):
        plans = [fftrw.Plan(d, P, None, flags=flags) for d, P in items]
        fused = sum(p.describe()[1].startswith("fused|") for p in plans)
        launches = sum(len(d) if p.describe()[1].startswith("fused|") else 2 * len(d)
                       for (d, _), p in zip(items, plans))
        for _ in range(2):
            for p, x, y in zip(plans, xs, ys):
                p.exec_fwd(x, y, stream)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            for p, x, y in zip(plans, xs, ys):
                p.exec_fwd(x, y, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        for p in plans:
            p.destroy()
        return e0.elapsed_time(e1) / reps, launches, fused

    ms_loop, launches_loop, n_fused = run_loop(fftrw.FLAG_FUSED_FFT)
    ms_loop_sep, launches_sep, _ = run_loop(fftrw.FLAG_SEPARATE)
    res = {"workload": "256 items, M in {3,4,5}, sizes 2^a3^b5^c in [12,192], T<=2^22, P in [1,64], "
                       "best orders, complex64, seed 13026189+5",
           "points": sum(Ts), "units_per_launch": st["units"],
           # time-outs summed over every launch of the timed batch (sticky count)
           "barrier_timeouts": st["error"],
           "device_counts_match_analytic": counts_ok,
           "persistent_graph": {"ms": round(ms_batch, 4), "GFLOPs": round(flops / (ms_batch * 1e-3) / 1e9, 1),
                                "algorithmic_GBs": round(alg_bytes / (ms_batch * 1e-3) / 1e9, 1),
                                # fused stages: one read and one write of every point per step
                                "fused_hbm_GBs": round(alg_bytes / 2 / (ms_batch * 1e-3) / 1e9, 1),
                                "autotuned": True, "autotune_s": round(tune_s, 2),
                                "ms_without_autotune": round(ms_untuned, 4)},
           "per_item_loop": {"ms": round(ms_loop, 4), "GFLOPs": round(flops / (ms_loop * 1e-3) / 1e9, 1),
                             "algorithmic_GBs": round(alg_bytes / (ms_loop * 1e-3) / 1e9, 1),
                             "launches": launches_loop, "items_fused": n_fused,
                             "kernels": "each FFT step fused with its transpose where the plan fuses"},
           "per_item_loop_separate": {"ms": round(ms_loop_sep, 4),
                                      "GFLOPs": round(flops / (ms_loop_sep * 1e-3) / 1e9, 1),
                                      "launches": launches_sep,
                                      "kernels": "separate FFT and transpose kernels"},
           "speedup_vs_loop": round(ms_loop / ms_batch, 3),
           "speedup_vs_separate_loop": round(ms_loop_sep / ms_batch, 3)}
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--P", type=int, default=4096)
    ap.add_argument("--order", default="best", help="best, worst or a canonical order index")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the precision and batched legs")
    ap.add_argument("--staged", action="store_true",
                    help="also time the staged pack -> exchange -> unpack transposes")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="one forward transform plus a plain 1 GiB device copy, for counter runs")
    ap.add_argument("--batch-probe", action="store_true",
                    help="the 256-item batched form: one warm-up and one counted launch, for counter runs")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "fftrw runs on one GPU: the virtual processes of the decomposition "
                                   "share a single device; run with --gpus 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1302_6189_amd import fftrw, inputs

    if args.batch_probe:
        # counters are read per dispatch: the batched form's persistent kernel
        # (built-in radix lists, no autotuner), launched twice
        items = inputs.batch_items(256, seed=5)
        xs = [torch.from_numpy(inputs.uniform(d, 1000 + i, np.complex64)).cuda() for i, (d, _) in enumerate(items)]
        ys = [torch.empty_like(v) for v in xs]
        batch = fftrw.Batch(items, flags=fftrw.FLAG_COUNT_MOVED)
        for _ in range(2):
            batch.exec_fwd(xs, ys, torch.cuda.current_stream())
        torch.cuda.synchronize()
        st = batch.stats()
        batch.destroy()
        print(json.dumps({"batch_probe": "done", "units": st["units"], "timeouts": st["error"],
                          "counts_match": st["moved"] == st["analytic"]}), flush=True)
        return

    dims = (512, 512, 512)
    T = math.prod(dims)
    P = args.P
    search = fftrw.fft_order_search(dims, P)
    if args.order == "best":
        order = search["best_order"]
    elif args.order == "worst":
        order = search["worst_order"]
    else:
        order = fftrw.fft_order_at(3, int(args.order))
    plan = fftrw.Plan(dims, P, order, dtype=fftrw.C64, flags=fftrw.FLAG_COUNT_MOVED | fftrw.FLAG_FUSED_FFT)
    _, radices = plan.describe()
    fused = radices.startswith("fused|")

    x_host = inputs.uniform(dims, 2, np.complex64)
    x = torch.from_numpy(x_host).cuda()
    y = torch.empty_like(x)
    z = torch.empty_like(x)
    stream = torch.cuda.current_stream()

    if args.pmc_probe:
        # counters are read per dispatch: one forward transform, then a plain
        # copy of the same 1 GiB as the calibration for the HBM byte counters
        plan.exec_fwd(x, y, stream)
        torch.cuda.synchronize()
        z.copy_(x)
        torch.cuda.synchronize()
        # the staged path of the same order: pack, exchange and unpack per transpose
        sp = fftrw.Plan(dims, P, order, dtype=fftrw.C64, flags=fftrw.FLAG_STAGED)
        sp.exec_fwd(x, y, stream)
        torch.cuda.synchronize()
        steps, _, ret = fftrw.fft_comm_volume(dims, P, order)
        sp.destroy()
        print(json.dumps({"pmc_probe": "done", "bytes_per_copy": 2 * T * 8, "staged_moved": steps + [ret]}),
              flush=True)
        return

    for _ in range(args.warmup):
        plan.exec_fwd(x, y, stream)
        plan.exec_inv(y, z, stream)
    torch.cuda.synchronize()

    # ---- timed region: K steps of forward + inverse ----------------------------
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        plan.exec_fwd(x, y, stream)
        plan.exec_inv(y, z, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_per_step = e0.elapsed_time(e1) / args.steps
    analytic, moved = plan.stats()

    # ---- per-kernel durations from HIP events on the exec stream ---------------
    plan.set_timing(True)
    n_rep = max(3, args.steps // 2)
    stage_ms = None
    for _ in range(n_rep):
        for fn, a, b in ((plan.exec_fwd, x, y), (plan.exec_inv, y, z)):
            fn(a, b, stream)
            tms = plan.timings()
            stage_ms = [0.0] * len(tms) if stage_ms is None else stage_ms
            stage_ms = [s + t for s, t in zip(stage_ms, tms)]
    plan.set_timing(False)
    stage_ms = [s / (2 * n_rep) for s in stage_ms]
    bytes_per_launch = 2 * T * 8  # every point read once and written once
    if fused:
        # every launch of the timed region is this one kernel (3 per transform,
        # 2 transforms per step): its average duration is the region's time,
        # bracketed by HIP events on the exec stream, over its launches (the
        # gaps between launches, under 1%, included)
        kernels = {"fft_xpose_kernel": {"avg_ms": ms_per_step / (2 * len(stage_ms)),
                                        "launches_per_transform": len(stage_ms),
                                        "avg_ms_stage_events": sum(stage_ms) / len(stage_ms)}}
    else:
        fft_ms, xp_ms = stage_ms[0::2], stage_ms[1::2]
        kernels = {
            "fft_pow2_kernel": {"avg_ms": sum(fft_ms) / len(fft_ms), "launches_per_transform": len(fft_ms)},
            "xpose_kernel": {"avg_ms": sum(xp_ms) / len(xp_ms), "launches_per_transform": len(xp_ms)},
        }
    dom = max(kernels, key=lambda n: kernels[n]["avg_ms"] * kernels[n]["launches_per_transform"])
    ach = bytes_per_launch / (kernels[dom]["avg_ms"] * 1e-3) / 1e9
    for k in kernels.values():
        k["achieved_GBs"] = round(bytes_per_launch / (k["avg_ms"] * 1e-3) / 1e9, 1)
        k["avg_ms"] = round(k["avg_ms"], 5)
        if "avg_ms_stage_events" in k:
            k["avg_ms_stage_events"] = round(k["avg_ms_stage_events"], 5)
    traffic = measured_traffic(dom)

    flops_per_transform = 5 * T * math.log2(T)
    value = 2 * flops_per_transform / (ms_per_step * 1e-3) / 1e9
    # bytes the kernels move per transform: every launch reads and writes T points once
    launches = sum(k["launches_per_transform"] for k in kernels.values())
    moved_bytes_per_transform = launches * 2 * T * 8
    hbm_gbs = 2 * moved_bytes_per_transform / (ms_per_step * 1e-3) / 1e9

    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "3-D complex64 FFT 512x512x512, forward+inverse per step",
                   "P": P, "order": fftrw.order_to_str(order), "radices": radices,
                   "transpose": ("each FFT step fused with its transpose" if fused else "separate transpose kernels")
                                + ", owner changes counted on device",
                   "input": "re/im i.i.d. U[-1,1), seed 13026189+2"},
        "hbm_GBs": round(hbm_gbs, 1),
        "hbm_frac_of_peak": round(hbm_gbs / HBM_PEAK_GBS, 4),
        "kernel_launches_per_transform": launches,
        "ms_per_transform": round(ms_per_step / 2, 4),
        "comm_amount_points": {"per_step": analytic[:-1], "return": analytic[-1],
                               "device_counted": moved, "search_best": search["best_volume"],
                               "search_worst": search["worst_volume"]},
        "per_kernel": kernels,
        "stage_ms": [round(s, 4) for s in stage_ms],
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     # achieved = bytes_per_launch / avg_launch_ms; a launch moves every
                     # point once each way: 2 x 8 x T bytes
                     "bytes_per_launch": bytes_per_launch,
                     "avg_launch_ms": kernels[dom]["avg_ms"]},
        "wall_s_timed": round(wall, 3),
    }
    # the unfused pipeline (separate FFT and transpose kernels) for comparison
    plain = fftrw.Plan(dims, P, order, dtype=fftrw.C64, flags=fftrw.FLAG_COUNT_MOVED | fftrw.FLAG_SEPARATE)
    ms_plain = time_fwd(plain, x, y, stream, args.steps)
    plain.set_timing(True)
    plain.exec_fwd(x, y, stream)
    st_plain = plain.timings()
    plain.destroy()
    out["unfused_pipeline"] = {"ms_per_transform": round(ms_plain, 4),
                               "GFLOPs": round(flops_per_transform / (ms_plain * 1e-3) / 1e9, 1),
                               "stage_ms": [round(v, 4) for v in st_plain]}
    progress("headline and separate pipeline done")
    if args.staged:
        # explicit per-process buffers: pack, exchange of exactly the moved
        # points, unpack (the exchange's traffic is 2 x 8 x V_t bytes)
        stg = {}
        for Ps in sorted({8, P}):
            t0 = time.perf_counter()
            sp = fftrw.Plan(dims, Ps, order, dtype=fftrw.C64, flags=fftrw.FLAG_STAGED)
            plan_s = time.perf_counter() - t0
            ms_s = time_fwd(sp, x, y, stream, max(3, args.steps // 4), warm=1)
            sp.set_timing(True)
            sp.exec_fwd(x, y, stream)
            st_s = sp.timings()
            a_s, m_s = sp.stats()
            stg[f"P{Ps}"] = {"ms_per_transform": round(ms_s, 4), "plan_s": round(plan_s, 2),
                             "stage_ms": [round(v, 4) for v in st_s], "exchanged_points": m_s,
                             "analytic": a_s, "device_bytes": sp.workspace_bytes()}
            sp.destroy()
        out["staged_pipeline"] = stg
    del x, y, z
    if not args.no_forms:
        torch.cuda.empty_cache()
        out["precision_form"] = precision_forms(args.steps)
        progress("precision forms at 256^3 done")
        torch.cuda.empty_cache()
        out["precision_form_512cube"] = precision_forms(args.steps, (512, 512, 512), 4096)
        progress("precision forms at 512^3 done")
        torch.cuda.empty_cache()
        out["batched_form"] = batched_form(max(5, args.steps // 2))
        progress("batched form done")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(dims, x_host, P, order)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""Measured time of transpose orders against their communication amount.

Section 4 ranks transpose orders by the number of points each moves
(Eq. (20) counts the orders; Table 1).  This module times the orders on the
device and relates the time to that amount:

* every order of a 4-D array end to end, in three execution modes: the fused
  path (each FFT step fused with its transpose), separate FFT and transpose
  kernels, and the staged path (pack, exchange of exactly the moved points,
  unpack);
* for M = 5, where there are 7,962,624 orders, the time of an order composed
  from measured parts: one FFT step per row length and one transpose per
  distinct (layout, next layout) pair, checked end to end on a sample.

A transpose pi -> sigma of an array with sizes D is the same memory operation
as identity -> pi^{-1} o sigma on the array whose sizes are D permuted by pi
(the decomposition relabels the same way), so each pair is timed as the first
transpose of a plan over the permuted sizes.  Run as
``python -m paper_1302_6189_amd.order_study --dims 64,64,64,64 --P 48``.
"""
import argparse
import itertools
import json
import sys
import time

import numpy as np

from . import fftrw

MODES = {"fused": fftrw.FLAG_FUSED_FFT, "separate": fftrw.FLAG_SEPARATE, "staged": fftrw.FLAG_STAGED}
SEED = 13026189


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def order_table(M):
    """All orders as rows of indices into the lexicographic permutation list,
    in canonical order (row i is the order of canonical index i)."""
    perms = list(itertools.permutations(range(M)))
    last = np.array([p[-1] for p in perms], dtype=np.int64)
    seq = np.zeros((1, 1), dtype=np.int16)
    used = np.array([1 << (M - 1)], dtype=np.int64)
    for _ in range(1, M):
        ok = ((used[:, None] >> last[None, :]) & 1) == 0
        r, c = np.nonzero(ok)
        seq = np.hstack([seq[r], c[:, None].astype(np.int16)])
        used = used[r] | (np.int64(1) << last[c])
    return perms, seq


def complete_order(M, sigma):
    """A valid order that starts identity -> sigma."""
    order = [tuple(range(M)), tuple(sigma)]
    lasts = {M - 1, sigma[-1]}
    for l in range(M):
        if l in lasts:
            continue
        order.append(tuple([a for a in range(M) if a != l] + [l]))
        lasts.add(l)
    return tuple(order)


def relabel(dims, pi, sigma):
    """(sizes permuted by pi, pi^{-1} o sigma): the pair as a first transpose."""
    pos = {a: i for i, a in enumerate(pi)}
    return tuple(dims[a] for a in pi), tuple(pos[a] for a in sigma)


class Timer:
    def __init__(self, stream):
        import torch
        self.torch = torch
        self.stream = stream

    def __call__(self, fn, reps):
        torch = self.torch
        fn()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        ev[0].record(self.stream)
        for i in range(reps):
            fn()
            ev[i + 1].record(self.stream)
        torch.cuda.synchronize()
        return float(np.median([ev[i].elapsed_time(ev[i + 1]) for i in range(reps)]))


def linear_fit(v, t):
    v = np.asarray(v, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    if len(v) < 3 or np.ptp(v) == 0:
        return None
    b, a = np.polyfit(v, t, 1)
    pred = a + b * v
    ss_res = float(np.sum((t - pred) ** 2))
    ss_tot = float(np.sum((t - t.mean()) ** 2))
    rv = np.argsort(np.argsort(v))
    rt = np.argsort(np.argsort(t))
    spearman = float(np.corrcoef(rv, rt)[0, 1])
    out = {"intercept_ms": a, "slope_ms_per_point": b, "r2": 1 - ss_res / ss_tot if ss_tot > 0 else None,
           "pearson": float(np.corrcoef(v, t)[0, 1]), "spearman": spearman}
    # complex64: an exchanged point is read once and written once
    out["effective_exchange_GBs"] = (16.0 / (b * 1e-3) / 1e9) if b > 0 else None
    return out


def two_term_fit(v, n, t):
    """t = a + b v + c n (time per point and per message), least squares."""
    v, n, t = (np.asarray(z, dtype=np.float64) for z in (v, n, t))
    if len(t) < 4:
        return None
    A = np.stack([np.ones_like(v), v, n], axis=1)
    coef, *_ = np.linalg.lstsq(A, t, rcond=None)
    pred = A @ coef
    ss_tot = float(np.sum((t - t.mean()) ** 2))
    return {"intercept_ms": float(coef[0]), "ms_per_point": float(coef[1]), "ms_per_message": float(coef[2]),
            "r2": 1 - float(np.sum((t - pred) ** 2)) / ss_tot if ss_tot > 0 else None,
            "effective_exchange_GBs": (16.0 / (coef[1] * 1e-3) / 1e9) if coef[1] > 0 else None}


def summary(v, t):
    v = np.asarray(v)
    t = np.asarray(t)
    ib, iw, fb = int(np.argmin(v)), int(np.argmax(v)), int(np.argmin(t))
    return {"ms_min": float(t.min()), "ms_median": float(np.median(t)), "ms_max": float(t.max()),
            "ms_at_min_volume": float(t[ib]), "ms_at_max_volume": float(t[iw]),
            "volume_of_fastest": int(v[fb]), "volume_min": int(v.min()), "volume_max": int(v.max()),
            "fastest_is_min_volume": bool(v[fb] == v.min()), "fit": linear_fit(v, t)}


def buffers(dims):
    import torch
    x = torch.empty(tuple(dims), dtype=torch.complex64, device="cuda")
    g = torch.Generator(device="cuda")
    g.manual_seed(SEED + 3)
    x.normal_(generator=g)
    return x, torch.empty_like(x)


def time_orders(dims, P, indices, modes, reps, timer, x, y):
    """End-to-end forward time of the given canonical orders in each mode."""
    M = len(dims)
    res = {m: [] for m in modes}
    plan_s = {m: 0.0 for m in modes}
    t_start = time.perf_counter()
    for n, idx in enumerate(indices):
        order = fftrw.fft_order_at(M, int(idx))
        for m in modes:
            t0 = time.perf_counter()
            plan = fftrw.Plan(dims, P, order, flags=MODES[m])
            plan_s[m] += time.perf_counter() - t0
            res[m].append(timer(lambda: plan.exec_fwd(x, y), reps))
            plan.destroy()
        if (n + 1) % 50 == 0:
            log(f"  {dims} P={P}: {n + 1}/{len(indices)} orders timed ({time.perf_counter() - t_start:.0f} s)")
    return res, plan_s


def return_volumes(dims, P, perms):
    """Points moved by the return transpose pi -> natural, per permutation."""
    M = len(dims)
    ident = tuple(range(M))
    out = np.zeros(len(perms), dtype=np.int64)
    for i, p in enumerate(perms):
        if p == ident or p[-1] == M - 1:
            continue
        C = fftrw.fft_pair_counts(dims, P, p, ident)
        out[i] = int(C.sum() - np.trace(C))
    return out


def transpose_parts(dims, P, perms, modes, reps, timer, x, y):
    """Time of every transpose pi -> sigma an order can contain (and the FFT
    step of each row length), measured once per distinct relabelled pair."""
    M = len(dims)
    ident = tuple(range(M))
    index = {p: i for i, p in enumerate(perms)}
    pairs = set()
    for p in perms:
        if p != ident and p[-1] == M - 1:
            continue
        for s in perms:
            if s[-1] == p[-1] or (s != ident and s[-1] == M - 1):
                continue
            pairs.add((p, s))
    keys = {}
    for p, s in pairs:
        keys.setdefault(relabel(dims, p, s), []).append((p, s))
    X = {m: np.full((len(perms), len(perms)), np.nan) for m in modes}
    parts = []
    t_start = time.perf_counter()
    for n, ((D, sig), members) in enumerate(sorted(keys.items())):
        order = complete_order(M, sig)
        for m in modes:
            plan = fftrw.Plan(D, P, order, flags=MODES[m])
            xv, yv = x.view(D), y.view(fftrw_layout(D, sig))
            ms = timer(lambda: plan.exec_transpose(0, xv, yv), reps)
            if m == "staged":
                # pack / exchange / unpack of this transpose (the plan's first),
                # from the stage timings of whole forward transforms
                plan.set_timing(True)
                st = []
                for _ in range(reps):
                    plan.exec_fwd(x.view(D), y.view(D))
                    st.append(plan.timings()[1:4])
                st = np.median(np.array(st), axis=0)
                vol = fftrw.fft_comm_volume(D, P, order)[0][0]
                parts.append({"sizes": list(D), "to": list(sig), "volume": int(vol), "messages": plan.messages()[0],
                              "transpose_ms": ms,
                              "pack_ms": float(st[0]), "exchange_ms": float(st[1]), "unpack_ms": float(st[2])})
            plan.destroy()
            for p, s in members:
                X[m][index[p], index[s]] = ms
        if (n + 1) % 50 == 0:
            log(f"  {dims} P={P}: {n + 1}/{len(keys)} transposes timed ({time.perf_counter() - t_start:.0f} s)")
    # FFT steps: one per row length, timed as step 0 of sizes ending in that length
    F = np.zeros(len(perms))
    by_len = {}
    for L in sorted(set(dims)):
        D = tuple(sorted(dims, key=lambda n: n == L))  # L last
        order = complete_order(M, tuple(list(range(M - 2)) + [M - 1, M - 2]))
        plan = fftrw.Plan(D, P, order, flags=0)
        xv, yv = x.view(D), y.view(D)
        by_len[L] = timer(lambda: plan.exec_fft_step(0, -1, xv, yv), reps)
        plan.destroy()
    for i, p in enumerate(perms):
        F[i] = by_len[dims[p[-1]]]
    return X, F, len(keys), by_len, parts


def fftrw_layout(dims, perm):
    return tuple(dims[a] for a in perm)


def composed_times(seq, X, F):
    M = seq.shape[1]
    t = np.zeros(len(seq))
    for s in range(M):
        t += F[seq[:, s]]
    for s in range(M - 1):
        t += X[seq[:, s], seq[:, s + 1]]
    t += X[seq[:, M - 1], 0]
    return t


def study(dims, P, modes, reps, all_orders, compose, n_random, n_ties):
    import torch
    fftrw.lib()
    M = len(dims)
    stream = torch.cuda.current_stream()
    timer = Timer(stream)
    x, y = buffers(dims)
    perms, seq = order_table(M)
    for i in (0, 1, len(seq) // 3, len(seq) - 1):
        assert tuple(perms[j] for j in seq[i]) == tuple(fftrw.fft_order_at(M, i)), i
    t0 = time.perf_counter()
    V = fftrw.fft_order_volumes(dims, P)
    R = return_volumes(dims, P, perms)
    ret = R[seq[:, -1]]
    out = {"dims": list(dims), "P": P, "orders": int(len(seq)), "modes": modes, "reps": reps,
           "volume_s": round(time.perf_counter() - t0, 2),
           "volume": {"min": int(V.min()), "max": int(V.max()), "median": float(np.median(V)),
                      "n_min": int((V == V.min()).sum()), "n_max": int((V == V.max()).sum()),
                      "max_over_min": float(V.max() / V.min())}}
    sr = fftrw.fft_order_search(dims, P)
    out["best_index"], out["worst_index"] = sr["best_index"], sr["worst_index"]
    if all_orders:
        idx = np.arange(len(seq))
        res, plan_s = time_orders(dims, P, idx, modes, reps, timer, x, y)
        out["all_orders"] = {m: summary(V, res[m]) for m in modes}
        out["all_orders_fit_with_return"] = {m: linear_fit(V + ret, res[m]) for m in modes}
        out["plan_s_total"] = {m: round(v, 2) for m, v in plan_s.items()}
        out["per_order_ms"] = {m: [round(v, 5) for v in res[m]] for m in modes}
        out["per_order_volume"] = V.tolist()
    if compose:
        cm = [m for m in modes if m != "fused"]
        X, F, nkeys, by_len, parts = transpose_parts(dims, P, perms, cm, reps, timer, x, y)
        out["composed"] = {"distinct_transposes": nkeys, "fft_step_ms_by_length": by_len}
        if parts:
            vol = [q["volume"] for q in parts]
            out["staged_parts"] = {
                "transposes": parts,
                "exchange_fit": linear_fit(vol, [q["exchange_ms"] for q in parts]),
                "exchange_fit_volume_messages": two_term_fit(vol, [q["messages"] for q in parts],
                                                             [q["exchange_ms"] for q in parts]),
                "pack_ms_median": float(np.median([q["pack_ms"] for q in parts])),
                "unpack_ms_median": float(np.median([q["unpack_ms"] for q in parts])),
                "transpose_fit": linear_fit(vol, [q["transpose_ms"] for q in parts])}
        comp = {}
        for m in cm:
            t = composed_times(seq, X[m], F)
            comp[m] = t
            out["composed"][m] = summary(V, t)
        # end-to-end check on a sample: best/worst by volume, ties at the
        # minimum, random orders
        rng = np.random.default_rng(SEED + 31)
        ties = np.flatnonzero(V == V.min())
        sample = {int(sr["best_index"]), int(sr["worst_index"])}
        sample |= set(rng.choice(ties, size=min(n_ties, len(ties)), replace=False).tolist())
        sample |= set(rng.integers(0, len(seq), size=n_random).tolist())
        sample = np.array(sorted(sample))
        res, _ = time_orders(dims, P, sample, cm, reps, timer, x, y)
        chk = {"n": int(len(sample))}
        for m in cm:
            meas = np.array(res[m])
            pred = comp[m][sample]
            rel = (pred - meas) / meas
            chk[m] = {"median_rel_error": float(np.median(rel)), "max_abs_rel_error": float(np.max(np.abs(rel))),
                      "measured": summary(V[sample], meas)}
            if all_orders:
                chk[m]["all_orders_composed_vs_measured_max_abs_rel"] = float(
                    np.max(np.abs(comp[m] - np.array(out["per_order_ms"][m])) / np.array(out["per_order_ms"][m])))
        out["composed"]["end_to_end_check"] = chk
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--dims", required=True, help="comma-separated sizes, e.g. 64,64,64,64")
    ap.add_argument("--P", type=int, required=True)
    ap.add_argument("--modes", default="fused,separate,staged")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--all-orders", action="store_true", help="time every order end to end")
    ap.add_argument("--compose", action="store_true", help="compose every order's time from measured parts")
    ap.add_argument("--random", type=int, default=1000, help="random orders checked end to end (with --compose)")
    ap.add_argument("--ties", type=int, default=96, help="minimum-volume orders checked end to end")
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    dims = tuple(int(v) for v in a.dims.split(","))
    res = study(dims, a.P, a.modes.split(","), a.reps, a.all_orders, a.compose, a.random, a.ties)
    with open(a.out, "w") as f:
        json.dump(res, f)
    log(json.dumps({k: v for k, v in res.items() if k not in ("per_order_ms", "per_order_volume")})[:3000])


if __name__ == "__main__":
    main()

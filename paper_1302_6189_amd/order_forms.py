"""Balanced-split forms of transpose orders and the exact optimum beyond 5-D.

Section 3.3 describes the best orders by their shape: an M-D order of the form
m1+m2 first transforms the last m2 axes while the first m1 stay in front in
natural order, then moves one arrangement of those m2 axes to the front and
transforms the first m1 axes behind it (3-D: 1+2 or 2+1; 4-D: 2+2; 5-D: 2+3
or 3+2), and expects 3+3 to be the good form for 6-D, whose
2,985,984,000,000 orders it could not search.

The library's order search is exact for every M (a dynamic program over the
current decomposition and the set of axes already transformed), so here the
expectation is checked: for each N_p the optimum over all orders against the
best order of each form, and across a range of N_p whether any order is best
at every N_p ("always best") and whether such orders have the 3+3 form.  An
order is always best exactly when its amount summed over the N_p equals the
sum of the per-N_p optima, so the same dynamic program on the summed
transpose amounts finds and counts them.

Run as ``python -m paper_1302_6189_amd.order_forms --dims 4,4,4,4,4,4
--P 2,4,8,16,32,64,128,256,512,1024 --ownership matched``.
"""
import argparse
import itertools
import json
import sys

import numpy as np

from . import fftrw


def form_orders(M, m1):
    """Orders of the form m1+m2 as tuples of permutations (sorted): the first
    m2 decompositions are the natural prefix (0..m1-1) followed by arrangements
    of the other axes, one transforming each of them; the last m1 share one
    arrangement of those axes as prefix, followed by arrangements of the first
    m1 axes, one transforming each."""
    m2 = M - m1
    head = tuple(range(m1))
    tail = tuple(range(m1, M))

    def chains(axes, start, n):
        # sequences of n arrangements of `axes` with distinct last axes, the
        # first one fixed to `start` when given
        out = []

        def rec(seq, used):
            if len(seq) == n:
                out.append(tuple(seq))
                return
            for p in itertools.permutations(axes):
                if p[-1] not in used:
                    rec(seq + [p], used | {p[-1]})

        if start is None:
            rec([], set())
        else:
            rec([start], {start[-1]})
        return out

    firsts = chains(tail, tail, m2)
    seconds = chains(head, None, m1)
    orders = []
    for f in firsts:
        for lead in itertools.permutations(tail):
            for s in seconds:
                orders.append(tuple(head + p for p in f) + tuple(lead + q for q in s))
    return sorted(orders)


def _perm_list(M):
    return list(itertools.permutations(range(M)))


def order_rows(orders, M):
    """Orders as rows of lexicographic permutation indices."""
    idx = {p: i for i, p in enumerate(_perm_list(M))}
    return np.array([[idx[p] for p in o] for o in orders], dtype=np.int64)


def amounts(table, rows):
    """Total amount of each order (rows of permutation indices)."""
    return sum(table[rows[:, t], rows[:, t + 1]] for t in range(rows.shape[1] - 1))


def optimum_count(table, M):
    """(least total, number of orders attaining it) over all orders for a
    transpose table (-1 = pair in no order), by the dynamic program over
    (decomposition, transformed axes)."""
    perms = _perm_list(M)
    n = len(perms)
    last = np.array([p[-1] for p in perms])
    full = (1 << M) - 1
    big = np.iinfo(np.int64).max // 4
    val = {}
    cnt = {}
    masks = sorted((U for U in range(1, full + 1) if U >> (M - 1) & 1), key=lambda U: -bin(U).count("1"))
    for U in masks:
        v = np.full(n, big, dtype=np.int64)
        c = np.zeros(n, dtype=np.int64)
        if U == full:
            v[:] = 0
            c[:] = 1
        else:
            for a in range(n):
                if not (U >> last[a]) & 1:
                    continue
                if last[a] == M - 1 and (a != 0 or U != 1 << (M - 1)):
                    continue
                best, ways = big, 0
                for ax in range(M):
                    if (U >> ax) & 1:
                        continue
                    nxt = U | (1 << ax)
                    bs = np.flatnonzero(last == ax)
                    tot = table[a, bs] + val[nxt][bs]
                    m = tot.min()
                    if m < best:
                        best, ways = m, int(cnt[nxt][bs][tot == m].sum())
                    elif m == best:
                        ways += int(cnt[nxt][bs][tot == m].sum())
                v[a], c[a] = best, ways
        val[U], cnt[U] = v, c
    start = 1 << (M - 1)
    return int(val[start][0]), int(cnt[start][0])


def study(dims, Ps, ownership=fftrw.OWN_LITERAL, forms=None):
    M = len(dims)
    if forms is None:
        forms = [m1 for m1 in range(1, M) if min(m1, M - m1) >= M // 2 - 1] if M > 3 else [1, 2]
    fam = {m1: order_rows(form_orders(M, m1), M) for m1 in forms}
    per_p = []
    summed = None
    fam_sum = {m1: np.zeros(len(r), dtype=np.int64) for m1, r in fam.items()}
    opt_sum = 0
    for P in Ps:
        tab = fftrw.fft_transpose_volumes(dims, P, ownership)
        r = fftrw.fft_order_search(dims, P, ownership=ownership)
        row = {"P": P, "best": r["best_volume"], "n_best": r["n_best"], "worst": r["worst_volume"],
               "best_order": fftrw.order_to_str(r["best_order"]), "forms": {}}
        for m1, rows in fam.items():
            v = amounts(tab, rows)
            fam_sum[m1] += v
            row["forms"][f"{m1}+{M - m1}"] = {"best": int(v.min()),
                                             "at_optimum": int(np.count_nonzero(v == r["best_volume"])),
                                             "size": len(rows)}
        per_p.append(row)
        opt_sum += r["best_volume"]
        masked = np.where(tab < 0, 0, tab)
        summed = masked if summed is None else summed + masked
    summed = np.where(tab < 0, -1, summed)
    least, ways = optimum_count(summed, M)
    always = ways if least == opt_sum else 0
    fam_always = {f"{m1}+{M - m1}": int(np.count_nonzero(s == opt_sum)) for m1, s in fam_sum.items()}
    return {"dims": list(dims), "P": list(Ps), "ownership": "matched" if ownership else "literal",
            "per_P": per_p, "always_best": always, "always_best_by_form": fam_always}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--dims", required=True)
    ap.add_argument("--P", required=True, help="comma-separated process counts")
    ap.add_argument("--ownership", choices=["literal", "matched"], default="literal")
    ap.add_argument("--forms", default=None, help="comma-separated m1 values (default: the balanced ones)")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    dims = tuple(int(x) for x in a.dims.split(","))
    Ps = [int(x) for x in a.P.split(",")]
    forms = [int(x) for x in a.forms.split(",")] if a.forms else None
    res = study(dims, Ps, fftrw.OWN_MATCHED if a.ownership == "matched" else fftrw.OWN_LITERAL, forms)
    text = json.dumps(res, indent=1)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text + "\n")
    print(text)
    return 0


if __name__ == "__main__":
    sys.exit(main())

"""Transpose orders (Section 3.2, Eq. (20), Table 1) for the oracle.

TEST INFRASTRUCTURE ONLY: imported by tests and the benchmark's CPU-baseline
leg, never by the product path.

An order is a sequence of M decompositions pi_1, ..., pi_M (axis permutations
written slowest -> fastest).  pi_1 is the natural order (the paper's first
transpose has a single case); the 1-D FFTs of step t run along the last axis
of pi_t (Fig. 4), so the last axes of pi_1..pi_M are all different, while the
other M-1 axes of each pi_t may be arranged freely.

Canonical enumeration: all valid (pi_2, ..., pi_M) in lexicographic order,
each permutation compared as a string over the letters a, b, c, ...
"""
from __future__ import annotations

import itertools

LETTERS = "abcdefgh"


def perm_to_str(perm) -> str:
    return "".join(LETTERS[a] for a in perm)


def str_to_perm(s: str):
    return tuple(LETTERS.index(ch) for ch in s.strip())


def order_to_str(order) -> str:
    return "->".join(perm_to_str(p) for p in order)


def parse_order(s: str):
    """'abc->acb->bca' (or with unicode arrows) -> ((0,1,2),(0,2,1),(1,2,0))."""
    parts = s.replace("→", "->").split("->")
    return tuple(str_to_perm(p) for p in parts)


def all_orders(M: int):
    """Generate every valid order of an M-D FFT in canonical order."""
    ident = tuple(range(M))
    perms = list(itertools.permutations(range(M)))  # lexicographic

    def rec(prefix, used_last):
        if len(prefix) == M:
            yield tuple(prefix)
            return
        for p in perms:
            if p[-1] not in used_last:
                yield from rec(prefix + [p], used_last | {p[-1]})

    yield from rec([ident], {ident[-1]})


def count_by_enumeration(M: int) -> int:
    return sum(1 for _ in all_orders(M))


def count_by_steps(M: int) -> int:
    """Count orders without listing them: at each later stage, count (by
    checking all M! permutations) those whose last axis is still unused; the
    count depends only on how many axes are used, so the stages multiply."""
    perms = list(itertools.permutations(range(M)))
    total = 1
    used = {M - 1}                     # pi_1 = identity transforms the last axis
    for _t in range(2, M + 1):
        choices = [p for p in perms if p[-1] not in used]
        total *= len(choices)
        used = used | {choices[0][-1]}  # which axis does not change the next count
    return total


def is_valid_order(order, M: int) -> bool:
    if len(order) != M or tuple(order[0]) != tuple(range(M)):
        return False
    lasts = set()
    for p in order:
        if sorted(p) != list(range(M)):
            return False
        lasts.add(p[-1])
    return len(lasts) == M


def fft_axis_sequence(order):
    """Axis transformed at each step (the last axis of each decomposition)."""
    return [p[-1] for p in order]


def form_orders(M: int, m1: int):
    """The orders of the form m1+m2 (m2 = M - m1), the shape Section 3.3 gives
    the best orders: with X the first m1 axes and Y the other m2,
    decompositions 1..m2 start with X in natural order and arrange Y after it
    (so their FFTs run along Y's axes); decompositions m2+1..M start with one
    common arrangement of Y and arrange X after it (FFTs along X's axes).
    3-D a(bc) is 1+2 (abc->acb->cba), (ab)c is 2+1 (abc->cab->cba); 4-D
    (ab)(cd) is 2+2 (abcd->abdc->dcba->dcab).  Built directly; sorted."""
    X = tuple(range(m1))
    Y = tuple(range(m1, M))
    m2 = M - m1
    ys = list(itertools.permutations(Y))
    xs = list(itertools.permutations(X))
    out = []
    for rest in itertools.product(ys, repeat=m2 - 1):
        first = [Y] + list(rest)
        if len({p[-1] for p in first}) != m2:
            continue
        for lead in ys:
            for second in itertools.product(xs, repeat=m1):
                if len({p[-1] for p in second}) != m1:
                    continue
                out.append(tuple(X + p for p in first) + tuple(lead + q for q in second))
    return sorted(out)

"""Pins for the transpose-order oracle (Eq. (20), Table 1)."""
import os

import pytest

from oracle import orders

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _table1():
    out = {}
    with open(os.path.join(GOLDEN, "table1_order_counts.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                m, c = line.split()
                out[int(m)] = int(c)
    return out


def test_table1_by_enumeration():
    t1 = _table1()
    for M in (2, 3, 4):
        assert orders.count_by_enumeration(M) == t1[M]


def test_table1_by_stage_counting():
    t1 = _table1()
    for M in (2, 3, 4, 5, 6):
        assert orders.count_by_steps(M) == t1[M]


@pytest.mark.slow
def test_table1_five_d_by_enumeration():
    assert orders.count_by_enumeration(5) == _table1()[5]


def test_three_d_list():
    got = [orders.order_to_str(o) for o in orders.all_orders(3)]
    assert got == ["abc->acb->bca", "abc->acb->cba", "abc->bca->acb", "abc->bca->cab",
                   "abc->cab->bca", "abc->cab->cba", "abc->cba->acb", "abc->cba->cab"]
    # the two orders of Fig. 2 and the four listed in Section 3.1 are all valid
    for s in ["abc->cab->cba", "abc->cab->bca", "abc->acb->bca", "abc->acb->cba", "abc->cba->cab"]:
        assert orders.parse_order(s) in set(orders.all_orders(3))


def test_listed_orders_are_valid_and_canonical_is_sorted():
    with open(os.path.join(GOLDEN, "paper_best_orders.txt")) as f:
        listed = [l.split() for l in f if l.strip() and not l.startswith("#")]
    for m, s in listed:
        assert orders.is_valid_order(orders.parse_order(s), int(m))
    o4 = list(orders.all_orders(4))
    assert o4 == sorted(o4) and len(set(o4)) == len(o4)
    for o in o4:
        assert orders.is_valid_order(o, 4)


def test_invalid_orders():
    assert not orders.is_valid_order(((0, 1, 2), (0, 1, 2), (1, 2, 0)), 3)   # repeated FFT axis
    assert not orders.is_valid_order(((1, 0, 2), (0, 2, 1), (1, 2, 0)), 3)   # does not start natural
    assert not orders.is_valid_order(((0, 1, 2), (0, 2, 2), (1, 2, 0)), 3)   # not a permutation

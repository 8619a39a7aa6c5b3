"""Staged transposes (pack -> exchange -> unpack) under the matched ownership
reading: the ranges of each new decomposition are handed to the processes of
a maximum matching of the overlap counts, so the exchange copies exactly
T minus the matching's weight in every transpose.  Checked on the orders the
paper lists as always best (Sections 3.1 and 3.3), where the literal and the
matched readings give different amounts:

* exchanged (device-counted) points equal the oracle's matched amount;
* messages equal the off-diagonal non-zeros of the pair matrix after the
  oracle's relabelling;
* values are bit-identical to the fused permutation's and within 1e-5 of the
  FP64 oracle.
"""
import numpy as np
import pytest

from oracle import decomp, dft, orders
from paper_1302_6189_amd import fftrw, inputs
from tests.gpu_util import empty_dev, to_dev, to_host

pytestmark = pytest.mark.gpu

LISTED_3D = ["abc->acb->bca", "abc->acb->cba", "abc->cba->cab", "abc->cab->cba"]
LISTED_4D = ["abcd->abdc->dcba->dcab", "abcd->abdc->dcab->dcba", "abcd->abdc->cdab->cdba",
             "abcd->abdc->cdba->cdab"]
CASES = [((64, 64, 64), 128, o) for o in LISTED_3D] + [((8, 8, 8, 8), 128, o) for o in LISTED_4D] + \
        [((24, 20, 30), 50, "abc->cab->bca"), ((12, 10, 8, 6), 33, "abcd->dabc->bcda->cdab")]


def _oracle_messages(dims, P, a, b):
    """Off-diagonal non-zeros of C after relabelling by a maximum matching:
    pairs that share points and are not matched to each other."""
    from scipy.optimize import linear_sum_assignment
    C = decomp.pair_matrix(dims, P, a, b)
    rows, cols = linear_sum_assignment(C, maximize=True)
    return int(np.count_nonzero(C) - np.count_nonzero(C[rows, cols]))


@pytest.mark.parametrize("dims,P,order_s", CASES)
def test_staged_matched_exchange(gpu_lib, dims, P, order_s):
    M = len(dims)
    order = fftrw.order_from(order_s, M)
    flags = fftrw.FLAG_STAGED | fftrw.FLAG_OWN_MATCHED | fftrw.FLAG_COUNT_MOVED
    plan = fftrw.Plan(dims, P, order, flags=flags)
    x = inputs.uniform(dims, 31, np.complex64)
    xd = to_dev(x)
    yd = empty_dev(dims, np.complex64)
    plan.exec_fwd(xd, yd)
    y = to_host(yd)
    analytic, moved = plan.stats()
    steps, ret = decomp.order_volumes(dims, P, order, ownership="matched")
    lit_steps, lit_ret = decomp.order_volumes(dims, P, order)
    print(dims, P, order_s, "matched", steps, ret, "literal", lit_steps, lit_ret, flush=True)
    assert analytic == steps + [ret]
    assert moved == analytic  # the exchange copied exactly the matched amounts
    seq = list(order) + [tuple(range(M))]
    want_msgs = [_oracle_messages(dims, P, seq[t], seq[t + 1]) for t in range(M)]
    assert plan.messages() == want_msgs
    ref = dft.fftn_direct(x, orders.fft_axis_sequence(order))
    assert dft.rel_l2(y, ref) < 1e-5
    fused = fftrw.Plan(dims, P, order, flags=fftrw.FLAG_OWN_MATCHED | fftrw.FLAG_COUNT_MOVED)
    zd = empty_dev(dims, np.complex64)
    fused.exec_fwd(xd, zd)
    assert np.array_equal(to_host(zd), y)
    assert fused.stats()[1] == moved
    # the inverse through the same staged plan
    plan.exec_inv(yd, zd)
    assert dft.rel_l2(to_host(zd), x) < 1e-5
    assert plan.stats()[1] == analytic


def test_matched_differs_from_literal_somewhere(gpu_lib):
    # the cases above exercise the relabelling: on at least one transpose the
    # matched amount is below the literal one
    dims, P = (64, 64, 64), 128
    diffs = 0
    for o in LISTED_3D:
        order = fftrw.order_from(o, 3)
        m, mr = decomp.order_volumes(dims, P, order, ownership="matched")
        l, lr = decomp.order_volumes(dims, P, order)
        diffs += sum(a < b for a, b in zip(m + [mr], l + [lr]))
    assert diffs > 0

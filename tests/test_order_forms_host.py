"""The balanced-split study (paper_1302_6189_amd.order_forms) on the CPU: its
form generator against the oracle's, its dynamic program against the
library's search, and its always-best counts against the sets the oracle
pins to Section 3.3 (4 for 3-D, 4 for 4-D, 96 for 5-D under the matched
reading)."""
import pytest

from oracle import orders
from paper_1302_6189_amd import fftrw, order_forms


@pytest.mark.parametrize("M,m1", [(3, 1), (3, 2), (4, 1), (4, 2), (4, 3), (5, 2), (5, 3), (6, 3), (6, 2)])
def test_forms_match_oracle(M, m1):
    got = order_forms.form_orders(M, m1)
    assert got == orders.form_orders(M, m1)
    assert all(orders.is_valid_order(o, M) for o in got)


@pytest.mark.parametrize("dims,P,own", [((8, 8, 8, 8), 48, fftrw.OWN_LITERAL), ((3, 2, 2, 2, 2), 20, fftrw.OWN_MATCHED),
                                        ((2, 3, 2, 2, 3, 2), 20, fftrw.OWN_LITERAL)])
def test_dynamic_program_matches_library_search(dims, P, own):
    tab = fftrw.fft_transpose_volumes(dims, P, own)
    r = fftrw.fft_order_search(dims, P, ownership=own)
    assert order_forms.optimum_count(tab, len(dims)) == (r["best_volume"], r["n_best"])


def test_always_best_counts_and_forms():
    r3 = order_forms.study((8, 8, 8), [2 ** i for i in range(1, 7)], fftrw.OWN_MATCHED)
    assert r3["always_best"] == 4 and r3["always_best_by_form"] == {"1+2": 2, "2+1": 2}
    r4 = order_forms.study((8, 8, 8, 8), [2 ** i for i in range(1, 10)], fftrw.OWN_MATCHED)
    assert r4["always_best"] == 4 and r4["always_best_by_form"] == {"1+3": 0, "2+2": 4, "3+1": 0}
    r5 = order_forms.study((4,) * 5, [2 ** i for i in range(1, 9)], fftrw.OWN_MATCHED)
    assert r5["always_best"] == 96
    assert r5["always_best_by_form"] == {"1+4": 0, "2+3": 48, "3+2": 48, "4+1": 0}


def test_six_d_three_plus_three_at_sixty_four_processes():
    r = order_forms.study((4,) * 6, [64], fftrw.OWN_LITERAL, forms=[3])
    row = r["per_P"][0]
    assert row["n_best"] == row["forms"]["3+3"]["at_optimum"] == 2304

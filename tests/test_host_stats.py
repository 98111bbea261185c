"""Host statistics of the start-proposal evaluation (no GPU): the exact
sign test against scipy's binomial test, and the paired summary on
hand-made rows."""

import pytest
from scipy.stats import binomtest

from paper_2403_09225_amd.learned_start import paired_comparison, sign_test


@pytest.mark.parametrize("a,b", [(10, 3), (3, 10), (20, 8), (0, 7), (5, 5), (1, 0), (40, 22)])
def test_sign_test_matches_binomial_test(a, b):
    assert sign_test(a, b) == pytest.approx(binomtest(a, a + b, 0.5).pvalue, rel=1e-12)


def test_sign_test_without_discordant_pairs():
    assert sign_test(0, 0) == 1.0


def test_paired_comparison_counts():
    rows = []
    for sa, sb, ia, ib in [(True, True, 10, 12), (True, False, 10, 50), (True, False, 11, 40),
                           (False, True, 60, 9), (False, False, 70, 70)]:
        rows.append({"proposal_success": sa, "blind_success": sb,
                     "proposal_iterations": ia, "blind_iterations": ib})
    r = paired_comparison(rows, "proposal", "blind")
    assert (r["both"], r["only_proposal"], r["only_blind"], r["neither"]) == (1, 2, 1, 1)
    assert r["sign_test_p"] == pytest.approx(1.0)
    assert r["mean_iteration_difference"] == pytest.approx((-2 - 40 - 29 + 51 + 0) / 5)
    assert 0.0 < r["wilcoxon_p"] <= 1.0

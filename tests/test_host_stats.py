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


def test_wilson_interval_against_closed_form_cases():
    """Known values: k = 0 gives [0, z^2 / (n + z^2)]; symmetric about 1/2
    for k = n / 2; statsmodels-style reference for 12 of 40."""
    from paper_2403_09225_amd.learned_start import wilson_interval
    z = 1.959963984540054
    lo, hi = wilson_interval(0, 20)
    assert lo == 0.0 and hi == pytest.approx(z * z / (20 + z * z), rel=1e-12)
    lo, hi = wilson_interval(25, 50)
    assert lo + hi == pytest.approx(1.0, rel=1e-12)
    # 12 / 40: centre (p + z^2/2n) / (1 + z^2/n), half-width as defined by Wilson (1927)
    p, n = 0.3, 40
    c = (p + z * z / (2 * n)) / (1 + z * z / n)
    h = z / (1 + z * z / n) * (p * (1 - p) / n + z * z / (4 * n * n)) ** 0.5
    assert wilson_interval(12, 40) == pytest.approx([c - h, c + h], rel=1e-12)
    assert wilson_interval(12, 40) == pytest.approx([0.1806, 0.4543], abs=2e-4)


def test_mean_interval():
    from paper_2403_09225_amd.learned_start import mean_interval
    x = [1.0, 2.0, 3.0, 4.0]
    m, se = 2.5, (5.0 / 3.0) ** 0.5 / 2.0
    assert mean_interval(x) == pytest.approx([m - 1.959963984540054 * se, m + 1.959963984540054 * se])


def test_split_counts_covers_every_item_evenly():
    from paper_2403_09225_amd.learned_start import split_counts
    for n, parts in [(0, 3), (7, 1), (10, 3), (96, 8), (5, 8)]:
        c = split_counts(n, parts)
        assert len(c) == parts and sum(c) == n and max(c) - min(c) <= 1


def test_paired_costs_against_hand_computed_differences():
    from scipy.stats import wilcoxon
    from paper_2403_09225_amd.learned_start import paired_costs
    pi = [10.0, 80.0, 30.0, 200.0, 5.0, 60.0]
    ri = [50.0, 70.0, 90.0, 210.0, 45.0, 100.0]
    rows = [{"proposal_iterations": a, "random_iterations": b,
             "proposal_seconds": a / 100, "random_seconds": b / 100} for a, b in zip(pi, ri)]
    r = paired_costs(rows, "proposal", "random")
    d = [a - b for a, b in zip(pi, ri)]
    assert r["mean_iterations_difference"] == pytest.approx(sum(d) / 6)
    assert r["median_iterations_difference"] == pytest.approx(-40.0)   # -60, -40, -40, -40, -10, 10
    assert r["iterations_wilcoxon_p"] == pytest.approx(wilcoxon(d).pvalue)
    assert r["mean_seconds_difference"] == pytest.approx(sum(d) / 600)
    assert r["toys_proposal_cheaper"] == 5

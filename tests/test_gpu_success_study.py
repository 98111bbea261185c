"""The random multi-start success study on a small model: its bookkeeping,
and the property that makes its xtol comparison meaningful — from the same
start, a fit at a tighter xtol follows the looser fit's trajectory (the
driver is deterministic and only its stopping test differs) and so ends at
an NLL no higher, after at least as many iterations."""

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_success_study_small():
    from paper_2403_09225_amd.success_study import run
    summary, rows = run(K=4, n_events=4000, n_mc=200_000, n_starts=10, xtols=(1e-5, 1e-8),
                        time_cap_s=60.0, seed=3)
    say(f"[study] {summary}")
    a, b = rows["xtol_1e-05"], rows["xtol_1e-08"]
    fin = np.isfinite(a["nll"]) & np.isfinite(b["nll"])
    assert fin.sum() >= 8
    assert np.all(b["nll"][fin] <= a["nll"][fin] + 1e-9 * np.abs(a["nll"][fin]))
    assert np.all(b["iterations"][fin] >= a["iterations"][fin])
    nll_min = summary["nll_min"]
    for r in (a, b):
        assert np.all(r["nll"][np.isfinite(r["nll"])] >= nll_min)
    assert summary["nll_truth_fit"] >= nll_min
    for key in ("xtol_1e-05", "xtol_1e-08"):
        s = summary[key]
        assert 0.0 <= s["success_rate"] <= 1.0
        assert s["n_success"] == int(rows[key]["success"].sum())
        assert s["hit_time_cap"] == 0
    # every success at the looser xtol is one at the tighter xtol
    assert np.all(b["success"][a["success"]])

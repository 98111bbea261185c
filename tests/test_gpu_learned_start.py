"""What the trained start proposal gains over the method without it.

The K = 12 proposal shipped with the package (trained by
`python -m paper_2403_09225_amd.learned_start` on 4500 toy fits) is run on
fresh toys drawn from its prior (a seed it was not trained or validated on).
Per toy, Newton-CG is started from the truth, from the proposal, from the
blind start (the mean training label, which ignores the data) and from 8
random draws of the prior; the global minimum is the lowest NLL among them
and a fit succeeds within 0.01 of it.

Checked: the proposal succeeds more often than a random start, and the
proposal strategy (its fit, then random starts if it fails) reaches the
global minimum in fewer expected Newton iterations than random multi-start.
"""

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_proposal_beats_random_multistart():
    from paper_2403_09225_amd.learned_start import ToyStudy, load_proposal, resonance_layout
    net, prior, blind, meta = load_proposal()
    K = int(meta["K"])
    ch, sp = resonance_layout(K)
    say(f"[learned start] K = {K}, proposal trained on {int(meta['train_toys'])} toys")
    study = ToyStudy(ch, sp, 200_000, prior=prior, seed=2024)
    summary, rows = study.evaluate(net, n_toys=24, n_events=20_000, n_random=8, blind=blind,
                                   log_every=4)
    say(f"[learned start] {summary}")
    assert summary["proposal_success_rate"] > summary["random_start_success_rate"]
    assert summary["mean_iterations_proposal_strategy"] < summary["mean_iterations_random_strategy"]

"""Statistical pin of the oracle: a Newton-CG fit (the paper's optimiser,
scipy's method="Newton-CG" with gradient and Hessian-vector product, Sec. 3)
of data generated from known parameters recovers them within errors.

Data: 10k events by accept-reject from the two-resonance model of the
CPU-sized workload (J = 0 at 0.90/0.10 GeV and J = 1 at 0.892/0.05 GeV in
channel (12), c = (1, 0.6 e^{1.2 i})).

The normalisation sum uses a midpoint grid over the Dalitz region instead of
the workload's 50k random MC events: with a 50 MeV-wide resonance the random
MC's own noise moves the fitted parameters by O(1) of the data-statistics
errors, which the inverse-Hessian errors do not include.  With the grid the
pulls measure the data statistics alone.
"""

import numpy as np
import pytest

import oracle
import synth


@pytest.fixture(scope="module")
def k2_fit():
    W = synth.workload("k2_fit")
    mc = synth.midpoint_grid(500, 500)
    data = synth.accept_reject(
        W.n_data, lambda x, y: oracle.intensity((x, y), W, W.theta_true),
        synth.rng_for("k2_fit", synth.workloads.STREAM_DATA), scan=200_000, batch=1 << 16)
    return W, data, mc


def _gauge_fix(th):
    """Rotate and scale all couplings so that c_1 = 1 (the NLL is invariant)."""
    c = th[0::4] + 1j * th[1::4]
    c = c / c[0]
    out = th.copy()
    out[0::4], out[1::4] = c.real, c.imag
    return out


@pytest.mark.slow
def test_newton_cg_recovers_truth(k2_fit):
    W, data, mc = k2_fit
    rng = synth.rng_for("k2_fit", synth.workloads.STREAM_TEST)
    th0 = W.theta_true + rng.normal(scale=[0.1, 0.1, 0.01, 0.01] * 2)
    res = oracle.newton_cg_fit(data, mc, W, th0, xtol=1e-8)
    thf = _gauge_fix(res.x)
    _, g = oracle.grad(data, mc, W, thf)
    S = oracle.grad_scale(data, mc, W, thf)
    assert np.all(np.abs(g) <= 1e-6 * S)           # at a stationary point
    H = oracle.hessian(data, mc, W, thf)
    free = [2, 3, 4, 5, 6, 7]                      # c_1 fixed at 1
    cov = np.linalg.inv(H[np.ix_(free, free)])
    sig = np.sqrt(np.diag(cov))
    pull = (thf[free] - W.theta_true[free]) / sig
    assert np.all(np.abs(pull) < 3.0), pull
    # positive definite in the gauge-fixed subspace: a minimum, not a saddle
    assert np.all(np.linalg.eigvalsh(H[np.ix_(free, free)]) > 0)

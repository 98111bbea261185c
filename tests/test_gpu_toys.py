"""Per-event intensity and the GPU toy generator against the oracle.

* pwa_intensity: omega(x) of eq. (1) per event, FP64 event stream to 1e-12
  relative of the oracle's (the same FP64 formula, one reciprocal).  FP32
  stream: the rounding of s, u, g to 2^-24 is amplified near a pole by
  s / |M^2 - s - i M Gamma| and then by any cancellation between
  resonances, so the bound is on the scale without cancellation:
  |d omega| <= 1e-5 (sum_k |c_k a_k|)^2.
* Toys: events drawn by accept-reject on the GPU follow the oracle's
  intensity: a binned chi-square of the drawn sample against the expected
  bin contents (the oracle's intensity integrated over each bin by a large
  uniform sample) is compatible with its degrees of freedom.
"""

import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_cases import Model, case, likelihood, rng

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.parametrize("K", [2, 12])
def test_intensity_matches_oracle(K):
    say(f"[intensity] K={K}")
    model, th, data, mc, _ = case(K, 3001, 5003, 300 + K)
    lik = likelihood(model, data, mc, streams=("f64", "f32"))
    for which, ev in (("data", data), ("mc", mc)):
        ref = oracle.intensity(ev, model, th)
        got = lik.intensity(th, which).cpu().numpy()
        assert got.shape == ref.shape
        assert np.max(np.abs(got - ref) / ref) <= 1e-12
    lik.set_precision("f32")
    got = lik.intensity(th, "mc").cpu().numpy()
    ref = oracle.intensity(mc, model, th)
    a = oracle.amplitudes(mc, model, th)
    scale = sum(np.abs((th[4 * k] + 1j * th[4 * k + 1]) * a[k]) for k in range(K)) ** 2
    assert np.all(np.abs(got - ref) <= 1e-5 * scale)
    assert np.median(np.abs(got - ref) / ref) <= 1e-6


def test_toys_follow_the_intensity():
    from paper_2403_09225_amd.toys import ToyGenerator
    W = synth.workload("k2_fit")
    model = Model(W.channel, W.spin)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2403)
    n = 200_000
    say("[toys] drawing 200k events (k2_fit model)")
    tg = ToyGenerator(W.channel, W.spin, batch=1 << 20, scan=1 << 18)
    s12, s13 = tg.draw(W.theta_true, n, gen)
    s12, s13 = s12.cpu().numpy(), s13.cpu().numpy()
    assert s12.shape == (n,) and np.all(synth.events.inside(s12, s13))
    # expected bin contents from the oracle's intensity on uniform events
    mc = synth.uniform_phase_space(2_000_000, rng(77))
    w = oracle.intensity(mc, model, W.theta_true)
    (a0, a1), (b0, b1) = synth.bounding_box()
    edges = (np.linspace(a0, a1, 21), np.linspace(b0, b1, 21))
    obs, _, _ = np.histogram2d(s12, s13, bins=edges)
    exp_w, _, _ = np.histogram2d(mc[0], mc[1], bins=edges, weights=w)
    exp_w2, _, _ = np.histogram2d(mc[0], mc[1], bins=edges, weights=w * w)
    scale = n / w.sum()
    exp = exp_w * scale
    var = exp + exp_w2 * scale * scale     # Poisson plus the integration sample's own error
    m = exp >= 20
    chi2 = float(np.sum((obs[m] - exp[m]) ** 2 / var[m]))
    ndf = int(m.sum()) - 1
    say(f"[toys] chi2/ndf = {chi2:.1f}/{ndf}")
    assert ndf > 100
    assert chi2 < ndf + 5.0 * np.sqrt(2.0 * ndf)
    assert obs[~m].sum() <= 2 * exp[~m].sum() + 50

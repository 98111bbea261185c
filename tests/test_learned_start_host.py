"""Host logic of the start proposal (no GPU): the prior, the canonical
coding of parameter vectors and the shipped network file."""

import os

import numpy as np
import pytest

from paper_2403_09225_amd import learned_start as LS


def _rng(s):
    return np.random.Generator(np.random.PCG64(s))


def test_prior_ranges_and_thresholds():
    ch, _ = LS.resonance_layout(12)
    wide = LS.Prior.wide(ch)
    for s in range(50):
        th = wide.draw(_rng(s)).reshape(12, 4)
        assert np.all(th[:, 2] >= 0.6 - 1e-12) and np.all(th[:, 2] <= 1.6 + 1e-12)
        assert np.all(th[:, 2] >= wide.thr + 0.02)
        assert np.all(th[:, 3] >= 0.03 - 1e-12) and np.all(th[:, 3] <= 0.3 + 1e-12)
        mag = np.hypot(th[:, 0], th[:, 1])
        assert np.all(mag >= 0.2 - 1e-12) and np.all(mag <= 1.0 + 1e-12)


def test_coding_is_invariant_under_the_likelihood_symmetries():
    ch, sp = LS.resonance_layout(12)
    nom = LS.Prior.wide(ch).draw(_rng(7))
    prior = LS.Prior(ch, nom[2::4], nom[3::4], 0.03, 0.2)
    coder = LS.StartCoder(ch, sp, prior)
    th = prior.draw(_rng(3))
    y = coder.encode(th)
    # global phase and scale of the couplings
    t2 = th.reshape(12, 4).copy()
    c = (t2[:, 0] + 1j * t2[:, 1]) * 2.5 * np.exp(1j * 0.7)
    t2[:, 0], t2[:, 1] = c.real, c.imag
    assert np.allclose(coder.encode(t2.reshape(-1)), y, rtol=0, atol=1e-12)
    # interchangeable resonances (same channel and spin): 0 and 9
    t3 = th.reshape(12, 4).copy()
    t3[[0, 9]] = t3[[9, 0]]
    y3 = coder.encode(t3.reshape(-1))
    # c_0 sets the phase convention, so compare the physical content instead
    assert np.allclose(np.sort(coder.canonical(t3.reshape(-1)).reshape(12, 4)[[0, 9], 2]),
                       np.sort(th.reshape(12, 4)[[0, 9], 2]))
    assert np.all(np.isfinite(y3))
    # decode inverts encode on canonical vectors inside the prior
    assert np.allclose(coder.decode(y), coder.canonical(th), rtol=0, atol=1e-12)


def test_shipped_network_file():
    path = os.path.join(LS.DATA, "start_proposal_k12.npz")
    d = np.load(path, allow_pickle=False)
    dims = tuple(int(x) for x in d["dims"])
    assert dims == (1024, 512, 512, 48)
    n_in, h1, h2, n_out = dims
    assert d["w"].shape == (h1 * n_in + h1 + h2 * h1 + h2 + n_out * h2 + n_out,)
    assert d["w"].dtype == np.float32 and np.all(np.isfinite(d["w"]))
    assert int(d["K"]) == 12 and d["blind"].shape == (48,)
    for k in ("m_nom", "g_nom", "m_spread", "g_spread"):
        assert d[k].shape == (12,)

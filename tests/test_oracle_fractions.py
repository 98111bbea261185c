"""Pins of the oracle's fit fractions (Table 1 column F_i, read as
F_k = sum_MC |c_k a_k|^2 / sum_MC |sum_l c_l a_l|^2) and of their
gradients, against facts that do not come from the oracle's own code:
the algebraic identity |sum y|^2 = sum |y|^2 + sum_{k<l} 2 Re(conj(y_k) y_l),
Legendre orthogonality on a mirror-symmetric MC sample, a closed form for
two resonances with identical lineshapes, the likelihood's coupling
symmetries, and central finite differences."""

import numpy as np
import pytest

import oracle
import synth


def _events(n, seed):
    return synth.uniform_phase_space(n, np.random.Generator(np.random.PCG64(seed)))


def _case(make_model, K=6, nm=1500, seed=5):
    ch, sp = synth.resonance_layout(K)
    model = make_model(ch, sp)
    th = synth.draw_theta(ch, sp, np.random.Generator(np.random.PCG64(seed)))
    return model, th, _events(nm, seed + 2)


def test_fractions_and_interference_add_up_to_one(make_model):
    """sum_k F_k + sum_{k<l} I_kl = 1 (expansion of |sum_k y_k|^2).  A dropped
    or doubled interference term, or a wrong denominator, breaks it."""
    model, th, mc = _case(make_model)
    Phi = oracle.fraction_matrix(mc, model, th)
    assert np.all(np.tril(Phi, -1) == 0.0)
    assert np.sum(np.triu(Phi)) == pytest.approx(1.0, abs=1e-13)
    assert np.all(np.diag(Phi) > 0.0)
    F, _ = oracle.fit_fractions(mc, model, th)
    np.testing.assert_allclose(F, np.diag(Phi), rtol=1e-13, atol=0)


def test_s_p_interference_vanishes_on_mirror_mc(make_model):
    """S and P waves in the same channel: on an MC sample paired under
    cos(theta) -> -cos(theta) the S-P interference cancels event pair by event
    pair, so F_S + F_P = 1 to rounding."""
    model = make_model([0, 0], [0, 1])
    th = np.array([1.0, 0.0, 0.9, 0.1, 0.6, 0.3, 0.892, 0.05])
    ev = synth.mirror_symmetric(*_events(20000, 21))
    Phi = oracle.fraction_matrix(ev, model, th)
    assert abs(Phi[0, 1]) <= 1e-12
    F, _ = oracle.fit_fractions(ev, model, th)
    assert F.sum() == pytest.approx(1.0, abs=1e-12)


def test_identical_lineshapes_closed_form(make_model):
    """Two resonances with the same channel, spin, mass and width have the
    same a(x), so F_k = |c_k|^2 / |c_1 + c_2|^2 exactly, and
    I_12 = 2 Re(conj(c_1) c_2) / |c_1 + c_2|^2."""
    model = make_model([1, 1], [2, 2])
    c1, c2 = 0.8 - 0.3j, -0.2 + 0.5j
    th = np.array([c1.real, c1.imag, 1.25, 0.12, c2.real, c2.imag, 1.25, 0.12])
    mc = _events(3000, 31)
    Phi = oracle.fraction_matrix(mc, model, th)
    den = abs(c1 + c2) ** 2
    assert Phi[0, 0] == pytest.approx(abs(c1) ** 2 / den, rel=1e-13)
    assert Phi[1, 1] == pytest.approx(abs(c2) ** 2 / den, rel=1e-13)
    assert Phi[0, 1] == pytest.approx(2 * (np.conj(c1) * c2).real / den, rel=1e-12)
    F, dF = oracle.fit_fractions(mc, model, th)
    # d/dRe c1 of |c1|^2 / |c1 + c2|^2, by hand
    s = c1 + c2
    d = 2 * c1.real / den - abs(c1) ** 2 * 2 * s.real / den ** 2
    assert dF[0, 0] == pytest.approx(d, rel=1e-12)
    # moving both masses (or both widths) together keeps the lineshapes
    # equal, so F does not change along those directions
    scale = np.max(np.abs(dF))
    assert np.max(np.abs(dF[:, 2] + dF[:, 6])) <= 1e-12 * scale
    assert np.max(np.abs(dF[:, 3] + dF[:, 7])) <= 1e-12 * scale


def test_single_resonance(make_model):
    """K = 1: F = 1 and every derivative vanishes."""
    model = make_model([2], [1])
    th = np.array([0.7, -0.4, 1.2, 0.15])
    F, dF = oracle.fit_fractions(_events(900, 9), model, th)
    assert F[0] == pytest.approx(1.0, abs=1e-15)
    assert np.max(np.abs(dF)) <= 1e-13


def test_coupling_symmetries(make_model):
    """F is unchanged by one complex factor on all couplings; hence its
    gradient is orthogonal to the generators J theta (phase) and Pi theta
    (scale) of that symmetry."""
    model, th, mc = _case(make_model, K=4, nm=1200, seed=8)
    F, dF = oracle.fit_fractions(mc, model, th)
    th2 = th.copy()
    c = (th[0::4] + 1j * th[1::4]) * (1.7 * np.exp(0.9j))
    th2[0::4], th2[1::4] = c.real, c.imag
    F2, _ = oracle.fit_fractions(mc, model, th2)
    np.testing.assert_allclose(F2, F, rtol=1e-12, atol=0)
    Jt = np.zeros_like(th)
    Jt[0::4], Jt[1::4] = -th[1::4], th[0::4]
    Pt = np.zeros_like(th)
    Pt[0::4], Pt[1::4] = th[0::4], th[1::4]
    scale = np.abs(dF) @ np.abs(th)
    assert np.all(np.abs(dF @ Jt) <= 1e-12 * scale)
    assert np.all(np.abs(dF @ Pt) <= 1e-12 * scale)


def test_gradient_matches_central_differences(make_model):
    """dF_k/dtheta_p against (F(theta + h e_p) - F(theta - h e_p)) / 2h."""
    model, th, mc = _case(make_model, K=4, nm=1200, seed=12)
    _, dF = oracle.fit_fractions(mc, model, th)
    h = 1e-6
    for p in range(th.size):
        e = np.zeros_like(th)
        e[p] = h
        fd = (oracle.fit_fractions(mc, model, th + e)[0]
              - oracle.fit_fractions(mc, model, th - e)[0]) / (2 * h)
        assert np.max(np.abs(fd - dF[:, p])) <= 1e-7 * max(1.0, np.max(np.abs(dF))), p

"""Pins of the oracle's spin-1 parent (the helicity sum of eq. (1), mu = +1,
-1) against facts independent of its code:

* a tiny case against the 50-digit implementation in tests/indep_mp.py,
  which builds the daughters' four-vectors along another route (boosted
  from the pair frame, turned to the reference plane) and sums the two
  helicity amplitudes itself;
* orientation averages with exact quadrature: sum_mu |e_mu . v|^2 averaged
  over rotations is (2/3) |v|^2, for v = p^_c, p^_c x q^ and the rank-2
  contraction (pins the polarisation vectors, the rotation and the tensors);
* a rotation about the polarisation axis leaves the helicity-summed
  intensity unchanged;
* dual-number gradient and H v against central differences.
"""

import mpmath as mp
import numpy as np
import pytest

import oracle
import synth
from tests import indep_mp


def _spin1_model(make_model, channel, spin, lineshape=None):
    m = make_model(channel, spin, lineshape=lineshape)
    m.parent_spin = 1
    return m


def _events4(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    s12, s13 = synth.uniform_phase_space(n, rng)
    cb, g = synth.uniform_orientation(n, rng)
    return s12, s13, cb, g


def test_spin1_tiny_case_against_independent_50_digit(make_model):
    mp.mp.dps = 50
    model = _spin1_model(make_model, [0, 1, 2, 0], [0, 1, 2, 2])
    th = np.array([1.0, 0.0, 0.95, 0.12, 0.4, -0.7, 1.05, 0.09,
                   -0.3, 0.5, 1.25, 0.2, 0.8, 0.2, 1.45, 0.15])
    ev = _events4(12, 31)
    got = oracle.intensity(ev, model, th)
    for i in range(len(ev[0])):
        ref = indep_mp.spin1_omega(ev[0][i], ev[1][i], ev[2][i], ev[3][i], model.channel,
                                   model.spin, th, synth.PARENT_MASS, synth.DAUGHTER_MASSES,
                                   synth.R_BARRIER)
        assert abs(float(ref) - got[i]) <= 1e-11 * float(ref), (i, float(ref), got[i])


@pytest.mark.parametrize("J", [0, 1, 2])
def test_orientation_average_of_helicity_sum(make_model, J):
    """With one resonance of spin J the helicity-summed angular factor,
    averaged over rotations, is (2/3) |v|^2 (v = p^_c, p^_c x q^,
    q^ (q^.p^_c) - p^_c/3): Gauss-Legendre in cos beta and a uniform grid in
    gamma integrate these degree-2 polynomials exactly."""
    model = _spin1_model(make_model, [0], [J])
    s12, s13 = synth.uniform_phase_space(5, np.random.Generator(np.random.PCG64(4)))
    xb, wb = np.polynomial.legendre.leggauss(6)
    ng = 8
    gg = 2 * np.pi * np.arange(ng) / ng
    for i in range(5):
        cb = np.repeat(xb, ng)
        g = np.tile(gg, len(xb))
        w = np.repeat(wb, ng) / (2 * ng)
        n = cb.size
        p4 = oracle.daughter_momenta(np.full(n, s12[i]), np.full(n, s13[i]), cb, g, model)
        Y = oracle.angular_factors(p4, 0, J)
        avg = np.sum(w * (np.abs(Y[0]) ** 2 + np.abs(Y[1]) ** 2))
        # |v|^2 is rotation invariant: take it from the first orientation
        pc = p4[0, 2, 1:] / np.linalg.norm(p4[0, 2, 1:])
        L = oracle.pwa_oracle._boost_matrix((p4[:, 0] + p4[:, 1])[:1])[0]
        qa = (L @ p4[0, 0])[1:]
        qa = qa / np.linalg.norm(qa)
        v = [pc, np.cross(pc, qa), qa * (qa @ pc) - pc / 3][J]
        assert avg == pytest.approx(2.0 / 3.0 * (v @ v), rel=1e-12, abs=1e-15)


def test_rotation_about_polarisation_axis(make_model):
    """Rotating every daughter about z by alpha multiplies z^mu by the phase
    exp(-i mu alpha) (or its inverse), so sum_mu |z^mu|^2 is unchanged."""
    model = _spin1_model(make_model, [0, 1, 2], [1, 0, 2])
    th = np.array([1.0, 0.0, 0.95, 0.1, 0.5, 0.5, 1.1, 0.2, -0.4, 0.3, 1.3, 0.15])
    ev = _events4(50, 8)
    p4 = oracle.daughter_momenta(*ev, model)
    w0 = oracle.intensity(ev, model, th)
    alpha = 0.731
    Rz = np.array([[np.cos(alpha), -np.sin(alpha), 0], [np.sin(alpha), np.cos(alpha), 0], [0, 0, 1]])
    p4r = p4.copy()
    p4r[:, :, 1:] = p4[:, :, 1:] @ Rz.T
    # recompute the helicity sum from the rotated momenta
    kin = {ch: oracle.kinematics(ev[0], ev[1], ch, model) for ch in (0, 1, 2)}
    z = [0, 0]
    for k, (ch, J) in enumerate(zip(model.channel, model.spin)):
        Y = oracle.angular_factors(p4r, ch, J)
        for mu in range(2):
            a = oracle.amplitude(kin[ch], ch, J, th[4 * k + 2], th[4 * k + 3], model, 0, Y[mu])
            z[mu] = z[mu] + (th[4 * k] + 1j * th[4 * k + 1]) * a
    w1 = np.abs(z[0]) ** 2 + np.abs(z[1]) ** 2
    np.testing.assert_allclose(w1, w0, rtol=1e-12)
    # and a single helicity term alone does change (the test has teeth)
    assert np.max(np.abs(np.abs(z[0]) ** 2 - np.abs(z[1]) ** 2)) > 1e-6


def test_spin1_gradient_and_hessian_match_differences(make_model):
    """Through the helicity sum, with a Flatte scalar among the resonances."""
    model = _spin1_model(make_model, [2, 0, 1], [0, 1, 2], lineshape=[1, 0, 0])
    th = np.array([1.0, 0.0, synth.FLATTE_F0[0], synth.FLATTE_F0[1],
                   0.7, 0.4, 0.892, 0.05, 0.3, -0.5, 1.43, 0.11])
    data = _events4(300, 12)
    mc = _events4(1500, 13)
    _, g = oracle.grad(data, mc, model, th)
    S = oracle.grad_scale(data, mc, model, th)
    h = 1e-6
    for p in range(th.size):
        e = np.zeros_like(th)
        e[p] = h
        fd = (oracle.nll(data, mc, model, th + e) - oracle.nll(data, mc, model, th - e)) / (2 * h)
        assert abs(fd - g[p]) <= 1e-6 * S[p] + 1e-7 * abs(g[p]), p
    v = np.random.Generator(np.random.PCG64(19)).normal(size=th.size)
    _, _, hv = oracle.hvp(data, mc, model, th, v)
    hs = 1e-5
    fd = (oracle.grad(data, mc, model, th + hs * v)[1] - oracle.grad(data, mc, model, th - hs * v)[1]) / (2 * hs)
    SH = oracle.hvp_scale(data, mc, model, th, v)
    np.testing.assert_array_less(np.abs(fd - hv), 1e-5 * SH + 1e-6 * np.abs(hv))

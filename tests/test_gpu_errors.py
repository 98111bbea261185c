"""GPU parity of what is read off at a minimum: the full Hessian
(pwa_hessian), the fit fractions and their gradients (pwa_fit_fractions),
and the error matrix built from them, against the FP64 oracle on the same
seeded inputs; at the full GPU-scale size through identities that hold at
any size."""

import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_cases import assert_close, case, likelihood, rng

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _np(t):
    return t.detach().cpu().numpy()


def _unit(P, j):
    e = np.zeros(P)
    e[j] = 1.0
    return e


@pytest.mark.parametrize("K,nd,nm,seed", [(1, 401, 2003, 40), (2, 2011, 9013, 41),
                                          (6, 1999, 7001, 42), (12, 1001, 4001, 43)])
def test_hessian_parity(K, nd, nm, seed):
    """Every entry of the symmetrised GPU Hessian against the oracle's exact
    Hessian, to 1e-10 of the larger absolute-sum scale of its two mirror
    entries (each comes from its own pass)."""
    say(f"[hessian] K={K} nd={nd} nm={nm}")
    model, th, data, mc, _ = case(K, nd, nm, seed)
    lik = likelihood(model, data, mc)
    H = _np(lik.hessian(th))
    P = 4 * K
    assert np.array_equal(H, H.T)
    Ho = np.empty((P, P))
    Sc = np.empty((P, P))
    for j in range(P):
        e = _unit(P, j)
        _, _, col = oracle.hvp(data, mc, model, th, e)
        SH = oracle.hvp_scale(data, mc, model, th, e)
        Ho[:, j] = col
        Sc[:, j] = SH
    Ho = 0.5 * (Ho + Ho.T)
    bound = np.maximum(Sc, Sc.T)
    for j in range(P):
        assert_close(f"H[:, {j}]", H[:, j], Ho[:, j], bound[:, j], 1e-10)


@pytest.mark.parametrize("K,nm,seed", [(1, 3001, 51), (2, 9013, 52), (6, 7001, 53),
                                       (12, 12007, 54), (30, 4001, 55)])
def test_fit_fraction_parity(K, nm, seed):
    """F_k and dF_k/dtheta against the oracle's direct per-event sums (the
    GPU switches the other couplings off and differentiates the MC sum)."""
    say(f"[fit fractions] K={K} nm={nm}")
    model, th, data, mc, _ = case(K, 301, nm, seed)
    lik = likelihood(model, data, mc)
    F, dF = lik.fit_fractions(th)
    F, dF = _np(F), _np(dF)
    Fo, dFo = oracle.fit_fractions(mc, model, th)
    np.testing.assert_allclose(F, Fo, rtol=1e-11, atol=1e-15)
    # (F is dimensionless and theta is O(1): an absolute floor of 1e-10 covers
    # components that vanish, e.g. all of them at K = 1)
    np.testing.assert_allclose(dF, dFo, rtol=1e-9, atol=1e-10 * (1.0 + np.max(np.abs(dFo))))
    assert np.array_equal(_np(lik.fit_fractions(th, with_grad=False)), F)


def test_fit_fractions_ignore_data_and_keep_status_clean():
    """The fractions are MC integrals: binding different data changes them
    only through the summation order (the grid depends on the event count),
    and no status bit is raised by the masked passes."""
    model, th, data, mc, _ = case(6, 1501, 6007, 56)
    a = likelihood(model, data, mc)
    b = likelihood(model, (data[0][:7], data[1][:7]), mc)
    Fa, dFa = a.fit_fractions(th)
    Fb, dFb = b.fit_fractions(th)
    torch.testing.assert_close(Fb, Fa, rtol=1e-13, atol=0)
    torch.testing.assert_close(dFb, dFa, rtol=1e-11, atol=1e-13 * float(dFa.abs().max()))
    assert a.device_status() == 0


def test_error_matrix_after_fit():
    """Fit a two-resonance model (one coupling fixed) to events drawn from
    it, then: the covariance is the inverse of the oracle's Hessian at the
    fitted point (free block), the propagated fit-fraction errors match the
    oracle's gradients, and the fit lies within a few standard deviations of
    the generating point."""
    from paper_2403_09225_amd.toys import ToyGenerator
    model, th, _, mc, _ = case(2, 0, 40000, 57)
    th = th.copy()
    th[0], th[1] = abs(complex(th[0], th[1])), 0.0   # c_0 real positive, fixed
    gen = torch.Generator(device="cuda")
    gen.manual_seed(58)
    d12, d13 = ToyGenerator(model.channel, model.spin).draw(th, 8000, gen)
    data = (d12.cpu().numpy(), d13.cpu().numpy())
    lik = likelihood(model, data, mc)
    free = np.ones(8, bool)
    free[[0, 1]] = False
    start = th + rng(59).normal(scale=0.005, size=8) * free
    fit, rep = lik.fit(start, xtol=1e-8, forcing="relative", free_mask=free)
    assert rep["converged"] == 1, rep
    thf = _np(fit)
    say(f"[errors] fit nll {rep['nll']:.6f} in {rep['iterations']} iterations")
    res = lik.errors(thf, free_mask=free)
    Ho = oracle.hessian(data, mc, model, thf)
    Ho = 0.5 * (Ho + Ho.T)
    Co = np.zeros((8, 8))
    Co[np.ix_(free, free)] = np.linalg.inv(Ho[np.ix_(free, free)])
    np.testing.assert_allclose(res["covariance"], Co, rtol=1e-7, atol=1e-9 * np.max(np.abs(Co)))
    assert np.all(res["sigma"][free] > 0) and np.all(res["sigma"][~free] == 0)
    Fo, dFo = oracle.fit_fractions(mc, model, thf)
    sig_o = np.sqrt(np.einsum("ri,ij,rj->r", dFo, Co, dFo))
    np.testing.assert_allclose(res["fit_fractions"], Fo, rtol=1e-11)
    np.testing.assert_allclose(res["fit_fraction_sigma"], sig_o, rtol=1e-6)
    # the fit lands within a few standard deviations of the generating point
    pull = (thf - th)[free] / res["sigma"][free]
    say(f"[errors] pulls {np.round(pull, 2)}")
    assert np.all(np.abs(pull) < 6.0)


@pytest.fixture(scope="module")
def k12_hvp():
    W = synth.workload("k12_hvp")
    say("[errors fullsize] generating 1M + 5M events")
    mc = synth.uniform_phase_space(W.n_mc, synth.rng_for("k12_hvp", synth.workloads.STREAM_MC))
    data = synth.resonant_like(W.n_data, W.channel, W.theta_true,
                               synth.rng_for("k12_hvp", synth.workloads.STREAM_DATA))
    lik = likelihood(W, data, mc, streams=("f64", "f32"))
    return W, data, mc, lik


def test_fullsize_hessian_identities(k12_hvp):
    """At 1M + 5M events: H (J theta) = J g and H (Pi theta) = -Pi g (the
    coupling phase and scale symmetries), and every column equals pwa_hvp
    along that unit vector to rounding (the symmetrisation averages it with
    row j)."""
    W, data, mc, lik = k12_hvp
    th = W.theta_true + synth.rng_for("k12_hvp", 4).normal(scale=0.01, size=48)
    H = _np(lik.hessian(th))
    _, g = lik.grad(th)
    g = _np(g)
    Jt = np.zeros(48)
    Jt[0::4], Jt[1::4] = -th[1::4], th[0::4]
    Pt = np.zeros(48)
    Pt[0::4], Pt[1::4] = th[0::4], th[1::4]
    Jg = np.zeros(48)
    Jg[0::4], Jg[1::4] = -g[1::4], g[0::4]
    Pg = np.zeros(48)
    Pg[0::4], Pg[1::4] = g[0::4], g[1::4]
    scale = np.abs(H) @ np.abs(th) + np.abs(g)
    assert np.all(np.abs(H @ Jt - Jg) <= 1e-9 * scale)
    assert np.all(np.abs(H @ Pt + Pg) <= 1e-9 * scale)
    for j in (0, 7, 30, 47):
        hv, _, _ = lik.hvp(th, _unit(48, j))
        hv = _np(hv)
        # symmetrisation averages with row j: within rounding of the column
        assert np.max(np.abs(H[:, j] - hv)) <= 1e-10 * np.max(np.abs(hv))


def test_fullsize_fit_fractions(k12_hvp):
    """At 5M MC events: F_k against the oracle's direct sums over all of
    them; dF through its symmetry identities and a central difference of the
    GPU fractions."""
    W, data, mc, lik = k12_hvp
    th = W.theta_true
    F, dF = lik.fit_fractions(th)
    F, dF = _np(F), _np(dF)
    say("[errors fullsize] oracle fractions over 5M MC events")
    Phi = oracle.fraction_matrix(mc, W, th)
    np.testing.assert_allclose(F, np.diag(Phi), rtol=1e-11)
    Jt = np.zeros(48)
    Jt[0::4], Jt[1::4] = -th[1::4], th[0::4]
    Pt = np.zeros(48)
    Pt[0::4], Pt[1::4] = th[0::4], th[1::4]
    scale = np.abs(dF) @ np.abs(th)
    assert np.all(np.abs(dF @ Jt) <= 1e-10 * scale)
    assert np.all(np.abs(dF @ Pt) <= 1e-10 * scale)
    d = synth.rng_for("k12_hvp", 5).normal(size=48)
    h = 1e-6
    Fp = _np(lik.fit_fractions(th + h * d, with_grad=False))
    Fm = _np(lik.fit_fractions(th - h * d, with_grad=False))
    np.testing.assert_allclose((Fp - Fm) / (2 * h), dF @ d, rtol=1e-5,
                               atol=1e-7 * np.max(np.abs(dF @ d)))


def test_fp32_stream_hessian_and_fractions():
    """The same entry points on the FP32 event stream: Hessian entries to
    1e-4 of their scale, fractions to 1e-5 relative.  (Random directions
    meet 3e-5; a unit direction along a mass or width isolates the second
    derivatives, which carry w^3 terms and so three times the FP32 relative
    rounding of w = 1/D near a pole, with no averaging over components.)"""
    model, th, data, mc, _ = case(6, 1999, 7001, 80)
    lik = likelihood(model, data, mc, streams=("f64", "f32"))
    lik.set_precision("f32")
    H = _np(lik.hessian(th))
    F, dF = lik.fit_fractions(th)
    P = 24
    Ho = np.empty((P, P))
    Sc = np.empty((P, P))
    for j in range(P):
        e = _unit(P, j)
        _, _, col = oracle.hvp(data, mc, model, th, e)
        SH = oracle.hvp_scale(data, mc, model, th, e)
        Ho[:, j] = col
        Sc[:, j] = SH
    # symmetrised entries mix two passes: bound by the larger of their scales
    Ho = 0.5 * (Ho + Ho.T)
    bound = np.maximum(Sc, Sc.T)
    for j in range(P):
        assert_close(f"H32[:, {j}]", H[:, j], Ho[:, j], bound[:, j], 1e-4)
    Fo, dFo = oracle.fit_fractions(mc, model, th)
    np.testing.assert_allclose(_np(F), Fo, rtol=1e-5)
    np.testing.assert_allclose(_np(dF), dFo, rtol=1e-4, atol=1e-5 * (1.0 + np.max(np.abs(dFo))))


@pytest.mark.parametrize("K,nm,seed", [(1, 3001, 81), (2, 9013, 82), (6, 7001, 83), (12, 12007, 84),
                                       (24, 5003, 85)])
def test_fraction_matrix_parity(K, nm, seed):
    """Fit fractions and interference terms from the FP64 matrix-core Gram
    matrix against the oracle's direct sums; they add up to 1, and the
    diagonal equals pwa_fit_fractions (masked gradient passes)."""
    say(f"[fraction matrix] K={K} nm={nm}")
    model, th, data, mc, _ = case(K, 301, nm, seed)
    lik = likelihood(model, data, mc)
    Phi = _np(lik.fraction_matrix(th))
    Po = oracle.fraction_matrix(mc, model, th)
    np.testing.assert_allclose(Phi, Po, rtol=1e-10, atol=1e-12)
    assert abs(Phi.sum() - 1.0) <= 1e-12
    assert np.all(np.tril(Phi, -1) == 0.0)
    F = _np(lik.fit_fractions(th, with_grad=False))
    np.testing.assert_allclose(np.diag(Phi), F, rtol=1e-11)


def test_edge_cases_at_the_minimum():
    """No data events (MC only), a resonance whose coupling is zero (its
    fraction, its interference terms and the gradient of its fraction along
    the other parameters vanish), and an FP32-only context."""
    model, th, data, mc, _ = case(5, 0, 4001, 90)
    th = th.copy()
    th[8:10] = 0.0                                  # c_2 = 0
    lik = likelihood(model, (np.zeros(0), np.zeros(0)), mc)
    F, dF = lik.fit_fractions(th)
    F, dF = _np(F), _np(dF)
    Fo, dFo = oracle.fit_fractions(mc, model, th)
    np.testing.assert_allclose(F, Fo, rtol=1e-11, atol=1e-15)
    assert F[2] == 0.0 and np.all(dF[2] == 0.0)
    Phi = _np(lik.fraction_matrix(th))
    np.testing.assert_allclose(Phi, oracle.fraction_matrix(mc, model, th), rtol=1e-10, atol=1e-12)
    assert np.all(Phi[2, :] == 0.0) and np.all(Phi[:, 2] == 0.0)
    H = _np(lik.hessian(th))
    assert np.all(np.isfinite(H)) and np.array_equal(H, H.T)
    assert lik.device_status() == 0
    lik32 = likelihood(model, data, mc, streams=("f32",))
    H32 = _np(lik32.hessian(th))
    F32 = _np(lik32.fit_fractions(th, with_grad=False))
    np.testing.assert_allclose(F32, Fo, rtol=1e-5, atol=1e-12)
    assert np.all(np.isfinite(H32))
    with pytest.raises(ValueError):
        lik32.fraction_matrix(th)                   # Gram route needs the FP64 stream

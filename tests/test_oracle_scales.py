"""Pins of the oracle's error yardsticks: the gradient scale
S_p = sum_data |d ln w/d theta_p| + (N_D/G) sum_MC |dw/d theta_p|
(`oracle.grad_scale`) and the Hessian-vector scale of eq. (7)
(`oracle.hvp_scale`).  Every GPU parity bound on a gradient or H v component
is a multiple of one of them, so a slip that inflated them would silently
loosen every check.  They are pinned against:

* closed forms for one resonance with a real coupling (every per-event term
  then has one sign and a value fixed by |c| alone);
* brute force on a tiny case: per-event derivatives by central differences of
  `oracle.intensity` (no dual numbers, a different code path), summed by hand;
* exact symmetries: duplicating every event doubles both scales (catches a
  lost N_D/G), and scaling the couplings by lambda scales S on the couplings
  by 1/lambda and leaves it unchanged on M and Gamma (catches a lost data
  1/w or a lost N_D/G);
* the triangle inequality: S >= |gradient| and hvp_scale >= |H v|, with a
  component that cancels, where S is far above |g| (catches abs-of-sum in
  place of sum-of-abs).
"""

import math

import numpy as np
import pytest

import oracle
import synth


def _events(n, seed):
    return synth.uniform_phase_space(n, np.random.Generator(np.random.PCG64(seed)))


def test_closed_form_one_resonance_real_coupling(make_model):
    """K = 1, c real.  Per data event d ln w/d Re c = 2/c and per MC event
    dw/d Re c = 2c|a|^2, so S_Rec = N_D (2/c) + (N_D/(c^2 sum|a|^2)) 2c sum|a|^2
    = 4 N_D / c, and S_Imc = 0.  Along v = e_Rec: per data event
    d^2 ln w/d Re c^2 = -2/c^2, |H_w v|/w = 2/c^2 and |dw| |wdot|/w^2 = 4/c^2;
    per MC event d^2 w/d Re c^2 = 2|a|^2.  So grad_scale's H v part is
    N_D 2/c^2 + (N_D/G) 2 sum|a|^2 = 4 N_D/c^2, and hvp_scale is
    6 N_D/c^2 + 2 N_D/c^2 + 2 (N_D/G^2)(2c sum|a|^2)^2 = 16 N_D/c^2."""
    model = make_model([0], [1])
    c = 0.7
    th = np.array([c, 0.0, 0.95, 0.12])
    data, mc = _events(37, 1), _events(53, 2)
    nd = 37
    S = oracle.grad_scale(data, mc, model, th)
    assert S[0] == pytest.approx(4 * nd / c, rel=1e-13)
    assert abs(S[1]) <= 1e-14 * S[0]
    e0 = np.array([1.0, 0.0, 0.0, 0.0])
    Sv, SH = oracle.grad_scale(data, mc, model, th, v=e0)
    assert Sv[0] == pytest.approx(4 * nd / c, rel=1e-13)
    assert SH[0] == pytest.approx(4 * nd / c ** 2, rel=1e-13)
    Hs = oracle.hvp_scale(data, mc, model, th, e0)
    assert Hs[0] == pytest.approx(16 * nd / c ** 2, rel=1e-13)
    # the value itself: the NLL does not depend on c at K = 1
    _, g, hv = oracle.hvp(data, mc, model, th, e0)
    assert abs(g[0]) <= 1e-13 * S[0] and abs(hv[0]) <= 1e-13 * Hs[0]


def _per_event_derivs(events, model, th, v, h=1e-5, t=1e-4):
    """Per event: w, dw/d theta_p (central differences of oracle.intensity)
    and (H_w v)_p (central difference of those along v)."""
    P = th.size

    def dw(x):
        out = np.empty((P, len(events[0])))
        for p in range(P):
            e = np.zeros(P)
            e[p] = h
            out[p] = (oracle.intensity(events, model, x + e) - oracle.intensity(events, model, x - e)) / (2 * h)
        return out

    w = oracle.intensity(events, model, th)
    g = dw(th)
    hv = (dw(th + t * v) - dw(th - t * v)) / (2 * t)
    return w, g, hv


def test_brute_force_tiny_case(make_model):
    """Both scales summed by hand from per-event central differences of the
    intensity (4 data events, 3 MC events, K = 2 in two channels)."""
    ch, sp = [0, 1], [0, 1]
    model = make_model(ch, sp)
    th = np.array([1.0, 0.0, 0.9, 0.1, 0.5, 0.4, 1.05, 0.08])
    data, mc = _events(4, 3), _events(3, 4)
    v = np.random.Generator(np.random.PCG64(5)).normal(size=th.size)
    wd, gd, hd = _per_event_derivs(data, model, th, v)
    wm, gm, hm = _per_event_derivs(mc, model, th, v)
    nd, G = len(wd), math.fsum(wm)
    S_bf = np.abs(gd / wd).sum(axis=1) + nd / G * np.abs(gm).sum(axis=1)
    wdot = v @ gd
    A = np.abs(gm).sum(axis=1)
    H_bf = ((np.abs(hd) / wd + np.abs(gd) * np.abs(wdot) / wd ** 2).sum(axis=1)
            + nd / G * np.abs(hm).sum(axis=1) + 2 * nd / G ** 2 * A * (np.abs(v) @ A))
    S = oracle.grad_scale(data, mc, model, th)
    np.testing.assert_allclose(S, S_bf, rtol=1e-7)
    Hs = oracle.hvp_scale(data, mc, model, th, v)
    np.testing.assert_allclose(Hs, H_bf, rtol=1e-5)
    # grad_scale's H v part is the absolute sum of the combined per-event terms
    _, SH = oracle.grad_scale(data, mc, model, th, v=v)
    SH_bf = np.abs(hd / wd - gd * wdot / wd ** 2).sum(axis=1) + nd / G * np.abs(hm).sum(axis=1)
    np.testing.assert_allclose(SH, SH_bf, rtol=1e-5)


def test_duplicating_events_doubles_the_scales(make_model):
    """Every event twice: N_D and G double, so N_D/G is unchanged and both
    absolute sums double exactly.  With 1/G in place of N_D/G the MC part
    would stay the same."""
    ch, sp = synth.resonance_layout(4)
    model = make_model(ch, sp)
    th = synth.draw_theta(ch, sp, np.random.Generator(np.random.PCG64(6)))
    data, mc = _events(60, 7), _events(90, 8)
    v = np.random.Generator(np.random.PCG64(9)).normal(size=th.size)
    d2 = (np.concatenate([data[0], data[0]]), np.concatenate([data[1], data[1]]))
    m2 = (np.concatenate([mc[0], mc[0]]), np.concatenate([mc[1], mc[1]]))
    np.testing.assert_allclose(oracle.grad_scale(d2, m2, model, th),
                               2 * oracle.grad_scale(data, mc, model, th), rtol=1e-13)
    np.testing.assert_allclose(oracle.hvp_scale(d2, m2, model, th, v),
                               2 * oracle.hvp_scale(data, mc, model, th, v), rtol=1e-13)
    # more MC alone leaves S's MC part per unit of N_D/G: doubling only the MC
    # halves N_D/G and doubles the MC sums, so S is unchanged
    np.testing.assert_allclose(oracle.grad_scale(data, m2, model, th),
                               oracle.grad_scale(data, mc, model, th), rtol=1e-13)


def test_coupling_rescaling(make_model):
    """c -> lambda c multiplies w by lambda^2: d ln w/dc scales as 1/lambda,
    (N_D/G) dw/dc as 1/lambda, and both are unchanged on M and Gamma.  A
    dropped data 1/w would make the data part scale as lambda (couplings) or
    lambda^2 (M, Gamma); a dropped N_D/G the MC part likewise."""
    ch, sp = synth.resonance_layout(5)
    model = make_model(ch, sp)
    th = synth.draw_theta(ch, sp, np.random.Generator(np.random.PCG64(10)))
    data, mc = _events(80, 11), _events(120, 12)
    lam = 3.0
    th2 = th.copy()
    th2[0::4] *= lam
    th2[1::4] *= lam
    S1 = oracle.grad_scale(data, mc, model, th)
    S2 = oracle.grad_scale(data, mc, model, th2)
    cpl = np.zeros(th.size, bool)
    cpl[0::4] = cpl[1::4] = True
    np.testing.assert_allclose(S2[cpl], S1[cpl] / lam, rtol=1e-12)
    np.testing.assert_allclose(S2[~cpl], S1[~cpl], rtol=1e-12)


def test_scales_bound_the_values_and_are_sums_of_abs(make_model):
    """Triangle inequality: S >= |g| and hvp_scale >= |H v| componentwise.
    Near a cancelling component the scale is far above the value (a scale
    computed as |sum| instead of sum |.| would equal it)."""
    ch, sp = synth.resonance_layout(6)
    model = make_model(ch, sp)
    th = synth.draw_theta(ch, sp, np.random.Generator(np.random.PCG64(13)))
    data = synth.resonant_like(300, ch, th, np.random.Generator(np.random.PCG64(14)))
    mc = _events(1200, 15)
    v = np.random.Generator(np.random.PCG64(16)).normal(size=th.size)
    _, g, hv = oracle.hvp(data, mc, model, th, v)
    S = oracle.grad_scale(data, mc, model, th)
    Hs = oracle.hvp_scale(data, mc, model, th, v)
    assert np.all(np.abs(g) <= S * (1 + 1e-12))
    assert np.all(np.abs(hv) <= Hs * (1 + 1e-12))
    assert np.max(S / np.maximum(np.abs(g), 1e-300)) > 10
    assert np.max(Hs / np.maximum(np.abs(hv), 1e-300)) > 10

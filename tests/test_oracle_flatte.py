"""Pins of the oracle's Flatte lineshape (the f0(980) form of the paper's
test model, Sec. 3 and Table 1) against facts that hold independently of its
code:

* with no coupling to the second channel it is the mass-dependent-width
  Breit-Wigner of a scalar, once g_1 = M Gamma / rho_ab(M^2);
* below the second threshold its phase-space factor is the value of the
  above-threshold expression at s + i0 (the physical sheet), evaluated here
  with complex 40-digit arithmetic;
* unitarity: Im T = |T|^2 for the open channel alone (below the second
  threshold, and for a single channel), and Im T_11 = |T_11|^2 + |T_12|^2
  with both channels open;
* the oracle's dual-number gradient and Hessian through the Flatte
  resonance match central finite differences of its NLL.
"""

import mpmath as mp
import numpy as np
import pytest

import oracle
import synth

M_F, G1_F = synth.FLATTE_F0
MK = synth.FLATTE_MASSES[0]
MPI = synth.DAUGHTER_MASSES[1]


def _s_grid(lo, hi, n=200):
    return np.linspace(lo, hi, n)


def test_flatte_without_second_channel_is_the_scalar_breit_wigner(make_model):
    """r = 0 and g_1 = M Gamma / rho_ab(M^2): identical to the J = 0
    Breit-Wigner with M Gamma(s) = Gamma M^2 q / (q0 sqrt s), in the pi pi
    channel (23) and in the K pi channel (12).  A wrong rho (q instead of
    2q/sqrt(s)) or a lost factor breaks it."""
    for ch in (2, 0):
        model = make_model([ch], [0], lineshape=[1], flatte_ratio=0.0)
        a, b, _ = synth.CHANNEL_PAIRS[ch]
        ma, mb = synth.DAUGHTER_MASSES[a], synth.DAUGHTER_MASSES[b]
        M, Gam = 1.1, 0.12
        rho0 = oracle.phase_space_factor(M * M, ma, mb).real
        g1 = M * Gam / rho0
        s = _s_grid((ma + mb) ** 2 * 1.0001, 2.5)
        # the scalar amplitudes depend on s alone: evaluate both forms at s
        q = np.sqrt(oracle.kallen(s, ma * ma, mb * mb)) / (2 * np.sqrt(s))
        bw = oracle.amplitude((s, q, np.zeros_like(s)), ch, 0, M, Gam, model, 0)
        fl = oracle.amplitude((s, q, np.zeros_like(s)), ch, 0, M, g1, model, 1)
        np.testing.assert_allclose(fl, bw, rtol=1e-13, atol=0)


def test_flatte_continuation_below_second_threshold(make_model):
    """Below 4 m_K^2 the K Kbar factor is the above-threshold expression
    sqrt(1 - 4 m^2 / s) (its cut is s < 4 m^2) evaluated at s + i eps, eps
    -> 0, in 40-digit complex arithmetic: positive imaginary, so the closed
    channel raises the real part of the denominator.  The amplitude is
    continuous across the threshold."""
    mp.mp.dps = 40
    model = make_model([2], [0], lineshape=[1])
    sth = 4 * MK * MK
    for s in _s_grid(4 * MPI * MPI * 1.01, sth * 0.999, 40):
        eps = mp.mpf("1e-25")
        sc = mp.mpf(float(s)) + 1j * eps
        ref = mp.sqrt(1 - 4 * mp.mpf(MK) ** 2 / sc)
        got = oracle.phase_space_factor(np.array([s]), MK, MK)[0]
        assert abs(complex(ref) - got) <= 1e-12 * abs(got)   # s - 4 m^2 cancels near threshold
        assert got.imag > 0 and abs(got.real) == 0.0
    # continuity of the amplitude at the threshold
    lo = oracle.amplitude((np.array([sth * (1 - 1e-12)]), None, None), 2, 0, M_F, G1_F, model, 1)
    hi = oracle.amplitude((np.array([sth * (1 + 1e-12)]), None, None), 2, 0, M_F, G1_F, model, 1)
    assert abs(lo[0] - hi[0]) <= 1e-4 * abs(hi[0])


def test_flatte_unitarity(make_model):
    """T_11 = g_1 rho_1 a: Im T_11 = |T_11|^2 where only the pi pi channel is
    open (with or without the K Kbar coupling) and, above 4 m_K^2,
    Im T_11 = |T_11|^2 + |T_12|^2 with T_12 = g_1 sqrt(r rho_1 rho_2) a.
    Pins the sign of i in the denominator and the factor r on rho_2."""
    for r in (0.0, synth.FLATTE_RATIO):
        model = make_model([2], [0], lineshape=[1], flatte_ratio=r)
        for s in np.concatenate([_s_grid(0.1, 0.97, 50), _s_grid(0.98, 1.8, 50)]):
            a = oracle.amplitude((np.array([s]), None, None), 2, 0, M_F, G1_F, model, 1)[0]
            rho1 = oracle.phase_space_factor(np.array([s]), MPI, MPI)[0].real
            rho2 = oracle.phase_space_factor(np.array([s]), MK, MK)[0]
            T11 = G1_F * rho1 * a
            if s < 4 * MK * MK or r == 0.0:
                assert abs(T11.imag - abs(T11) ** 2) <= 1e-12
            else:
                T12 = G1_F * np.sqrt(r * rho1 * rho2.real) * a
                assert abs(T11.imag - abs(T11) ** 2 - abs(T12) ** 2) <= 1e-12


def _flatte_case(make_model, n_data=300, n_mc=1500, seed=5):
    model = make_model([2, 0, 1], [0, 1, 2], lineshape=[1, 0, 0])
    rng = np.random.Generator(np.random.PCG64(seed))
    th = np.array([1.0, 0.0, M_F, G1_F,
                   0.7, 0.4, 0.892, 0.05,
                   0.3, -0.5, 1.43, 0.11])
    data = synth.uniform_phase_space(n_data, rng)
    mc = synth.uniform_phase_space(n_mc, rng)
    return model, th, data, mc


def test_flatte_gradient_and_hessian_match_differences(make_model):
    """Dual-number gradient and H v through the Flatte resonance (M, g_1)
    against central differences of the oracle's own NLL and gradient."""
    model, th, data, mc = _flatte_case(make_model)
    f0, g = oracle.grad(data, mc, model, th)
    S = oracle.grad_scale(data, mc, model, th)
    h = 1e-6
    for p in range(th.size):
        e = np.zeros_like(th)
        e[p] = h
        fd = (oracle.nll(data, mc, model, th + e) - oracle.nll(data, mc, model, th - e)) / (2 * h)
        assert abs(fd - g[p]) <= 1e-6 * S[p] + 1e-7 * abs(g[p]), p
    v = np.random.Generator(np.random.PCG64(9)).normal(size=th.size)
    _, _, hv = oracle.hvp(data, mc, model, th, v)
    hstep = 1e-5
    gp = oracle.grad(data, mc, model, th + hstep * v)[1]
    gm = oracle.grad(data, mc, model, th - hstep * v)[1]
    fd = (gp - gm) / (2 * hstep)
    SH = oracle.hvp_scale(data, mc, model, th, v)
    np.testing.assert_array_less(np.abs(fd - hv), 1e-5 * SH + 1e-6 * np.abs(hv))


def test_flatte_nll_reduces_to_breit_wigner_model(make_model):
    """Whole likelihood: a model whose scalar is a Flatte without the second
    channel equals the Breit-Wigner model with g_1 = M Gamma / rho_ab(M^2)."""
    model_f, th, data, mc = _flatte_case(make_model)
    model_f.flatte_ratio = 0.0
    model_b = make_model([2, 0, 1], [0, 1, 2])
    M, Gam = 0.98, 0.07
    rho0 = oracle.phase_space_factor(M * M, MPI, MPI).real
    th_b = th.copy()
    th_b[2:4] = (M, Gam)
    th_f = th.copy()
    th_f[2:4] = (M, M * Gam / rho0)
    assert oracle.nll(data, mc, model_f, th_f) == pytest.approx(
        oracle.nll(data, mc, model_b, th_b), rel=1e-13)

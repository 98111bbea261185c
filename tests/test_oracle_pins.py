"""Pins of the FP64 oracle against facts fixed by mathematics and by the
paper's definitions, independent of the oracle's own code path.

Each test names what it pins and what a plausible slip would break:
kinematics against explicit Lorentz boosts, barrier factors against
spherical Hankel functions, Legendre against scipy, the Breit-Wigner
against its closed-form integral, derivatives against finite differences
and exact symmetries, eq. (4)-(7) against the unsharded sums, and a tiny
case against an independent 50-digit implementation.
"""

import math

import mpmath as mp
import numpy as np
import pytest
from scipy import special

import oracle
import synth
from tests import indep_mp

M_P = synth.PARENT_MASS
MASSES = synth.DAUGHTER_MASSES


def _events(n, seed):
    return synth.uniform_phase_space(n, np.random.Generator(np.random.PCG64(seed)))


# ---------------------------------------------------------------- kinematics
def test_kinematics_against_lorentz_boosts(make_model):
    """cos(theta) and q of all three channels from explicit four-vectors
    (boost into the pair's rest frame) equal the oracle's closed form.
    Pins the helicity-angle formula, its sign convention (angle to -p_c) and
    the channel -> (a, b, c) table."""
    mp.mp.dps = 30
    model = make_model([0, 1, 2], [0, 0, 0])
    s12, s13 = _events(40, 11)
    for ch in range(3):
        s, q, cos = oracle.kinematics(s12, s13, ch, model)
        for i in range(len(s12)):
            vecs = indep_mp.four_vectors(s12[i], s13[i], M_P, MASSES)
            s_i, q_i, c_i = indep_mp.channel_kin(vecs, ch)
            assert abs(float(s_i) - s[i]) <= 1e-12 * s[i]
            assert abs(float(q_i) - q[i]) <= 1e-11 * q[i]
            assert abs(float(c_i) - cos[i]) <= 1e-9
    # invariant sum: s12 + s13 + s23 = M^2 + sum m^2
    s23 = oracle.kinematics(s12, s13, 2, model)[0]
    tot = M_P ** 2 + sum(m * m for m in MASSES)
    np.testing.assert_allclose(s12 + s13 + s23, tot, rtol=1e-14)


def test_helicity_angle_is_pm1_on_boundary(make_model):
    """On the Dalitz boundary (computed by the input generator's independent
    formula) the channel-(12) helicity angle is exactly +-1."""
    model = make_model([0], [0])
    s12 = np.linspace(0.45, 2.9, 50)
    lo, hi = synth.s13_range(s12)
    _, _, c_lo = oracle.kinematics(s12, lo, 0, model)
    _, _, c_hi = oracle.kinematics(s12, hi, 0, model)
    np.testing.assert_allclose(c_lo, -1.0, atol=1e-9)
    np.testing.assert_allclose(c_hi, 1.0, atol=1e-9)


def test_dalitz_area():
    """Area of the Dalitz region by quadrature equals the box area times the
    acceptance of uniform box points (two independent estimates)."""
    (a0, a1), (b0, b1) = synth.bounding_box()
    x = np.linspace(a0, a1, 200001)
    lo, hi = synth.s13_range(x)
    area = np.trapezoid(hi - lo, x)
    rng = np.random.Generator(np.random.PCG64(5))
    u = rng.uniform(a0, a1, 2_000_000)
    v = rng.uniform(b0, b1, 2_000_000)
    frac = synth.events.inside(u, v).mean()
    assert abs(area - frac * (a1 - a0) * (b1 - b0)) < 4e-3 * area
    assert abs(area - 3.1563) < 1e-3


# ---------------------------------------------------- barrier and Legendre
@pytest.mark.parametrize("J", [0, 1, 2])
def test_barrier_matches_spherical_hankel(J):
    """F_J(z)^-2 = z^J |x h_J(x)|^2 (x = sqrt z): the Blatt-Weisskopf
    factors are the outgoing-wave normalisation of the radial solution."""
    x = np.linspace(0.05, 6.0, 40)
    z = x * x
    h2 = special.spherical_jn(J, x) ** 2 + special.spherical_yn(J, x) ** 2
    expect = 1.0 / (z ** J * x * x * h2)
    got = np.asarray(oracle.barrier(J, z), dtype=float) ** 2 * np.ones_like(z)
    np.testing.assert_allclose(got, expect, rtol=1e-12)


@pytest.mark.parametrize("J", [0, 1, 2])
def test_legendre_matches_scipy(J):
    x = np.linspace(-1, 1, 33)
    np.testing.assert_allclose(oracle.legendre(J, x), special.eval_legendre(J, x),
                               rtol=0, atol=1e-15)


# ------------------------------------------------------ Breit-Wigner integral
def _bw_closed(M, G, lo, hi):
    mg = M * G
    return (math.atan((hi - M * M) / mg) - math.atan((lo - M * M) / mg)) / mg


def test_bw_integral_constant_width(make_model):
    """Constant width, J = 0: G * h over a midpoint grid in s12 equals the
    closed form of the integral of |1/(M^2 - s - i M Gamma)|^2
    [atan((s_hi - M^2)/(M Gamma)) - atan((s_lo - M^2)/(M Gamma))]/(M Gamma).
    Pins the BW denominator (sign of i M Gamma, M^2 - s) and the G sum."""
    model = make_model([0], [0], width_mode=1)
    M, G = 1.1, 0.08
    th = np.array([1.0, 0.0, M, G])
    n = 400_000
    s12, s13, h = synth.midpoint_line_s12(n)
    p = oracle.partials((s12[:1], s13[:1]), (s12, s13), model, th, order=0)
    (a0, a1), _ = synth.bounding_box()
    exact = _bw_closed(M, G, a0, a1)
    assert abs(p["G"] * h - exact) <= 1e-9 * exact
    # and it tends to pi/(M Gamma) for a narrow, central resonance
    Gn = 1e-3
    th = np.array([1.0, 0.0, M, Gn])
    p = oracle.partials((s12[:1], s13[:1]), (s12, s13), model, th, order=0)
    assert abs(p["G"] * h - math.pi / (M * Gn)) <= 2e-3 * math.pi / (M * Gn)


def test_bw_integral_mass_dependent_narrow(make_model):
    """Mass-dependent width, J = 0, Gamma/M = 1e-3: the integral over s12
    tends to pi/(M Gamma) (Gamma(s) -> Gamma at the pole), to O(Gamma/M)."""
    model = make_model([0], [0], width_mode=0)
    M, G = 1.1, 1.1e-3
    th = np.array([1.0, 0.0, M, G])
    s12, s13, h = synth.midpoint_line_s12(2_000_000)
    p = oracle.partials((s12[:1], s13[:1]), (s12, s13), model, th, order=0)
    ref = math.pi / (M * G)
    assert abs(p["G"] * h - ref) <= 5e-3 * ref


# -------------------------------------------------------------- derivatives
def _small_case(make_model, K=6, nd=300, nm=1500, seed=3):
    ch, sp = synth.resonance_layout(K)
    model = make_model(ch, sp)
    th = synth.draw_theta(ch, sp, np.random.Generator(np.random.PCG64(seed)))
    data = synth.resonant_like(nd, ch, th, np.random.Generator(np.random.PCG64(seed + 1)))
    mc = _events(nm, seed + 2)
    return model, th, data, mc


def test_gradient_matches_central_differences(make_model):
    """Analytic gradient vs central differences (h = 1e-6), compared on the
    absolute-sum scale S_p (a plain relative test fails where g ~ 0)."""
    model, th, data, mc = _small_case(make_model)
    f0, g = oracle.grad(data, mc, model, th)
    S = oracle.grad_scale(data, mc, model, th)
    h = 1e-6
    for p in range(th.size):
        e = np.zeros_like(th)
        e[p] = h
        fd = (oracle.nll(data, mc, model, th + e) - oracle.nll(data, mc, model, th - e)) / (2 * h)
        assert abs(fd - g[p]) <= 1e-6 * S[p] + 1e-7 * abs(g[p]), p
    assert f0 == pytest.approx(oracle.nll(data, mc, model, th), rel=1e-14)


def test_hessian_symmetric_and_matches_fd(make_model):
    """Exact (dual-number) Hessian is symmetric to rounding and equals the
    central difference of the analytic gradient."""
    model, th, data, mc = _small_case(make_model, K=4, nd=200, nm=1000)
    H = oracle.hessian(data, mc, model, th)
    assert np.max(np.abs(H - H.T)) <= 1e-10 * np.max(np.abs(H))
    h = 1e-6
    for p in range(th.size):
        e = np.zeros_like(th)
        e[p] = h
        col = (oracle.grad(data, mc, model, th + e)[1] - oracle.grad(data, mc, model, th - e)[1]) / (2 * h)
        assert np.max(np.abs(col - H[:, p])) <= 1e-5 * np.max(np.abs(H)), p


def _J(th):
    """90-degree rotation of every (Re c, Im c) pair; zero on M, Gamma."""
    out = np.zeros_like(th)
    out[0::4] = -th[1::4]
    out[1::4] = th[0::4]
    return out


def _Jvec(g):
    out = np.zeros_like(g)
    out[0::4] = -g[1::4]
    out[1::4] = g[0::4]
    return out


def _Jabs(s):
    """|J| applied to a nonnegative scale vector (swaps each coupling pair)."""
    out = np.zeros_like(s)
    out[0::4] = s[1::4]
    out[1::4] = s[0::4]
    return out


def _Pi(th):
    out = np.zeros_like(th)
    out[0::4] = th[0::4]
    out[1::4] = th[1::4]
    return out


def test_phase_invariance(make_model):
    """NLL(e^{i phi} c) = NLL(c); grad . J theta = 0; H (J theta) = J grad.
    (The last follows from differentiating grad(R theta) . J R theta = 0.)"""
    model, th, data, mc = _small_case(make_model)
    f0 = oracle.nll(data, mc, model, th)
    ph = 0.7
    th2 = th.copy()
    c = (th[0::4] + 1j * th[1::4]) * np.exp(1j * ph)
    th2[0::4], th2[1::4] = c.real, c.imag
    assert oracle.nll(data, mc, model, th2) == pytest.approx(f0, rel=1e-13)
    Jt = _J(th)
    _, g, hv = oracle.hvp(data, mc, model, th, Jt)
    S = oracle.grad_scale(data, mc, model, th)
    SH = oracle.hvp_scale(data, mc, model, th, Jt)
    assert abs(g @ Jt) <= 1e-12 * (S @ np.abs(Jt))
    Jg = _Jvec(g)
    # J g carries the gradient's rounding: bound by both scales
    assert np.all(np.abs(hv - Jg) <= 1e-11 * (SH + _Jabs(S)))


def test_scale_invariance(make_model):
    """NLL(lambda c) = NLL(c); grad . Pi theta = 0; H (Pi theta) = -Pi grad."""
    model, th, data, mc = _small_case(make_model)
    f0 = oracle.nll(data, mc, model, th)
    th2 = th.copy()
    th2[0::4] *= 2.5
    th2[1::4] *= 2.5
    assert oracle.nll(data, mc, model, th2) == pytest.approx(f0, rel=1e-13)
    Pt = _Pi(th)
    _, g, hv = oracle.hvp(data, mc, model, th, Pt)
    S = oracle.grad_scale(data, mc, model, th)
    SH = oracle.hvp_scale(data, mc, model, th, Pt)
    assert abs(g @ Pt) <= 1e-12 * (S @ np.abs(Pt))
    # Pi g carries the gradient's rounding: bound by both scales
    assert np.all(np.abs(hv + _Pi(g)) <= 1e-11 * (SH + _Pi(S)))


def test_single_resonance_coupling_free(make_model):
    """K = 1: the NLL does not depend on c, so dNLL/dc = 0 and the Hessian
    rows and columns of c vanish (to rounding)."""
    model = make_model([1], [1])
    th = np.array([0.7, -0.4, 1.2, 0.15])
    data = _events(200, 8)
    mc = _events(900, 9)
    _, g, _ = oracle.hvp(data, mc, model, th, np.ones(4))
    S = oracle.grad_scale(data, mc, model, th)
    assert abs(g[0]) <= 1e-12 * S[0] and abs(g[1]) <= 1e-12 * S[1]
    H = oracle.hessian(data, mc, model, th)
    assert np.max(np.abs(H[:2, :])) <= 1e-10 * np.max(np.abs(H))


# ------------------------------------------------ Legendre orthogonality
@pytest.mark.parametrize("J1,J2", [(0, 1), (0, 2), (1, 2)])
def test_legendre_orthogonality_on_symmetric_rule(make_model, J1, J2):
    """Two resonances of spins J1 != J2 in channel (12).  At each s12 of a
    grid, three MC points sit at cos(theta) = 0, +-1/sqrt(2) (placed with the
    generator's boundary, which is independent of the oracle): this
    equal-weight (Chebyshev) rule integrates polynomials of degree <= 3 in
    cos(theta) exactly, so the interference term of the Gram matrix vanishes
    while no amplitude is zero at the nodes."""
    model = make_model([0, 0], [J1, J2])
    th = np.array([1.0, 0.0, 0.9, 0.1, 1.0, 0.0, 1.3, 0.2])
    (a0, a1), _ = synth.bounding_box()
    s12 = np.linspace(a0, a1, 3002)[1:-1]
    lo, hi = synth.s13_range(s12)
    nodes = (-1.0 / math.sqrt(2.0), 0.0, 1.0 / math.sqrt(2.0))
    s13 = np.concatenate([lo + (hi - lo) * (1 + x) / 2 for x in nodes])
    ev = (np.concatenate([s12] * 3), s13)
    Gm = oracle.gram(ev, model, th)
    assert abs(Gm[0, 1]) <= 1e-12 * math.sqrt(Gm[0, 0].real * Gm[1, 1].real)


def test_legendre_orthogonality_mirror_mc(make_model):
    """S-P interference vanishes on a mirror-symmetric random MC (each point
    paired with its cos(theta) -> -cos(theta) image)."""
    model = make_model([0, 0], [0, 1])
    th = np.array([1.0, 0.0, 0.9, 0.1, 0.6, 0.3, 0.892, 0.05])
    ev = synth.mirror_symmetric(*_events(20000, 21))
    Gm = oracle.gram(ev, model, th)
    assert abs(Gm[0, 1]) <= 1e-12 * math.sqrt(Gm[0, 0].real * Gm[1, 1].real)


# ------------------------------------------------------- shard identity
def test_shard_combine_equals_unsharded(make_model):
    """Eq. (4)-(7): per-shard F_m, G_m and derivatives combined equal the
    unsharded NLL, gradient and HVP (the middle term of eq. (7) summed over
    shards)."""
    model, th, data, mc = _small_case(make_model)
    v = np.random.Generator(np.random.PCG64(77)).normal(size=th.size)
    f, g, hv = oracle.hvp(data, mc, model, th, v)
    cuts_d = [0, 37, 150, len(data[0])]
    cuts_m = [0, 500, 501, len(mc[0])]
    parts = []
    for i in range(3):
        d = (data[0][cuts_d[i]:cuts_d[i + 1]], data[1][cuts_d[i]:cuts_d[i + 1]])
        m = (mc[0][cuts_m[i]:cuts_m[i + 1]], mc[1][cuts_m[i]:cuts_m[i + 1]])
        parts.append(oracle.partials(d, m, model, th, v=v))
    out = oracle.combine(parts, v=v)
    S = oracle.grad_scale(data, mc, model, th)
    SH = oracle.hvp_scale(data, mc, model, th, v)
    assert out["nll"] == pytest.approx(f, rel=1e-13)
    assert np.all(np.abs(out["grad"] - g) <= 1e-13 * S)
    assert np.all(np.abs(out["hv"] - hv) <= 1e-12 * SH)


# -------------------------------------------- tiny independent brute force
def test_tiny_case_against_independent_50_digit_implementation(make_model):
    """N_D = 3, N_MC = 5, one resonance per channel with J = 0, 1, 2:
    NLL, gradient and H v of the oracle vs an independent mpmath
    implementation (four-vectors, spherical Hankel barriers, numerical
    differentiation at 50 digits)."""
    mp.mp.dps = 50
    ch, sp = [0, 1, 2], [1, 2, 0]
    model = make_model(ch, sp)
    th = np.array([1.0, 0.0, 0.92, 0.12, 0.5, -0.4, 1.05, 0.09, -0.3, 0.8, 0.75, 0.2])
    data = _events(3, 31)
    mc = _events(5, 32)
    v = np.random.Generator(np.random.PCG64(33)).normal(size=th.size)
    ref = indep_mp.TinyNLL(data, mc, ch, sp, M_P, MASSES, synth.R_BARRIER)
    f, g, hv = oracle.hvp(data, mc, model, th, v)
    f_ref = ref(*th)
    assert abs(f - float(f_ref)) <= 1e-13 * max(1.0, abs(float(f_ref)))
    P = th.size
    g_ref = np.array([float(mp.diff(lambda t: ref(*[th[j] + (t if j == p else 0) for j in range(P)]), 0))
                      for p in range(P)])
    S = oracle.grad_scale(data, mc, model, th)
    SH = oracle.hvp_scale(data, mc, model, th, v)
    assert np.all(np.abs(g - g_ref) <= 1e-12 * S)

    def dir2(p):
        f2 = lambda t, u: ref(*[th[j] + (t if j == p else 0) + u * v[j] for j in range(P)])  # noqa: E731
        return float(mp.diff(f2, (0, 0), (1, 1)))
    hv_ref = np.array([dir2(p) for p in range(P)])
    assert np.all(np.abs(hv - hv_ref) <= 1e-11 * SH)


def test_constant_width_tiny_case_independent(make_model):
    """Same as above with the constant-width option."""
    mp.mp.dps = 40
    ch, sp = [0, 0], [0, 2]
    model = make_model(ch, sp, width_mode=1)
    th = np.array([1.0, 0.0, 0.9, 0.1, 0.4, 0.4, 1.25, 0.18])
    data = _events(3, 41)
    mc = _events(4, 42)
    ref = indep_mp.TinyNLL(data, mc, ch, sp, M_P, MASSES, synth.R_BARRIER, width_mode=1)
    assert oracle.nll(data, mc, model, th) == pytest.approx(float(ref(*th)), rel=1e-13)


def test_below_threshold_is_infinite(make_model):
    """A resonance mass below its pair threshold makes the NLL +inf."""
    model = make_model([2], [0])
    data, mc = _events(5, 1), _events(7, 2)
    th = np.array([1.0, 0.0, 0.25, 0.1])      # threshold (23) is 0.28 GeV
    assert oracle.nll(data, mc, model, th) == math.inf


# -------------------------------------------------- batched (fixed M, Gamma)
def test_batched_gram_identity(make_model):
    """c^H Gm c equals sum_j |(A c)_j|^2 evaluated directly, and the batched
    per-start NLL equals the plain NLL with theta's couplings replaced."""
    ch, sp = synth.resonance_layout(5)
    model = make_model(ch, sp)
    th = synth.draw_theta(ch, sp, np.random.Generator(np.random.PCG64(4)))
    mc = _events(3000, 5)
    data = _events(400, 6)
    Gm = oracle.gram(mc, model, th)
    rng = np.random.Generator(np.random.PCG64(7))
    C = rng.normal(size=(5, 3)) + 1j * rng.normal(size=(5, 3))
    A = np.stack(oracle.amplitudes(mc, model, th), axis=1)
    for b in range(3):
        direct = math.fsum(np.abs(A @ C[:, b]) ** 2)
        quad = (C[:, b].conj() @ Gm @ C[:, b]).real
        assert quad == pytest.approx(direct, rel=1e-12)
    nb = oracle.nll_batched(data, mc, model, th, C)
    for b in range(3):
        t2 = th.copy()
        t2[0::4], t2[1::4] = C[:, b].real, C[:, b].imag
        assert nb[b] == pytest.approx(oracle.nll(data, mc, model, t2), rel=1e-12)


def test_round_to_formats():
    x = np.array([1.0, 1.0 + 2 ** -9, 1.0 + 3 * 2 ** -9, 3.14159265])
    np.testing.assert_array_equal(oracle.round_to(x, "bf16")[:3], [1.0, 1.0, 1.0 + 2 ** -7])
    assert oracle.round_to(np.array([1.0 + 2 ** -12]), "f16")[0] == 1.0


# ------------------------------------ sliced FP16 operand format (batched)
def test_fixed_slices_worked_example():
    """x = (1.5, 2^-20 + 2^-30): |max| = 1.5 < 2^1, so the row is scaled by
    2^8 to (384, 2^-12 + 2^-22); slice by slice (remainder times 2^9):
    q0 = (384, 0), q1 = (0, 0) [2^-3 + 2^-13 rounds to 0],
    q2 = (0, 64) [64 + 2^-4], q3 = (0, 32) [2^-4 * 2^9], remainder 0."""
    q, E = oracle.fixed_slices(np.array([[1.5, 2.0 ** -20 + 2.0 ** -30]]), axis=1)
    assert E[0, 0] == 1
    np.testing.assert_array_equal(np.array(q)[:, 0, :], [[384, 0], [0, 0], [0, 64], [0, 32]])


def test_fixed_slices_bounds_and_reconstruction():
    """Slices are integers with |q0| <= 512 and |q_s| <= 256 after it; the
    reconstruction misses x by at most 2^(E - 37); a value on the 2^(E-36)
    grid is reproduced exactly; zero vectors give E = 0 and zero slices."""
    rng = np.random.Generator(np.random.PCG64(21))
    x = rng.normal(size=(200, 40)) * 10.0 ** rng.uniform(-6, 6, size=(200, 1))
    x[7] = 0.0
    q, E = oracle.fixed_slices(x, axis=1)
    q = np.array(q)
    assert np.all(q == np.rint(q))
    assert np.max(np.abs(q[0])) <= 512 and np.max(np.abs(q[1:])) <= 256
    rec = sum(np.ldexp(q[s], E - 9 - 9 * s) for s in range(4))
    assert np.all(np.abs(rec - x) <= np.ldexp(1.0, E - 37))
    assert E[7, 0] == 0 and np.all(q[:, 7] == 0)
    assert np.all(np.abs(x) < np.ldexp(1.0, E)) and np.all(np.max(np.abs(x), axis=1, keepdims=True)[E != 0]
                                                         >= np.ldexp(1.0, E - 1)[E != 0])
    g = np.ldexp(rng.integers(-2 ** 35, 2 ** 35, size=(50, 8)).astype(float), -36)   # |g| < 2^-1
    g[:, 0] = 0.75                                                                   # E = 0 per row
    qg, Eg = oracle.fixed_slices(g, axis=1)
    assert np.all(Eg == 0)
    np.testing.assert_array_equal(sum(np.ldexp(qg[s], -9 - 9 * s) for s in range(4)), g)


def test_sliced_product_error_bound():
    """|Z - A C| <= K 2^(E_row + G_col - 35) elementwise: per term the
    remainders contribute at most 2^-28 of 512 in slice units (twice) and
    the dropped slice pairs (i + j = 4 .. 6) at most 3 2^-36 2^16 + 2 2^-45
    2^16 + 2^-54 2^16.  Dropping the last level breaks it more than
    tenfold."""
    rng = np.random.Generator(np.random.PCG64(22))
    K = 20
    A = (rng.normal(size=(300, K)) + 1j * rng.normal(size=(300, K))) * 10.0 ** rng.uniform(-3, 3, (300, K))
    C = rng.uniform(0, 1, (K, 16)) * np.exp(2j * np.pi * rng.uniform(size=(K, 16)))
    Z = oracle.sliced_product(A, C)
    _, Ea = oracle.fixed_slices(A, axis=1)
    _, Gc = oracle.fixed_slices(C, axis=0)
    exact = A @ C
    bound = K * np.ldexp(1.0, Ea + Gc - 35)
    assert np.all(np.abs(Z - exact) <= bound)
    assert np.max(np.abs(Z - exact) / bound) > 1e-6          # the bound is not vacuous
    # with one level fewer the error is far outside it
    qa, _ = oracle.fixed_slices(A, axis=1)
    qc, _ = oracle.fixed_slices(C, axis=0)
    Z2 = sum(np.ldexp(1.0, -9 * (i + j)) * (qa[i] @ qc[j]) for i in range(4) for j in range(4) if i + j <= 2)
    Z2 = Z2 * np.ldexp(1.0, Ea + Gc - 18)
    assert np.max(np.abs(Z2 - exact) / bound) > 10


def test_sliced_nll_matches_fp64_on_representable_operands(make_model):
    """Where every amplitude and coupling lies on its slice grid (here: C
    with 12-bit components, and the level sum holds them exactly), the
    sliced-format NLL equals the FP64 one up to the sums' rounding; on
    general operands it stays within the error the bound above allows."""
    ch, sp = synth.resonance_layout(4)
    model = make_model(ch, sp)
    th = synth.draw_theta(ch, sp, np.random.Generator(np.random.PCG64(31)))
    data, mc = _events(500, 32), _events(2000, 33)
    rng = np.random.Generator(np.random.PCG64(34))
    C = rng.uniform(0, 1, (4, 6)) * np.exp(2j * np.pi * rng.uniform(size=(4, 6)))
    ref = oracle.nll_batched(data, mc, model, th, C)
    got = oracle.nll_batched(data, mc, model, th, C, fmt="f16s")
    assert np.max(np.abs(got - ref)) <= 1e-6
    # an amplitude matrix on the grid: a row whose entries are small integers
    A = rng.integers(-300, 300, size=(50, 4)) + 1j * rng.integers(-300, 300, size=(50, 4))
    Cg = (rng.integers(-2048, 2048, size=(4, 6)) + 1j * rng.integers(-2048, 2048, size=(4, 6))) * 2.0 ** -11
    np.testing.assert_array_equal(oracle.sliced_product(A.astype(complex), Cg), A @ Cg)

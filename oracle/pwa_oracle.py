"""FP64 CPU oracle for the unbinned partial-wave-analysis likelihood, its
gradient and its Hessian-vector product.

TEST INFRASTRUCTURE ONLY: used by the test suite, the package smoke check and
the benchmark's CPU-baseline leg; never by the product path.  It shares no
code with the HIP library.

What is computed (paper Sec. 2.2 and 2.3):

* Intensity, eq. (1): omega(x) = |z(x)|^2 with z = sum_k c_k a_k(x).  The
  parent here has spin 0, so the helicity sum over mu has a single term, and
  the overall factor 1/2 is dropped exactly as eq. (3) drops it.
* Likelihood, eq. (2)-(3), efficiency = 1 (phase-space MC):
      ln L = sum_{data} ln omega - N_D ln( (1/N_MC) sum_{MC} omega ),
  and the oracle returns NLL = -ln L.
* Per-shard sums, eq. (4)-(5): F = sum_data ln omega, G = sum_MC omega, and
  their first derivatives and Hessian-vector products; eq. (6)-(7) combine
  them.  Eq. (7) as printed drops the sum over shards on its middle term;
  `combine` sums it over shards (the only reading consistent with eq. (4)).

Amplitude model (the paper builds covariant-tensor amplitudes, Sec. 2.2; for
a spin-0 parent decaying to three pseudoscalars the scalar isobar form is used):

    a_k(x) = P_J(cos th) * [F_J(z)/F_J(z0)] / (M^2 - s - i M Gamma(s))
    Gamma(s) = Gamma * (q/q0)^(2J+1) * (M/sqrt(s)) * [F_J(z)/F_J(z0)]^2
    z = (q r)^2, z0 = (q0 r)^2, q0 = q(s = M^2), r = 3 GeV^-1,
    F_0 = 1, F_1 = (1+z)^(-1/2), F_2 = (z^2+3z+9)^(-1/2)   (Blatt-Weisskopf)

Width mode 1 ("constant") sets Gamma(s) = Gamma.

Derivatives: the gradient is the analytic chain rule over the couplings and
over each amplitude's M and Gamma, the latter obtained exactly by forward-mode
dual numbers.  The Hessian-vector product is the same gradient code evaluated
on dual numbers whose tangent is v (forward over the analytic gradient), so
it carries no truncation error.  All event sums use math.fsum (correctly
rounded).
"""

import itertools
import math

import numpy as np

# Daughter pairs of each channel, 0-based: (a, b, bachelor c).
#   channel 0 = (12) with c = 3, channel 1 = (13) with c = 2,
#   channel 2 = (23) with c = 1.
_PAIRS = ((0, 1, 2), (0, 2, 1), (1, 2, 0))


class DomainError(ValueError):
    """A resonance mass at or below its two-body threshold (q0^2 <= 0)."""


# --------------------------------------------------------------------------
# Forward-mode dual numbers with tags (nested differentiation).
# --------------------------------------------------------------------------
_TAGS = itertools.count(1)


def new_tag():
    return next(_TAGS)


def _tag(x):
    return x.t if isinstance(x, Dual) else 0


def _parts(x, t):
    if isinstance(x, Dual) and x.t == t:
        return x.a, x.b
    return x, None


def _tadd(p, q):
    if p is None:
        return q
    if q is None:
        return p
    return p + q


def _add(x, y):
    t = max(_tag(x), _tag(y))
    xa, xb = _parts(x, t)
    ya, yb = _parts(y, t)
    return Dual(xa + ya, _tadd(xb, yb), t)


def _mul(x, y):
    t = max(_tag(x), _tag(y))
    xa, xb = _parts(x, t)
    ya, yb = _parts(y, t)
    tb = None
    if xb is not None:
        tb = xb * ya
    if yb is not None:
        tb = _tadd(tb, xa * yb)
    return Dual(xa * ya, tb, t)


def _div(x, y):
    t = max(_tag(x), _tag(y))
    xa, xb = _parts(x, t)
    ya, yb = _parts(y, t)
    q = xa / ya
    tb = None
    if xb is not None:
        tb = xb / ya
    if yb is not None:
        tb = _tadd(tb, -(q * yb) / ya)
    return Dual(q, tb, t)


class Dual:
    """a + b*eps with eps^2 = 0.  Components may be floats, numpy arrays
    (real or complex) or Duals of a lower tag; the highest tag is outermost."""
    __array_ufunc__ = None
    __slots__ = ("a", "b", "t")

    def __init__(self, a, b, t):
        self.a, self.b, self.t = a, b, t

    def __add__(self, o):
        return _add(self, o)

    def __radd__(self, o):
        return _add(o, self)

    def __sub__(self, o):
        return _add(self, -o)

    def __rsub__(self, o):
        return _add(o, -self)

    def __neg__(self):
        return Dual(-self.a, -self.b, self.t)

    def __mul__(self, o):
        return _mul(self, o)

    def __rmul__(self, o):
        return _mul(o, self)

    def __truediv__(self, o):
        return _div(self, o)

    def __rtruediv__(self, o):
        return _div(o, self)


def primal(x):
    while isinstance(x, Dual):
        x = x.a
    return x


def dsqrt(x):
    if isinstance(x, Dual):
        s = dsqrt(x.a)
        return Dual(s, x.b / (2.0 * s), x.t)
    return np.sqrt(x)


def dlog(x):
    if isinstance(x, Dual):
        return Dual(dlog(x.a), x.b / x.a, x.t)
    return np.log(x)


def dconj(x):
    if isinstance(x, Dual):
        return Dual(dconj(x.a), dconj(x.b), x.t)
    return np.conj(x)


def dreal(x):
    if isinstance(x, Dual):
        return Dual(dreal(x.a), dreal(x.b), x.t)
    return np.real(x)


def dimag(x):
    if isinstance(x, Dual):
        return Dual(dimag(x.a), dimag(x.b), x.t)
    return np.imag(x)


def dabs(x):
    """Componentwise absolute value (used only for error-scale sums)."""
    if isinstance(x, Dual):
        return Dual(dabs(x.a), dabs(x.b), x.t)
    return np.abs(x)


def fsum(x):
    """Correctly rounded sum of all elements (componentwise for Duals)."""
    if isinstance(x, Dual):
        return Dual(fsum(x.a), fsum(x.b), x.t)
    x = np.asarray(x)
    if np.iscomplexobj(x):
        return complex(math.fsum(np.ravel(x.real)), math.fsum(np.ravel(x.imag)))
    return math.fsum(np.ravel(x))


def ipow(x, n):
    out = x
    for _ in range(n - 1):
        out = out * x
    return out


# --------------------------------------------------------------------------
# Kinematics (two-body breakup momenta and helicity angles).
# --------------------------------------------------------------------------
def kallen(x, y, z):
    """Kallen triangle function lambda(x, y, z)."""
    return x * x + y * y + z * z - 2.0 * (x * y + x * z + y * z)


def breakup_sq(s, ma, mb):
    """Squared breakup momentum of a two-body system of mass^2 s into (ma, mb)."""
    return kallen(s, ma * ma, mb * mb) / (4.0 * s)


def kinematics(s12, s13, channel, model):
    """Invariant mass^2 s of the channel's pair (a b), breakup momentum q of
    a in the (ab) rest frame, and cos of the helicity angle: the angle in the
    (ab) rest frame between a and the direction opposite to the bachelor c.

    With E_a*, E_c* the energies of a and c in the (ab) frame and p* the
    bachelor momentum there:
        s_ac = m_a^2 + m_c^2 + 2 E_a* E_c* + 2 q p* cos(th)."""
    M = model.parent_mass
    m = model.masses
    a, b, c = _PAIRS[channel]
    ma2, mb2, mc2 = m[a] ** 2, m[b] ** 2, m[c] ** 2
    s12 = np.asarray(s12, dtype=np.float64)
    s13 = np.asarray(s13, dtype=np.float64)
    s23 = M * M + sum(mi * mi for mi in m) - s12 - s13
    s_ab, s_ac = ((s12, s13), (s13, s12), (s23, s12))[channel]
    rs = np.sqrt(s_ab)
    q = np.sqrt(np.maximum(kallen(s_ab, ma2, mb2), 0.0)) / (2.0 * rs)
    p = np.sqrt(np.maximum(kallen(M * M, s_ab, mc2), 0.0)) / (2.0 * rs)
    ea = (s_ab + ma2 - mb2) / (2.0 * rs)
    ec = (M * M - s_ab - mc2) / (2.0 * rs)
    cos = (s_ac - ma2 - mc2 - 2.0 * ea * ec) / (2.0 * q * p)
    return s_ab, q, cos


def barrier(J, z):
    """Blatt-Weisskopf damping factor F_J(z), z = (q r)^2."""
    if J == 0:
        return 1.0
    if J == 1:
        return 1.0 / dsqrt(1.0 + z)
    if J == 2:
        return 1.0 / dsqrt(z * z + 3.0 * z + 9.0)
    raise ValueError("spin must be 0, 1 or 2")


def legendre(J, x):
    if J == 0:
        return np.ones_like(x)
    if J == 1:
        return x
    if J == 2:
        return 1.5 * x * x - 0.5
    raise ValueError("spin must be 0, 1 or 2")


def phase_space_factor(s, ma, mb):
    """Two-body phase-space factor rho(s) = 2 q / sqrt(s) = sqrt(lambda(s, ma^2, mb^2)) / s,
    continued below threshold (lambda < 0) on the physical sheet (s + i0):
    rho = +i sqrt(-lambda) / s."""
    lam = kallen(np.asarray(s, dtype=np.float64), ma * ma, mb * mb)
    return np.where(lam >= 0.0, np.sqrt(np.abs(lam)) / s, 1j * np.sqrt(np.abs(lam)) / s)


def flatte_factor(s, channel, model):
    """The Flatte width factor rho_ab(s) + r rho_2(s) of a scalar resonance in
    `channel` (pair a b of the daughters): rho_ab of the channel's own pair and
    rho_2 of the coupled second channel (masses model.flatte_masses, coupling
    ratio r = model.flatte_ratio = g_2 / g_1), complex below its threshold."""
    a, b, _ = _PAIRS[channel]
    m1, m2 = model.flatte_masses
    return (phase_space_factor(s, model.masses[a], model.masses[b])
            + model.flatte_ratio * phase_space_factor(s, m1, m2))


def lineshape_of(model, k):
    """0: relativistic Breit-Wigner; 1: Flatte (scalar resonances only)."""
    ls = getattr(model, "lineshape", None)
    return 0 if ls is None else int(ls[k])


def amplitude(kin, channel, J, M, G, model, shape=0, angular=None):
    """a(x) = P_J(cos) (F_J(z)/F_J(z0)) / (M^2 - s - i M Gamma(s)), or for a
    Flatte resonance (shape 1, J = 0; G is the coupling g_1 in GeV^2)
        a(x) = 1 / (M^2 - s - i g_1 [rho_ab(s) + r rho_2(s)]).
    `angular` replaces P_J(cos) (a spin-1 parent's Y_J^mu).

    M and G may be dual numbers (for derivatives)."""
    s, q, cos = kin[:3]
    if shape == 1:
        if J != 0:
            raise ValueError("the Flatte lineshape is for scalar resonances")
        lin = 1.0 / (M * M - s - 1j * (G * flatte_factor(s, channel, model)))
        return lin if angular is None else angular * lin
    a, b, _ = _PAIRS[channel]
    ma, mb = model.masses[a], model.masses[b]
    r2 = model.r * model.r
    M2 = M * M
    q0sq = breakup_sq(M2, ma, mb)
    if not primal(q0sq) > 0.0:
        raise DomainError("resonance mass at or below threshold")
    ratio = barrier(J, q * q * r2) / barrier(J, q0sq * r2)
    if model.width_mode == 0:
        gs = G * ipow(q / dsqrt(q0sq), 2 * J + 1) * (M / np.sqrt(s)) * (ratio * ratio)
    else:
        gs = G
    ang = legendre(J, cos) if angular is None else angular
    return ang * ratio / (M2 - s - 1j * (M * gs))


# --------------------------------------------------------------------------
# Spin-1 parent (the helicity sum of eq. (1), mu = +1, -1).  Reading: events
# carry (s12, s13, cos beta, gamma); in the parent rest frame the daughters
# lie in the plane reached from the reference plane (p_1 along x, p_2 in the
# upper x-y half plane) by R_y(beta) R_z(gamma).  For channel (ab) with
# bachelor c, with p^_c the unit bachelor momentum and q^ the unit momentum
# of a in the (ab) rest frame, and e_+ = -(1, i, 0)/sqrt2,
# e_- = (1, -i, 0)/sqrt2:
#   Y_0 = e.p^_c,  Y_1 = e.(p^_c x q^),  Y_2 = e_i (q^_i q^_j - delta_ij/3) p^_c_j,
# and the amplitude's angular factor is Y_J^mu in place of P_J(cos theta).
# --------------------------------------------------------------------------
def parent_spin(model):
    return int(getattr(model, "parent_spin", 0))


def n_helicities(model):
    return 2 if parent_spin(model) == 1 else 1


POLARISATIONS = (np.array([-1.0, -1j, 0.0]) / math.sqrt(2.0),   # mu = +1
                 np.array([1.0, -1j, 0.0]) / math.sqrt(2.0))    # mu = -1


def daughter_momenta(s12, s13, cosb, gamma, model):
    """Four-momenta (n, 3, 4) of the daughters in the parent rest frame for
    the orientation (cos beta, gamma)."""
    M = model.parent_mass
    m = np.asarray(model.masses, dtype=np.float64)
    s12 = np.asarray(s12, dtype=np.float64)
    s13 = np.asarray(s13, dtype=np.float64)
    s23 = M * M + np.sum(m * m) - s12 - s13
    E = np.stack([(M * M + m[0] ** 2 - s23) / (2 * M), (M * M + m[1] ** 2 - s13) / (2 * M),
                  (M * M + m[2] ** 2 - s12) / (2 * M)], axis=1)
    pm = np.sqrt(np.maximum(E * E - m * m, 0.0))
    # |p_3|^2 = |p_1 + p_2|^2 fixes the angle between p_1 and p_2
    c12 = np.clip((pm[:, 2] ** 2 - pm[:, 0] ** 2 - pm[:, 1] ** 2) / (2 * pm[:, 0] * pm[:, 1]), -1, 1)
    s12a = np.sqrt(1.0 - c12 * c12)
    n = len(s12)
    body = np.zeros((n, 3, 3))
    body[:, 0, 0] = pm[:, 0]
    body[:, 1, 0] = pm[:, 1] * c12
    body[:, 1, 1] = pm[:, 1] * s12a
    body[:, 2] = -body[:, 0] - body[:, 1]
    cb = np.asarray(cosb, dtype=np.float64)
    sb = np.sqrt(np.maximum(1.0 - cb * cb, 0.0))
    g = np.asarray(gamma, dtype=np.float64)
    Rz = np.zeros((n, 3, 3))
    Rz[:, 0, 0], Rz[:, 0, 1], Rz[:, 1, 0], Rz[:, 1, 1], Rz[:, 2, 2] = np.cos(g), -np.sin(g), np.sin(g), np.cos(g), 1
    Ry = np.zeros((n, 3, 3))
    Ry[:, 0, 0], Ry[:, 0, 2], Ry[:, 1, 1], Ry[:, 2, 0], Ry[:, 2, 2] = cb, sb, 1, -sb, cb
    R = np.einsum("nij,njk->nik", Ry, Rz)
    lab = np.einsum("nij,ndj->ndi", R, body)
    return np.concatenate([E[:, :, None], lab], axis=2)


def _boost_matrix(P):
    """Lorentz boosts (n, 4, 4) into the rest frames of four-vectors P (n, 4)."""
    E = P[:, 0]
    b = P[:, 1:] / E[:, None]
    b2 = np.sum(b * b, axis=1)
    gam = 1.0 / np.sqrt(1.0 - b2)
    L = np.zeros((len(E), 4, 4))
    L[:, 0, 0] = gam
    L[:, 0, 1:] = -gam[:, None] * b
    L[:, 1:, 0] = -gam[:, None] * b
    with np.errstate(invalid="ignore", divide="ignore"):
        bb = np.where(b2[:, None, None] > 0, np.einsum("ni,nj->nij", b, b) / b2[:, None, None], 0.0)
    L[:, 1:, 1:] = np.eye(3) + (gam - 1.0)[:, None, None] * bb
    return L


def angular_factors(p4, channel, J):
    """Y_J^mu (list over mu = +1, -1 of complex arrays) of channel (ab)."""
    a, b, c = _PAIRS[channel]
    pc = p4[:, c, 1:]
    pch = pc / np.linalg.norm(pc, axis=1)[:, None]
    pa_star = np.einsum("nij,nj->ni", _boost_matrix(p4[:, a] + p4[:, b]), p4[:, a])[:, 1:]
    qh = pa_star / np.linalg.norm(pa_star, axis=1)[:, None]
    if J == 0:
        vec = pch
    elif J == 1:
        vec = np.cross(pch, qh)
    elif J == 2:
        T = np.einsum("ni,nj->nij", qh, qh) - np.eye(3) / 3.0
        vec = np.einsum("nij,nj->ni", T, pch)
    else:
        raise ValueError("spin must be 0, 1 or 2")
    return [vec @ e for e in POLARISATIONS]


def _kin_all(events, model):
    s12, s13 = events[0], events[1]
    need = sorted(set(model.channel))
    kin = {ch: kinematics(s12, s13, ch, model) for ch in need}
    if parent_spin(model) == 1:
        p4 = daughter_momenta(s12, s13, events[2], events[3], model)
        for ch in need:
            Js = sorted({J for c, J in zip(model.channel, model.spin) if c == ch})
            kin[ch] = kin[ch] + ({J: angular_factors(p4, ch, J) for J in Js},)
    return kin


def _angular(kin_ch, J, mu, model):
    """The angular factor of helicity term mu: P_J(cos theta) for a spin-0
    parent (one term), Y_J^mu for a spin-1 parent."""
    if parent_spin(model) == 0:
        return legendre(J, kin_ch[2])
    return kin_ch[3][J][mu]


def helicity_amplitudes(kin, model, th, need_grad):
    """z^mu = sum_k c_k a_k^mu for each helicity term and, with need_grad,
    the per-parameter columns dz^mu/dtheta_p (th: floats or duals)."""
    nmu = n_helicities(model)
    z = [0] * nmu
    cols = [[] for _ in range(nmu)]
    for k, (ch, J) in enumerate(zip(model.channel, model.spin)):
        c = th[4 * k] + 1j * th[4 * k + 1]
        M, G = th[4 * k + 2], th[4 * k + 3]
        shape = lineshape_of(model, k)
        if need_grad:
            am = amplitude(kin[ch], ch, J, Dual(M, 1.0, new_tag()), G, model, shape, angular=1.0)
            ag = amplitude(kin[ch], ch, J, M, Dual(G, 1.0, new_tag()), model, shape, angular=1.0)
        for mu in range(nmu):
            ang = _angular(kin[ch], J, mu, model)
            if need_grad:
                a = ang * am.a
                # dz/dRe c = a, dz/dIm c = i a, dz/dM = c da/dM, dz/dGamma = c da/dGamma
                cols[mu] += [a, 1j * a, c * (ang * am.b), c * (ang * ag.b)]
            else:
                a = amplitude(kin[ch], ch, J, M, G, model, shape, angular=ang)
            z[mu] = z[mu] + c * a
    return z, cols


def amplitudes(events, model, theta):
    """List of the K amplitude arrays a_k at the events (fixed M, Gamma);
    spin-0 parent (one helicity term)."""
    if parent_spin(model) != 0:
        raise ValueError("one amplitude per resonance: spin-0 parent only")
    kin = _kin_all(events, model)
    out = []
    for k, (ch, J) in enumerate(zip(model.channel, model.spin)):
        out.append(amplitude(kin[ch], ch, J, theta[4 * k + 2], theta[4 * k + 3], model,
                             lineshape_of(model, k)))
    return out


def intensity(events, model, theta):
    """omega(x) = sum_mu |sum_k c_k a_k^mu(x)|^2 (eq. (1); one term for a
    spin-0 parent)."""
    z, _ = helicity_amplitudes(_kin_all(events, model), model, [float(x) for x in theta], False)
    return sum(np.abs(zm) ** 2 for zm in z)


# --------------------------------------------------------------------------
# Event sums F, G and their derivatives (eq. (5) and its derivatives).
# --------------------------------------------------------------------------
def _event_sums(events, model, th, is_data, need_grad, abs_terms=False):
    """Sum over one event set.

    th: list of 4K parameters (floats, or duals carrying a tangent v).
    Returns S (F for data, G for MC) and, if need_grad, the list of dS/dtheta_p.
    With abs_terms the per-event terms are replaced by their absolute values
    (gives the error scale sum |term|, not a derivative)."""
    z, cols = helicity_amplitudes(_kin_all(events, model), model, th, need_grad)
    w = 0
    for zm in z:
        w = w + dreal(zm) * dreal(zm) + dimag(zm) * dimag(zm)
    term = dlog(w) if is_data else w
    S = fsum(dabs(term) if abs_terms else term)
    grads = []
    if need_grad:
        for p in range(len(cols[0])):
            dw = 0
            for zm, cm in zip(z, cols):
                dw = dw + 2.0 * dreal(dconj(zm) * cm[p])   # d omega / d theta_p
            t = dw / w if is_data else dw
            grads.append(fsum(dabs(t) if abs_terms else t))
    return S, grads


def _chunks(events, size):
    n = len(events[0])
    for i in range(0, max(n, 1), size):
        yield tuple(x[i:i + size] for x in events)


def _sums_chunked(events, model, th, is_data, need_grad, chunk, abs_terms=False):
    parts = [_event_sums(ev, model, th, is_data, need_grad, abs_terms)
             for ev in _chunks(events, chunk) if len(ev[0])]
    if not parts:
        return 0.0, [0.0] * len(th)
    S = _dual_fsum([p[0] for p in parts])
    grads = [_dual_fsum([p[1][j] for p in parts]) for j in range(len(th))] if need_grad else []
    return S, grads


def _dual_fsum(values):
    if any(isinstance(v, Dual) for v in values):
        t = max(_tag(v) for v in values)
        return Dual(_dual_fsum([_parts(v, t)[0] for v in values]),
                    _dual_fsum([_parts(v, t)[1] or 0.0 for v in values]), t)
    return math.fsum(values)


def partials(data, mc, model, theta, v=None, order=1, chunk=100_000):
    """Per-shard partial sums of eq. (5) and their derivatives.

    Returns dict with F, G (floats); dF, dG (arrays, order >= 1);
    HFv, HGv (arrays, when v is given); n_data, n_mc."""
    theta = np.asarray(theta, dtype=np.float64)
    P = theta.size
    need_grad = order >= 1 or v is not None
    if v is not None:
        t = new_tag()
        th = [Dual(float(theta[p]), float(v[p]), t) for p in range(P)]
    else:
        th = [float(x) for x in theta]
    F, dF = _sums_chunked(data, model, th, True, need_grad, chunk)
    G, dG = _sums_chunked(mc, model, th, False, need_grad, chunk)
    out = {"n_data": len(data[0]), "n_mc": len(mc[0])}
    if v is not None:
        out["F"], out["G"] = F.a, G.a
        out["dF"] = np.array([g.a for g in dF])
        out["dG"] = np.array([g.a for g in dG])
        out["HFv"] = np.array([g.b for g in dF])
        out["HGv"] = np.array([g.b for g in dG])
    else:
        out["F"], out["G"] = F, G
        if need_grad:
            out["dF"], out["dG"] = np.array(dF), np.array(dG)
    return out


def combine(parts, n_data=None, n_mc=None, v=None):
    """Combine per-shard partials with eq. (4), (6) and (7) for NLL = -ln L:
        NLL   = -sum F_m + N_D ln( sum G_m / N_MC )
        grad  = -sum dF_m + (N_D / G) sum dG_m
        H v   = -sum HFv_m + (N_D / G) sum HGv_m - (N_D / G^2) dG (dG . v)
    with G = sum_m G_m and dG = sum_m dG_m."""
    if n_data is None:
        n_data = sum(p["n_data"] for p in parts)
    if n_mc is None:
        n_mc = sum(p["n_mc"] for p in parts)
    F = math.fsum(p["F"] for p in parts)
    G = math.fsum(p["G"] for p in parts)
    out = {"nll": -F + n_data * math.log(G / n_mc)}
    if "dF" in parts[0]:
        P = parts[0]["dF"].size
        dF = np.array([math.fsum(p["dF"][j] for p in parts) for j in range(P)])
        dG = np.array([math.fsum(p["dG"][j] for p in parts) for j in range(P)])
        out["grad"] = -dF + (n_data / G) * dG
        if "HFv" in parts[0]:
            HF = np.array([math.fsum(p["HFv"][j] for p in parts) for j in range(P)])
            HG = np.array([math.fsum(p["HGv"][j] for p in parts) for j in range(P)])
            dGv = math.fsum(dG * np.asarray(v))
            out["hv"] = -HF + (n_data / G) * HG - (n_data / (G * G)) * dG * dGv
    return out


# --------------------------------------------------------------------------
# Public NLL / gradient / HVP.
# --------------------------------------------------------------------------
def _nll_from(th, data, mc, model, need_grad, chunk):
    F, dF = _sums_chunked(data, model, th, True, need_grad, chunk)
    G, dG = _sums_chunked(mc, model, th, False, need_grad, chunk)
    nd, nm = len(data[0]), len(mc[0])
    val = -F + nd * dlog(G / nm)
    grads = [-dF[j] + nd * dG[j] / G for j in range(len(dF))]
    return val, grads


def nll(data, mc, model, theta, chunk=100_000):
    """NLL = -ln L of eq. (3); +inf if a resonance mass is below threshold or
    the log's argument is not positive."""
    try:
        with np.errstate(divide="ignore", invalid="ignore"):
            val, _ = _nll_from([float(x) for x in theta], data, mc, model, False, chunk)
    except DomainError:
        return math.inf
    return float(val) if np.isfinite(val) else math.inf


def grad(data, mc, model, theta, chunk=100_000):
    """(NLL, gradient of NLL) with the analytic chain rule, eq. (6)."""
    val, g = _nll_from([float(x) for x in theta], data, mc, model, True, chunk)
    return float(val), np.array([float(x) for x in g])


def hvp(data, mc, model, theta, v, chunk=100_000):
    """(NLL, gradient, H v): the gradient evaluated on dual numbers whose
    tangent is v, so the tangent of the gradient is exactly H v."""
    t = new_tag()
    th = [Dual(float(theta[p]), float(v[p]), t) for p in range(len(theta))]
    val, g = _nll_from(th, data, mc, model, True, chunk)
    return float(val.a), np.array([x.a for x in g]), np.array([x.b for x in g])


def hessian(data, mc, model, theta, chunk=100_000):
    """Full Hessian from P exact Hessian-vector products."""
    P = len(theta)
    H = np.empty((P, P))
    for j in range(P):
        e = np.zeros(P)
        e[j] = 1.0
        H[:, j] = hvp(data, mc, model, theta, e, chunk)[2]
    return H


def grad_scale(data, mc, model, theta, v=None, chunk=100_000):
    """Absolute-sum error scale of the gradient (and of H v if v is given):
        S_p = sum_data |d ln omega/d theta_p| + (N_D/G) sum_MC |d omega/d theta_p|.
    A rounding-error bound for a summed quantity is proportional to it, which
    makes it the right yardstick where the sum itself cancels (near a minimum)."""
    theta = np.asarray(theta, dtype=np.float64)
    P = theta.size
    if v is not None:
        t = new_tag()
        th = [Dual(float(theta[p]), float(v[p]), t) for p in range(P)]
    else:
        th = [float(x) for x in theta]
    _, aF = _sums_chunked(data, model, th, True, True, chunk, abs_terms=True)
    G, _ = _sums_chunked(mc, model, [primal(x) for x in th], False, False, chunk)
    _, aG = _sums_chunked(mc, model, th, False, True, chunk, abs_terms=True)
    nd = len(data[0])
    if v is None:
        return np.array([aF[j] + nd / G * aG[j] for j in range(P)])
    sg = np.array([aF[j].a + nd / G * aG[j].a for j in range(P)])
    sh = np.array([aF[j].b + nd / G * aG[j].b for j in range(P)])
    return sg, sh


def _hvp_abs_sums(events, model, theta, v, is_data):
    """Per-parameter absolute sums over one event set of the pieces of the
    per-event Hessian-vector term (theta a float array, v the direction).
    Data events, d/d theta_p of (d ln w . v) = (H_w v)_p / w - dw_p wdot / w^2:
        returns sum |(H_w v)_p| / w + |dw_p| |wdot| / w^2 and sum |dw_p / w|.
    MC events: returns sum |(H_w v)_p| and sum |dw_p|.
    Also returns the plain sum of w (G for MC)."""
    P = theta.size
    t = new_tag()
    th = [Dual(float(theta[p]), float(v[p]), t) for p in range(P)]
    z, cols = helicity_amplitudes(_kin_all(events, model), model, th, True)
    w = 0
    for zm in z:
        w = w + dreal(zm) * dreal(zm) + dimag(zm) * dimag(zm)   # Dual: (w, wdot)
    hv_abs, g_abs = np.zeros(P), np.zeros(P)
    for p in range(P):
        dw = 0
        for zm, cm in zip(z, cols):
            dw = dw + 2.0 * dreal(dconj(zm) * cm[p])    # Dual: (dw_p, (H_w v)_p)
        if is_data:
            hv_abs[p] = math.fsum(np.abs(dw.b) / w.a + np.abs(dw.a) * np.abs(w.b) / (w.a * w.a))
            g_abs[p] = math.fsum(np.abs(dw.a) / w.a)
        else:
            hv_abs[p] = math.fsum(np.abs(dw.b))
            g_abs[p] = math.fsum(np.abs(dw.a))
    return hv_abs, g_abs, math.fsum(np.ravel(w.a))


def hvp_scale(data, mc, model, theta, v, chunk=100_000):
    """Rounding-error yardstick of the Hessian-vector product, eq. (7) for
    NLL = -ln L:
        H v = -H_F v + (N_D/G) H_G v - (N_D/G^2) dG (dG . v).
    An FP64 evaluation that sums per-event terms makes an error of order
    eps times the sum of the absolute values of what it adds up, so per
    component p the scale is
        sum_data [ |(H_w v)_p| / w + |dw_p| |wdot| / w^2 ]     (first term,
                   both pieces of d/d theta_p of dw.v / w kept apart)
      + (N_D/G) sum_MC |(H_w v)_p|                               (second term)
      + 2 (N_D/G^2) A_p sum_q |v_q| A_q,  A_q = sum_MC |dw_q|    (third term:
                   |dG_p| <= A_p and |dG . v| <= sum_q |v_q| A_q, and each
                   factor carries its own rounding)
    It bounds |H v| componentwise (triangle inequality) and has the units of
    H v, so a component that cancels to ~0 is judged against it."""
    theta = np.asarray(theta, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    P = theta.size
    hF, hG, aG = np.zeros(P), np.zeros(P), np.zeros(P)
    hF_parts, hG_parts, aG_parts, G_parts = [], [], [], []
    for ev in _chunks(data, chunk):
        if len(ev[0]):
            hF_parts.append(_hvp_abs_sums(ev, model, theta, v, True)[0])
    for ev in _chunks(mc, chunk):
        if len(ev[0]):
            h, a, g = _hvp_abs_sums(ev, model, theta, v, False)
            hG_parts.append(h)
            aG_parts.append(a)
            G_parts.append(g)
    for p in range(P):
        hF[p] = math.fsum(x[p] for x in hF_parts)
        hG[p] = math.fsum(x[p] for x in hG_parts)
        aG[p] = math.fsum(x[p] for x in aG_parts)
    G = math.fsum(G_parts)
    nd = len(data[0])
    return hF + (nd / G) * hG + 2.0 * (nd / (G * G)) * aG * math.fsum(np.abs(v) * aG)


# --------------------------------------------------------------------------
# Fixed-lineshape (batched) path: Gram matrix and per-start NLL.
# --------------------------------------------------------------------------
def gram(events, model, theta, chunk=100_000):
    """Gm = A^H A with A[j, k] = a_k(x_j): Gm[l, k] = sum_j conj(a_jl) a_jk."""
    K = len(model.channel)
    acc = np.zeros((K, K), dtype=complex)
    parts = []
    for ev in _chunks(events, chunk):
        if not len(ev[0]):
            continue
        A = np.stack(amplitudes(ev, model, theta), axis=1)
        parts.append(A.conj().T @ A)
    if parts:
        re = np.array([[math.fsum(p[i, j].real for p in parts) for j in range(K)] for i in range(K)])
        im = np.array([[math.fsum(p[i, j].imag for p in parts) for j in range(K)] for i in range(K)])
        acc = re + 1j * im
    return acc


def round_to(x, fmt):
    """Round float64 values to bf16 / fp16 / fp32 (round to nearest even)."""
    x = np.asarray(x, dtype=np.float64)
    if fmt == "f64":
        return x.copy()
    if fmt == "f32":
        return x.astype(np.float32).astype(np.float64)
    if fmt == "f16":
        return x.astype(np.float16).astype(np.float64)
    if fmt == "bf16":
        f = x.astype(np.float32)
        u = f.view(np.uint32).astype(np.uint64)
        lsb = (u >> 16) & 1
        u = ((u + 0x7FFF + lsb) >> 16) << 16
        return u.astype(np.uint32).view(np.float32).astype(np.float64)
    raise ValueError(fmt)


# Sliced FP16 operand format of the batched path: fixed-point slices.
SLICE_BITS = 9
SLICE_COUNT = 4
SLICE_LEVELS = 3   # slice pairs (i, j) with i + j <= 3 are multiplied


def fixed_slices(x, axis, count=SLICE_COUNT, bits=SLICE_BITS):
    """Cut every vector of x along `axis` into `count` integer slices: with E
    the exponent of the vector's largest real or imaginary magnitude
    (|max| < 2^E; E = 0 for a zero vector),
        x 2^(bits - E) = q_0 + 2^-bits q_1 + ... + 2^-(bits (count-1)) q_(count-1) + r,
    each q_s the nearest integer (ties to even) of the running remainder,
    which is then scaled by 2^bits.  Real and imaginary parts are cut
    separately with their common E.  Returns (list of q_s, E with the
    reduced axis kept)."""
    x = np.asarray(x)
    cplx = np.iscomplexobj(x)
    mag = np.maximum(np.abs(x.real), np.abs(x.imag)) if cplx else np.abs(x)
    m = np.max(mag, axis=axis, keepdims=True)
    E = np.where(m > 0, np.frexp(m)[1], 0)

    def cut(v):
        v = v * np.ldexp(1.0, bits - E)
        out = []
        for _ in range(count):
            q = np.rint(v)
            out.append(q)
            v = (v - q) * 2.0 ** bits
        return out

    if cplx:
        return [r + 1j * i for r, i in zip(cut(x.real), cut(x.imag))], E
    return cut(x), E


def sliced_product(A, C):
    """A @ C as the sliced FP16 format defines it: A cut per row, C per
    column, and only the slice pairs i + j <= SLICE_LEVELS multiplied:
        Z = 2^(E_row + G_col - 2 bits) sum_{i+j<=L} 2^(-bits (i+j)) q^A_i @ q^C_j.
    Every slice product is an integer dot product, exact in FP64, and the
    weighted sum spans fewer than 53 bits, so Z carries no rounding beyond
    the format's own."""
    qa, Ea = fixed_slices(A, axis=1)
    qc, Gc = fixed_slices(C, axis=0)
    Z = np.zeros((A.shape[0], C.shape[1]), dtype=complex)
    for i in range(SLICE_COUNT):
        for j in range(SLICE_COUNT):
            if i + j <= SLICE_LEVELS:
                Z += np.ldexp(1.0, -SLICE_BITS * (i + j)) * (qa[i] @ qc[j])
    return Z * np.ldexp(1.0, Ea + Gc - 2 * SLICE_BITS)


def nll_batched(data, mc, model, theta, C, fmt="f64", chunk=50_000, parts=False):
    """NLL_b = -sum_data ln |(A_D c_b)_i|^2 + N_D ln( c_b^H Gm c_b / N_MC )
    for every column c_b of the complex K x B matrix C (M, Gamma frozen at
    theta).  With fmt in ('f32', 'bf16', 'f16') the operands A and C are
    first rounded to that format (the contraction itself stays FP64), which
    isolates the error due to operand rounding; with fmt = 'f16s' the
    products are the sliced format's (sliced_product).  With parts=True
    returns (F_b, G_b)."""
    C = np.asarray(C, dtype=complex)
    B = C.shape[1]
    if fmt == "f16s":
        def zmat(ev):
            return sliced_product(np.stack(amplitudes(ev, model, theta), axis=1), C)
    else:
        Cr = round_to(C.real, fmt) + 1j * round_to(C.imag, fmt)

        def zmat(ev):
            A = np.stack(amplitudes(ev, model, theta), axis=1)
            return (round_to(A.real, fmt) + 1j * round_to(A.imag, fmt)) @ Cr

    Fp, Gp = [], []
    for ev in _chunks(data, chunk):
        if len(ev[0]):
            Z = zmat(ev)
            Fp.append(np.log(Z.real ** 2 + Z.imag ** 2))
    for ev in _chunks(mc, chunk):
        if len(ev[0]):
            Z = zmat(ev)
            Gp.append(Z.real ** 2 + Z.imag ** 2)
    F = np.array([math.fsum(np.concatenate([p[:, b] for p in Fp])) for b in range(B)])
    G = np.array([math.fsum(np.concatenate([p[:, b] for p in Gp])) for b in range(B)])
    if parts:
        return F, G
    nd, nm = len(data[0]), len(mc[0])
    return -F + nd * np.log(G / nm)


# --------------------------------------------------------------------------
# At the minimum: fit fractions (Table 1 quotes F_i per resonance without a
# definition; read here as the ratio of phase-space integrals, estimated by
# the MC sample) and the interference terms.
# --------------------------------------------------------------------------
def fraction_matrix(mc, model, theta, chunk=100_000):
    """K x K matrix Phi with, for y_k = c_k a_k and D = sum_MC |sum_k y_k|^2,
        Phi[k, k] = sum_MC |y_k|^2 / D                     (fit fraction F_k)
        Phi[k, l] = sum_MC 2 Re(conj(y_k) y_l) / D, k < l  (interference)
    and zero below the diagonal.  Per chunk the sums over events are one
    matrix product Y^H Y (Y: events x K); chunk sums are added with
    math.fsum."""
    theta = np.asarray(theta, dtype=np.float64)
    K = len(model.channel)
    m_parts, d_parts = [], []
    for ev in _chunks(mc, chunk):
        if not len(ev[0]):
            continue
        a = amplitudes(ev, model, theta)
        Y = np.stack([(theta[4 * k] + 1j * theta[4 * k + 1]) * a[k] for k in range(K)], axis=1)
        m_parts.append(Y.conj().T @ Y)
        d_parts.append(math.fsum(np.abs(Y.sum(axis=1)) ** 2))
    D = math.fsum(d_parts)
    Phi = np.zeros((K, K))
    for k in range(K):
        Phi[k, k] = math.fsum(m[k, k].real for m in m_parts) / D
        for l in range(k + 1, K):
            Phi[k, l] = 2.0 * math.fsum(m[k, l].real for m in m_parts) / D
    return Phi


def fit_fractions(mc, model, theta, chunk=100_000):
    """F_k = sum_MC |c_k a_k|^2 / sum_MC |sum_l c_l a_l|^2 and the gradients
    dF_k/dtheta (K x P).  Chain rule per event: d|y|^2 = 2 Re(conj(y) dy)
    with dy/dRe c = a, dy/dIm c = i a, dy/dM = c da/dM, dy/dGamma = c da/dGamma
    (the a-derivatives by dual numbers); then
    dF_k = dN_k / D - N_k dD / D^2.  Event sums by math.fsum per chunk, chunk
    sums by math.fsum."""
    if parent_spin(model) != 0:
        raise ValueError("fit fractions of one helicity term: spin-0 parent only")
    theta = np.asarray(theta, dtype=np.float64)
    K = len(model.channel)
    P = 4 * K
    n_parts = [[] for _ in range(K)]
    dn_parts = [[] for _ in range(P)]   # entry 4k + i: d N_k / d theta_{4k+i}
    d_parts = []
    dd_parts = [[] for _ in range(P)]
    for ev in _chunks(mc, chunk):
        if not len(ev[0]):
            continue
        kin = _kin_all(ev, model)
        y, cols = [], []
        for k, (ch, J) in enumerate(zip(model.channel, model.spin)):
            c = theta[4 * k] + 1j * theta[4 * k + 1]
            M, G = theta[4 * k + 2], theta[4 * k + 3]
            shape = lineshape_of(model, k)
            am = amplitude(kin[ch], ch, J, Dual(M, 1.0, new_tag()), G, model, shape)
            ag = amplitude(kin[ch], ch, J, M, Dual(G, 1.0, new_tag()), model, shape)
            a = am.a
            y.append(c * a)
            cols.append([a, 1j * a, c * am.b, c * ag.b])
        z = sum(y)
        d_parts.append(math.fsum(np.abs(z) ** 2))
        for k in range(K):
            n_parts[k].append(math.fsum(np.abs(y[k]) ** 2))
            for i in range(4):
                dn_parts[4 * k + i].append(math.fsum(2.0 * (np.conj(y[k]) * cols[k][i]).real))
                dd_parts[4 * k + i].append(math.fsum(2.0 * (np.conj(z) * cols[k][i]).real))
    D = math.fsum(d_parts)
    dD = np.array([math.fsum(t) for t in dd_parts])
    F = np.zeros(K)
    dF = np.zeros((K, P))
    for k in range(K):
        N = math.fsum(n_parts[k])
        F[k] = N / D
        dN = np.zeros(P)
        for i in range(4):
            dN[4 * k + i] = math.fsum(dn_parts[4 * k + i])
        dF[k] = dN / D - N * dD / (D * D)
    return F, dF


# --------------------------------------------------------------------------
# Reference fit: the paper's optimiser (scipy Newton-CG, Sec. 3).
# --------------------------------------------------------------------------
def newton_cg_fit(data, mc, model, theta0, xtol=1e-8, maxiter=200, chunk=100_000):
    """scipy.optimize.minimize(method='Newton-CG') on the oracle's NLL with
    its analytic gradient and exact Hessian-vector product."""
    from scipy.optimize import minimize

    cache = {}

    def f(th):
        key = th.tobytes()
        if key not in cache:
            cache.clear()
            cache[key] = grad(data, mc, model, th, chunk)
        return cache[key][0]

    def jac(th):
        f(th)
        return cache[th.tobytes()][1]

    def hessp(th, p):
        return hvp(data, mc, model, th, p, chunk)[2]

    return minimize(f, np.asarray(theta0, dtype=np.float64), jac=jac, hessp=hessp,
                    method="Newton-CG", options={"xtol": xtol, "maxiter": maxiter})


def bfgs_fit(data, mc, model, theta0, gtol=1e-5, maxiter=400, chunk=100_000):
    """scipy.optimize.minimize(method='BFGS') on the oracle's NLL with its
    analytic gradient: the gradient-only quasi-Newton comparator of the
    paper's Sec. 3 (Migrad with AD gradients there)."""
    from scipy.optimize import minimize

    cache = {}

    def f(th):
        key = th.tobytes()
        if key not in cache:
            cache.clear()
            try:
                cache[key] = grad(data, mc, model, th, chunk)
            except DomainError:
                # a trial step with a mass below threshold: +inf, which the
                # line search rejects (the NLL is +inf there, as in nll())
                cache[key] = (math.inf, np.zeros(len(th)))
        return cache[key][0]

    def jac(th):
        f(th)
        return cache[th.tobytes()][1]

    return minimize(f, np.asarray(theta0, dtype=np.float64), jac=jac, method="BFGS",
                    options={"gtol": gtol, "maxiter": maxiter})

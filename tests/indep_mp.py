"""Independent 50-digit implementation of the likelihood, used only to pin
the FP64 oracle on tiny inputs.

It deliberately takes a different route from the oracle wherever one exists:
  * kinematics from explicit four-vectors and Lorentz boosts (not from the
    closed-form helicity-angle expression);
  * Blatt-Weisskopf factors from spherical Hankel functions,
    F_J(z)^-2 = z^J |x h_J(x)|^2 with x = sqrt(z) (mpmath Bessel functions);
  * Legendre polynomials from mpmath;
  * the breakup momentum at the pole from the product form
    sqrt((M^2-(ma+mb)^2)(M^2-(ma-mb)^2)) / (2M);
  * derivatives by mpmath numerical differentiation at high precision.
"""

import mpmath as mp

PAIRS = ((0, 1, 2), (0, 2, 1), (1, 2, 0))


def _vec(E, px, py, pz):
    return [mp.mpf(E), mp.mpf(px), mp.mpf(py), mp.mpf(pz)]


def _add(p, q):
    return [p[i] + q[i] for i in range(4)]


def _dot(p, q):
    return p[0] * q[0] - p[1] * q[1] - p[2] * q[2] - p[3] * q[3]


def _boost_to_rest(p, P):
    """Boost four-vector p into the rest frame of four-vector P."""
    m = mp.sqrt(_dot(P, P))
    b = [P[1] / P[0], P[2] / P[0], P[3] / P[0]]
    b2 = b[0] ** 2 + b[1] ** 2 + b[2] ** 2
    if b2 == 0:
        return list(p)
    g = P[0] / m
    bp = b[0] * p[1] + b[1] * p[2] + b[2] * p[3]
    E = g * (p[0] - bp)
    k = (g - 1) * bp / b2 - g * p[0]
    return [E, p[1] + k * b[0], p[2] + k * b[1], p[3] + k * b[2]]


def four_vectors(s12, s13, M, m):
    """Daughter four-momenta for invariants (s12, s13), built in the (12)
    rest frame with particle 3 along -z and 1, 2 in the xz plane."""
    s12, s13 = mp.mpf(s12), mp.mpf(s13)
    m1, m2, m3 = (mp.mpf(x) for x in m)
    M = mp.mpf(M)
    rs = mp.sqrt(s12)
    E1 = (s12 + m1 ** 2 - m2 ** 2) / (2 * rs)
    E2 = rs - E1
    E3 = (M ** 2 - s12 - m3 ** 2) / (2 * rs)
    p1 = mp.sqrt(E1 ** 2 - m1 ** 2)
    p3 = mp.sqrt(E3 ** 2 - m3 ** 2)
    # p3 = (E3, 0, 0, -p3); p1 = (E1, p1 sin a, 0, p1 cos a); solve cos a from s13
    cos_a = (s13 - m1 ** 2 - m3 ** 2 - 2 * E1 * E3) / (2 * p1 * p3)
    sin_a = mp.sqrt(1 - cos_a ** 2)
    v1 = _vec(E1, p1 * sin_a, 0, p1 * cos_a)
    v2 = _vec(E2, -p1 * sin_a, 0, -p1 * cos_a)
    v3 = _vec(E3, 0, 0, -p3)
    return [v1, v2, v3]


def channel_kin(vecs, ch):
    """(s_ab, q, cos th) from four-vectors: boost into the (ab) frame; q is
    |p_a| there and th the angle between p_a and -p_c."""
    a, b, c = PAIRS[ch]
    Pab = _add(vecs[a], vecs[b])
    pa = _boost_to_rest(vecs[a], Pab)
    pc = _boost_to_rest(vecs[c], Pab)
    na = mp.sqrt(pa[1] ** 2 + pa[2] ** 2 + pa[3] ** 2)
    nc = mp.sqrt(pc[1] ** 2 + pc[2] ** 2 + pc[3] ** 2)
    cos = -(pa[1] * pc[1] + pa[2] * pc[2] + pa[3] * pc[3]) / (na * nc)
    return _dot(Pab, Pab), na, cos


def sph_hankel_abs2(J, x):
    """|h_J^(1)(x)|^2 from half-integer Bessel functions."""
    f = mp.sqrt(mp.pi / (2 * x))
    jn = f * mp.besselj(J + mp.mpf(1) / 2, x)
    yn = f * mp.bessely(J + mp.mpf(1) / 2, x)
    return jn ** 2 + yn ** 2


def bw_factor_sq(J, z):
    """F_J(z)^2 = 1 / (z^J |x h_J(x)|^2), x = sqrt(z)."""
    if J == 0:
        return mp.mpf(1)
    x = mp.sqrt(z)
    return 1 / (z ** J * (x * x) * sph_hankel_abs2(J, x))


def amp(kin, ch, J, M, G, m, r, width_mode=0, ang=None):
    s, q, cos = kin
    a, b, _ = PAIRS[ch]
    ma, mb = mp.mpf(m[a]), mp.mpf(m[b])
    q0 = mp.sqrt((M ** 2 - (ma + mb) ** 2) * (M ** 2 - (ma - mb) ** 2)) / (2 * M)
    r = mp.mpf(r)
    ratio = mp.sqrt(bw_factor_sq(J, (q * r) ** 2) / bw_factor_sq(J, (q0 * r) ** 2))
    if width_mode == 0:
        gs = G * (q / q0) ** (2 * J + 1) * (M / mp.sqrt(s)) * ratio ** 2
    else:
        gs = G
    a_ = mp.legendre(J, cos) if ang is None else ang
    return a_ * ratio / (M ** 2 - s - 1j * M * gs)


def _unit3(v):
    n = mp.sqrt(v[0] ** 2 + v[1] ** 2 + v[2] ** 2)
    return [x / n for x in v]


def spin1_omega(s12, s13, cosb, gam, channel, spin, th, M, m, r):
    """sum over mu = +1, -1 of |sum_k c_k Y_J^mu a_k|^2 for a vector parent:
    four-vectors from the (12) frame boosted to the parent rest frame, turned
    to the reference plane (p_1 along x, p_2 in the upper x-y half plane),
    rotated by R_y(beta) R_z(gamma); Y from the bachelor direction and the
    direction of a boosted into the pair's rest frame."""
    vecs = four_vectors(s12, s13, M, m)
    P = _add(_add(vecs[0], vecs[1]), vecs[2])
    vp = [_boost_to_rest(v, P) for v in vecs]
    e1 = _unit3(vp[0][1:])
    d = sum(vp[1][1 + i] * e1[i] for i in range(3))
    e2 = _unit3([vp[1][1 + i] - d * e1[i] for i in range(3)])
    e3 = [e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]]
    cb = mp.mpf(cosb)
    sb = mp.sqrt(1 - cb * cb)
    cg, sg = mp.cos(mp.mpf(gam)), mp.sin(mp.mpf(gam))
    lab = []
    for v in vp:
        x, y, z = (sum(v[1 + i] * e[i] for i in range(3)) for e in (e1, e2, e3))
        xr, yr = x * cg - y * sg, x * sg + y * cg          # R_z(gamma)
        lab.append([v[0], xr * cb + z * sb, yr, -xr * sb + z * cb])   # R_y(beta)
    zmu = [mp.mpc(0), mp.mpc(0)]
    for k, (ch, J) in enumerate(zip(channel, spin)):
        a, b, c = PAIRS[ch]
        pc = _unit3(lab[c][1:])
        qa = _unit3(_boost_to_rest(lab[a], _add(lab[a], lab[b]))[1:])
        if J == 0:
            vv = pc
        elif J == 1:
            vv = [pc[1] * qa[2] - pc[2] * qa[1], pc[2] * qa[0] - pc[0] * qa[2], pc[0] * qa[1] - pc[1] * qa[0]]
        else:
            qp = sum(qa[i] * pc[i] for i in range(3))
            vv = [qa[i] * qp - pc[i] / 3 for i in range(3)]
        ys = (-(vv[0] + 1j * vv[1]) / mp.sqrt(2), (vv[0] - 1j * vv[1]) / mp.sqrt(2))
        kin = channel_kin(vecs, ch)
        cpl = mp.mpf(th[4 * k]) + 1j * mp.mpf(th[4 * k + 1])
        for mu in range(2):
            zmu[mu] += cpl * amp(kin, ch, J, mp.mpf(th[4 * k + 2]), mp.mpf(th[4 * k + 3]), m, r,
                                 0, ys[mu])
    return abs(zmu[0]) ** 2 + abs(zmu[1]) ** 2


class TinyNLL:
    """NLL(theta) at high precision over a handful of events."""

    def __init__(self, data, mc, channel, spin, M, m, r, width_mode=0):
        self.channel, self.spin, self.m, self.r = channel, spin, m, r
        self.width_mode = width_mode
        self.kin_d = [self._kin(x, y, M, m) for x, y in zip(*data)]
        self.kin_m = [self._kin(x, y, M, m) for x, y in zip(*mc)]

    def _kin(self, s12, s13, M, m):
        vecs = four_vectors(s12, s13, M, m)
        return {ch: channel_kin(vecs, ch) for ch in set(self.channel)}

    def omega(self, kin, th):
        z = 0
        for k, (ch, J) in enumerate(zip(self.channel, self.spin)):
            c = th[4 * k] + 1j * th[4 * k + 1]
            z += c * amp(kin[ch], ch, J, th[4 * k + 2], th[4 * k + 3], self.m, self.r,
                         self.width_mode)
        return abs(z) ** 2

    def __call__(self, *th):
        th = [mp.mpf(x) for x in th]
        F = mp.fsum(mp.log(self.omega(k, th)) for k in self.kin_d)
        G = mp.fsum(self.omega(k, th) for k in self.kin_m)
        nd, nm = len(self.kin_d), len(self.kin_m)
        return -F + nd * mp.log(G / nm)

"""Seeded event generators over the Dalitz plane (s12, s13).

Only phase-space geometry lives here (the allowed region of a three-body
decay, from energy-momentum conservation in a two-body rest frame).  No
amplitude or likelihood is computed: `accept_reject` takes the intensity as
a caller-supplied function.
"""

import numpy as np

from .workloads import PARENT_MASS, DAUGHTER_MASSES, CHANNEL_PAIRS


def _sum_sq(parent=PARENT_MASS, masses=DAUGHTER_MASSES):
    return parent * parent + sum(m * m for m in masses)


def pair_range(s_ab, a, b, c, parent=PARENT_MASS, masses=DAUGHTER_MASSES):
    """Allowed range of s_ac at fixed s_ab (daughter indices a, b, c).

    Works in the (ab) rest frame: the energies of a and of the bachelor c are
    fixed by s_ab, and s_ac is extremal when their momenta are parallel or
    antiparallel."""
    s_ab = np.asarray(s_ab, dtype=np.float64)
    ma, mb, mc = masses[a], masses[b], masses[c]
    rs = np.sqrt(s_ab)
    ea = (s_ab - mb * mb + ma * ma) / (2.0 * rs)
    ec = (parent * parent - s_ab - mc * mc) / (2.0 * rs)
    pa = np.sqrt(np.maximum(ea * ea - ma * ma, 0.0))
    pc = np.sqrt(np.maximum(ec * ec - mc * mc, 0.0))
    e2 = (ea + ec) ** 2
    return e2 - (pa + pc) ** 2, e2 - (pa - pc) ** 2


def s13_range(s12, parent=PARENT_MASS, masses=DAUGHTER_MASSES):
    return pair_range(s12, 0, 1, 2, parent, masses)


def bounding_box(parent=PARENT_MASS, masses=DAUGHTER_MASSES):
    m1, m2, m3 = masses
    return ((m1 + m2) ** 2, (parent - m3) ** 2), ((m1 + m3) ** 2, (parent - m2) ** 2)


def inside(s12, s13, parent=PARENT_MASS, masses=DAUGHTER_MASSES):
    (lo12, hi12), _ = bounding_box(parent, masses)
    ok = (s12 >= lo12) & (s12 <= hi12)
    lo, hi = s13_range(np.clip(s12, lo12, hi12), parent, masses)
    return ok & (s13 >= lo) & (s13 <= hi)


def uniform_phase_space(n, rng, parent=PARENT_MASS, masses=DAUGHTER_MASSES,
                        batch=1 << 20):
    """n events uniform in the Dalitz plane (uniform phase-space density):
    uniform points in the bounding box, rejected outside the allowed region."""
    (a0, a1), (b0, b1) = bounding_box(parent, masses)
    out12, out13, got = [], [], 0
    while got < n:
        x = rng.uniform(a0, a1, batch)
        y = rng.uniform(b0, b1, batch)
        m = inside(x, y, parent, masses)
        x, y = x[m], y[m]
        out12.append(x)
        out13.append(y)
        got += x.size
    return np.concatenate(out12)[:n].copy(), np.concatenate(out13)[:n].copy()


def mirror_symmetric(s12, s13, parent=PARENT_MASS, masses=DAUGHTER_MASSES):
    """Append to each event its mirror image at fixed s12: s13 reflected about
    the middle of its allowed range.  For channel (12) this is the reflection
    of the helicity angle, cos(theta) -> -cos(theta), because s13 is linear in
    cos(theta) at fixed s12."""
    lo, hi = s13_range(s12, parent, masses)
    return np.concatenate([s12, s12]), np.concatenate([s13, lo + hi - s13])


def midpoint_line_s12(n, parent=PARENT_MASS, masses=DAUGHTER_MASSES):
    """n midpoints of a uniform grid over the full s12 range, each placed at
    the middle of its allowed s13 interval (so every point is physical)."""
    (a0, a1), _ = bounding_box(parent, masses)
    h = (a1 - a0) / n
    s12 = a0 + h * (np.arange(n) + 0.5)
    lo, hi = s13_range(s12, parent, masses)
    return s12, 0.5 * (lo + hi), h


def midpoint_grid(n12, n13, parent=PARENT_MASS, masses=DAUGHTER_MASSES):
    """Midpoints of an n12 x n13 grid over the bounding box that fall inside
    the Dalitz region: a deterministic stand-in for uniform MC whose
    integration error is far below the Monte-Carlo noise of a random sample."""
    (a0, a1), (b0, b1) = bounding_box(parent, masses)
    x = a0 + (a1 - a0) * (np.arange(n12) + 0.5) / n12
    y = b0 + (b1 - b0) * (np.arange(n13) + 0.5) / n13
    X, Y = np.meshgrid(x, y, indexing="ij")
    X, Y = X.ravel(), Y.ravel()
    m = inside(X, Y, parent, masses)
    return X[m].copy(), Y[m].copy()


def _to_s12_s13(channel, s_ab, s_ac, parent=PARENT_MASS, masses=DAUGHTER_MASSES):
    """Map (s_ab, s_ac) of a channel back to (s12, s13)."""
    if channel == 0:      # (12), c = 3, s_ac = s13
        return s_ab, s_ac
    if channel == 1:      # (13), c = 2, s_ac = s12
        return s_ac, s_ab
    # (23), c = 1, s_ac = s21 = s12; s13 from the invariant sum
    return s_ac, _sum_sq(parent, masses) - s_ab - s_ac


def resonant_like(n, channel, theta, rng, flat_fraction=0.2,
                  parent=PARENT_MASS, masses=DAUGHTER_MASSES):
    """Data-like events with resonance bands, drawn without any amplitude.

    A fraction `flat_fraction` is uniform phase space.  The rest is split
    evenly over the resonances: resonance k places s_ab of its channel on a
    Cauchy distribution of location M_k^2 and scale M_k Gamma_k (truncated to
    the kinematic range), and the other Dalitz variable uniformly inside the
    allowed interval.  This reproduces the structure of resonant data (bands
    at the resonance masses, their widths) for throughput workloads."""
    K = len(channel)
    comp = np.where(rng.uniform(size=n) < flat_fraction, -1, rng.integers(0, K, n))
    s12 = np.empty(n)
    s13 = np.empty(n)
    m_flat = comp < 0
    nf = int(m_flat.sum())
    if nf:
        s12[m_flat], s13[m_flat] = uniform_phase_space(nf, rng, parent, masses)
    for k in range(K):
        sel = comp == k
        nk = int(sel.sum())
        if not nk:
            continue
        a, b, c = CHANNEL_PAIRS[channel[k]]
        M, G = theta[4 * k + 2], theta[4 * k + 3]
        lo = (masses[a] + masses[b]) ** 2
        hi = (parent - masses[c]) ** 2
        loc, scale = M * M, M * G
        flo = np.arctan((lo - loc) / scale)
        fhi = np.arctan((hi - loc) / scale)
        s_ab = loc + scale * np.tan(rng.uniform(flo, fhi, nk))
        s_ab = np.clip(s_ab, lo * (1 + 1e-12), hi * (1 - 1e-12))
        r0, r1 = pair_range(s_ab, a, b, c, parent, masses)
        s_ac = r0 + (r1 - r0) * rng.uniform(size=nk)
        x, y = _to_s12_s13(channel[k], s_ab, s_ac, parent, masses)
        s12[sel], s13[sel] = x, y
    return s12, s13


def accept_reject(n, intensity, rng, parent=PARENT_MASS, masses=DAUGHTER_MASSES,
                  scan=1_000_000, batch=1 << 18, safety=1.2):
    """n events distributed as `intensity(s12, s13)` over phase space.

    The ceiling is `safety` times the largest intensity over a uniform scan;
    if any trial exceeds it, sampling restarts with twice the ceiling (the
    result stays a deterministic function of the generator's seed)."""
    x, y = uniform_phase_space(scan, rng, parent, masses)
    wmax = safety * float(np.max(intensity(x, y)))
    while True:
        out12, out13, got, bad = [], [], 0, False
        while got < n:
            x, y = uniform_phase_space(batch, rng, parent, masses)
            w = intensity(x, y)
            if np.any(w > wmax):
                bad = True
                break
            keep = rng.uniform(0.0, wmax, batch) < w
            out12.append(x[keep])
            out13.append(y[keep])
            got += int(keep.sum())
        if not bad:
            return np.concatenate(out12)[:n].copy(), np.concatenate(out13)[:n].copy()
        wmax *= 2.0


def uniform_orientation(n: int, rng: np.random.Generator):
    """Orientation of n decays, uniform over rotations: (cos beta, gamma)
    with cos beta ~ U[-1, 1] and gamma ~ U[0, 2 pi) (the third Euler angle,
    a rotation about the polarisation axis, does not enter a helicity-summed
    intensity)."""
    return rng.uniform(-1.0, 1.0, n), rng.uniform(0.0, 2.0 * np.pi, n)

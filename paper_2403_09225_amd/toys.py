"""Events drawn from the model on the GPU (toy data).

Candidates are uniform over the Dalitz plane (s12, s13) -- the phase-space
density of a three-body decay is flat in these variables -- and are kept
with probability omega(x) / omega_max, omega from the library's per-event
intensity (eq. (1)).  The ceiling omega_max is a safety factor times the
largest intensity over a uniform scan; if a later candidate exceeds it, the
draw restarts with twice the ceiling, so the sample is always distributed
exactly as omega and stays a deterministic function of the generator seed.
"""

import torch

from .api import Likelihood, PARENT_MASS, DAUGHTER_MASSES


def _s13_range(s12, parent, masses):
    """Allowed s13 at fixed s12: in the (12) rest frame the energies of
    daughter 1 and of the bachelor 3 are fixed by s12, and s13 is extremal
    when their momenta are parallel or antiparallel."""
    m1, m2, m3 = masses
    rs = torch.sqrt(s12)
    e1 = (s12 - m2 * m2 + m1 * m1) / (2.0 * rs)
    e3 = (parent * parent - s12 - m3 * m3) / (2.0 * rs)
    p1 = torch.sqrt(torch.clamp(e1 * e1 - m1 * m1, min=0.0))
    p3 = torch.sqrt(torch.clamp(e3 * e3 - m3 * m3, min=0.0))
    e2 = (e1 + e3) ** 2
    return e2 - (p1 + p3) ** 2, e2 - (p1 - p3) ** 2


def uniform_dalitz(n, gen, parent=PARENT_MASS, masses=DAUGHTER_MASSES, device="cuda"):
    """n events uniform over the Dalitz plane (FP64 on `device`)."""
    m1, m2, m3 = masses
    lo12, hi12 = (m1 + m2) ** 2, (parent - m3) ** 2
    lo13, hi13 = (m1 + m3) ** 2, (parent - m2) ** 2
    out12, out13, got = [], [], 0
    while got < n:
        m = max(1024, int(1.25 * (n - got)) + 1024)
        x = lo12 + (hi12 - lo12) * torch.rand(m, dtype=torch.float64, generator=gen, device=device)
        y = lo13 + (hi13 - lo13) * torch.rand(m, dtype=torch.float64, generator=gen, device=device)
        a, b = _s13_range(x, parent, masses)
        keep = (y >= a) & (y <= b)
        out12.append(x[keep])
        out13.append(y[keep])
        got += int(keep.sum())
    return torch.cat(out12)[:n], torch.cat(out13)[:n]


class ToyGenerator:
    """Draws events from |sum_k c_k a_k|^2 for a fixed resonance layout."""

    def __init__(self, channel, spin, parent=PARENT_MASS, masses=DAUGHTER_MASSES,
                 batch=1 << 21, scan=1 << 20, safety=1.5, device="cuda", **model_kw):
        self.lik = Likelihood(channel, spin, parent_mass=parent, masses=masses, device=device,
                              **model_kw)
        self.parent, self.masses = parent, masses
        self.batch, self.scan, self.safety = batch, scan, safety
        self.device = device

    def intensity(self, s12, s13, theta):
        self.lik.bind(s12, s13, s12[:1], s13[:1])
        return self.lik.intensity(theta, "data")

    def draw(self, theta, n, gen):
        """n events distributed as omega(x; theta), as (s12, s13) device tensors."""
        theta = torch.as_tensor(theta, dtype=torch.float64, device=self.device)
        x, y = uniform_dalitz(self.scan, gen, self.parent, self.masses, self.device)
        wmax = self.safety * float(self.intensity(x, y, theta).max())
        if not (wmax > 0.0) or wmax == float("inf"):
            raise ValueError("intensity is not positive and finite over the scan")
        while True:
            out12, out13, got, bad = [], [], 0, False
            while got < n:
                x, y = uniform_dalitz(self.batch, gen, self.parent, self.masses, self.device)
                w = self.intensity(x, y, theta)
                if bool((w > wmax).any()):
                    bad = True
                    break
                u = wmax * torch.rand(self.batch, dtype=torch.float64, generator=gen,
                                      device=self.device)
                keep = u < w
                out12.append(x[keep])
                out13.append(y[keep])
                got += int(keep.sum())
            if not bad:
                return torch.cat(out12)[:n].contiguous(), torch.cat(out13)[:n].contiguous()
            wmax *= 2.0

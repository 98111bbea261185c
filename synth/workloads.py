"""Workload definitions for the Dalitz-plot likelihood: decay masses,
resonance layouts and seeded parameter draws.

The paper's own test model (psi(3686) -> phi K+ K-, Table 1 and Sec. 3)
cannot be rebuilt: its couplings and phases are omitted and its sample is
not published.  These workloads stand in for it: a spin-0 parent of mass
1.865 GeV decaying to three distinguishable pseudoscalars (0.494, 0.140,
0.140 GeV), with K resonances in the three two-body channels.

Parameter vector layout (k-major, four reals per resonance):
    theta[4k + 0] = Re c_k, theta[4k + 1] = Im c_k,
    theta[4k + 2] = M_k,    theta[4k + 3] = Gamma_k.
"""

from dataclasses import dataclass, field
from typing import List

import numpy as np

PARENT_MASS = 1.865
DAUGHTER_MASSES = (0.494, 0.140, 0.140)
R_BARRIER = 3.0  # Blatt-Weisskopf radius, GeV^-1

# Coupled second channel of a Flatte (scalar) resonance: a K Kbar pair and
# the coupling ratio g_2 / g_1, values of the size quoted for f0(980) fits;
# with f0-like M = 0.965 GeV and g_1 = 0.165 GeV^2 in the (23) channel (the
# pi pi pair of these daughters) the K Kbar threshold (0.975 GeV^2) lies
# inside the Dalitz region.
FLATTE_MASSES = (0.493677, 0.493677)
FLATTE_RATIO = 4.21
FLATTE_F0 = (0.965, 0.165)   # (M, g_1)

# Channel c -> (a, b, bachelor) as 0-based daughter indices:
#   0 = (12) with bachelor 3, 1 = (13) with bachelor 2, 2 = (23) with bachelor 1.
CHANNEL_PAIRS = ((0, 1, 2), (0, 2, 1), (1, 2, 0))

BASE_SEED = 240309225

# Random streams per workload.
STREAM_MODEL, STREAM_MC, STREAM_DATA, STREAM_TEST = 0, 1, 2, 3


# Workload names and the seed index of each (seeds are BASE_SEED + 100 *
# index + stream, so every workload draws from its own streams).
SEED_INDEX = {"k2_fit": 0, "k12_hvp": 1, "k20_batched": 2, "k30_diff": 3, "k12_toys": 4}


def rng_for(name: str, stream: int) -> np.random.Generator:
    """Seeded generator for workload `name` and random stream `stream`."""
    return np.random.Generator(np.random.PCG64(BASE_SEED + 100 * SEED_INDEX[name] + stream))


def threshold(channel: int) -> float:
    a, b, _ = CHANNEL_PAIRS[channel]
    return DAUGHTER_MASSES[a] + DAUGHTER_MASSES[b]


def resonance_layout(n_res: int):
    """Channel and spin of resonance k: channel = k mod 3, J = floor(k/3) mod 3.

    With K >= 9 every (channel, J) pair occurs, which is the largest event
    stream (3 invariant masses, 6 angular planes, 9 width planes)."""
    ch = [k % 3 for k in range(n_res)]
    spin = [(k // 3) % 3 for k in range(n_res)]
    return ch, spin


def draw_theta(channel, spin, rng: np.random.Generator,
               m_lo=0.6, m_hi=1.6, g_lo=0.03, g_hi=0.3,
               c_lo=0.2, c_hi=1.0) -> np.ndarray:
    """Random parameters: M ~ U[m_lo, m_hi] (redrawn while below the channel
    threshold + 20 MeV), Gamma ~ U[g_lo, g_hi], |c| ~ U(c_lo, c_hi),
    arg c ~ U(0, 2 pi)."""
    n = len(channel)
    th = np.empty(4 * n)
    for k in range(n):
        thr = threshold(channel[k]) + 0.02
        m = rng.uniform(m_lo, m_hi)
        while m < thr:
            m = rng.uniform(m_lo, m_hi)
        g = rng.uniform(g_lo, g_hi)
        mag = rng.uniform(c_lo, c_hi)
        ph = rng.uniform(0.0, 2.0 * np.pi)
        th[4 * k:4 * k + 4] = (mag * np.cos(ph), mag * np.sin(ph), m, g)
    return th


@dataclass
class Workload:
    """One synthetic workload: model layout, true parameters and sizes."""
    key: str
    name: str
    n_res: int
    channel: List[int]
    spin: List[int]
    theta_true: np.ndarray
    n_data: int
    n_mc: int
    width_mode: int = 0          # 0 = mass-dependent width, 1 = constant width
    parent_mass: float = PARENT_MASS
    masses: tuple = DAUGHTER_MASSES
    r: float = R_BARRIER
    extra: dict = field(default_factory=dict)

    @property
    def n_par(self) -> int:
        return 4 * self.n_res


def workload(key: str) -> Workload:
    """The synthetic workloads by name:
        k2_fit      K = 2 in channel (12), J = 0, 1; 10k data / 50k MC (CPU-sized fit)
        k12_hvp     K = 12 over three channels; 1M data / 5M MC (NLL, gradient, HVP)
        k20_batched K = 20, frozen lineshapes; 2M data / 10M MC, 256 starts
        k30_diff    K = 30; 4M data / 20M MC (large differentiation)
        k12_toys    K = 12 toys for the start proposal"""
    if key == "k2_fit":
        c2 = 0.6 * np.exp(1.2j)
        th = np.array([1.0, 0.0, 0.90, 0.10, c2.real, c2.imag, 0.892, 0.05])
        return Workload(key, "cpu-sized K=2 channel (12), J=0,1", 2, [0, 0], [0, 1],
                        th, n_data=10_000, n_mc=50_000)
    if key in ("k12_hvp", "k12_toys"):
        ch, sp = resonance_layout(12)
        th = draw_theta(ch, sp, rng_for(key, STREAM_MODEL))
        if key == "k12_hvp":
            return Workload(key, "gpu-scale K=12, 1M data / 5M MC", 12, ch, sp, th,
                            n_data=1_000_000, n_mc=5_000_000)
        return Workload(key, "learned-start K=12 toys", 12, ch, sp, th,
                        n_data=50_000, n_mc=500_000,
                        extra={"n_train_toys": 20_000, "n_eval_toys": 200,
                               "eval_n_data": 1_000_000, "eval_n_mc": 5_000_000,
                               "n_random_starts": 256, "hist_bins": 32})
    if key == "k20_batched":
        ch, sp = resonance_layout(20)
        th = draw_theta(ch, sp, rng_for(key, STREAM_MODEL))
        return Workload(key, "batched fixed-lineshape K=20, 2M data / 10M MC, B=256",
                        20, ch, sp, th, n_data=2_000_000, n_mc=10_000_000,
                        extra={"n_starts": 256})
    if key == "k30_diff":
        ch, sp = resonance_layout(30)
        th = draw_theta(ch, sp, rng_for(key, STREAM_MODEL))
        return Workload(key, "differentiation K=30, 4M data / 20M MC", 30, ch, sp, th,
                        n_data=4_000_000, n_mc=20_000_000)
    raise ValueError(f"unknown workload {key}")

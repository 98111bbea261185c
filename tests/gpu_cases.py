"""Shared helpers of the GPU parity tests: seeded cases, oracle evaluation and
the tolerance rules.

Tolerances (FP64 path): the NLL to 1e-10 relative; every gradient component
to 1e-10 of its absolute-sum scale S_p = sum over events of |per-event term|
(oracle.grad_scale: a rounding bound for a summed quantity is proportional to
it; a plain relative test is meaningless where a component cancels to ~0);
every H v component to 1e-10 of the eq. (7) scale of oracle.hvp_scale (the
absolute sums of the three terms of eq. (7), each piece of the per-event data
term kept apart, plus the rounding of dG and dG.v in the last term).
FP32 path: NLL to 1e-5 relative; gradient and H v components to 3e-5 of the
same scales (single-precision per-event arithmetic has relative error of a few
units of 2^-24 = 6e-8 amplified by the cancellation in M^2 - s near a pole,
and event sums are FP64, so 3e-5 S_p bounds the sum with a wide margin).
"""

import numpy as np

import oracle
import synth


class Model:
    def __init__(self, channel, spin, width_mode=0):
        self.channel = list(channel)
        self.spin = list(spin)
        self.width_mode = width_mode
        self.parent_mass = synth.PARENT_MASS
        self.masses = synth.DAUGHTER_MASSES
        self.r = synth.R_BARRIER
        self.n_res = len(self.channel)


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def case(K, nd, nm, seed, width_mode=0):
    ch, sp = synth.resonance_layout(K)
    model = Model(ch, sp, width_mode)
    th = synth.draw_theta(ch, sp, rng(seed))
    data = synth.resonant_like(nd, ch, th, rng(seed + 1)) if nd else (np.zeros(0), np.zeros(0))
    mc = synth.uniform_phase_space(nm, rng(seed + 2))
    v = rng(seed + 3).normal(size=4 * K)
    return model, th, data, mc, v


def likelihood(model, data, mc, streams=("f64",)):
    from paper_2403_09225_amd import Likelihood
    lik = Likelihood(model.channel, model.spin, width_mode=model.width_mode, streams=streams)
    return lik.bind(data[0], data[1], mc[0], mc[1])


def oracle_all(model, data, mc, th, v):
    f, g, hv = oracle.hvp(data, mc, model, th, v)
    S = oracle.grad_scale(data, mc, model, th)
    SH = oracle.hvp_scale(data, mc, model, th, v)
    return f, g, hv, S, SH


def assert_close(name, got, ref, scale, tol):
    got = np.asarray(got, dtype=float)
    ref = np.asarray(ref, dtype=float)
    err = np.abs(got - ref)
    bound = tol * np.asarray(scale, dtype=float)
    bad = np.nonzero(~(err <= bound))[0]
    assert bad.size == 0, (f"{name}: {bad.size} components off, worst index {bad[np.argmax(err[bad] / bound[bad])]}"
                           f" err/bound = {np.max(err[bad] / bound[bad]):.3g}")
    return float(np.max(err / np.maximum(bound, 1e-300))) if err.size else 0.0

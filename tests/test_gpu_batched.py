"""Fixed-lineshape batched path on the GPU (matrix cores) against the oracle.

Tolerances:
* Gram matrix (FP64 MFMA): 1e-12 relative to its largest element.
* FP64 operands: NLL_b to 1e-10 relative (FP64 matrix cores, FP64 logs).
* FP32 and FP16 hi/lo-split operands: |NLL_b - oracle| <= 1e-3 absolute at
  these sizes (per-event relative error of |Z|^2 a few units of 2^-23 from
  operand rounding and FP32 accumulation, summed over the data events).
* BF16, FP16 operands: compared with the oracle evaluated on identically
  rounded operands (the rounding error itself is the format's, large; the
  check isolates the kernel's own error: FP32 accumulation of a rounded
  product and FP32 logs), 2e-6 relative per data event.
"""

import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_cases import Model, likelihood, rng

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _case(K, nd, nm, B, seed):
    ch, sp = synth.resonance_layout(K)
    model = Model(ch, sp)
    th = synth.draw_theta(ch, sp, rng(seed))
    data = synth.resonant_like(nd, ch, th, rng(seed + 1))
    mc = synth.uniform_phase_space(nm, rng(seed + 2))
    r = rng(seed + 3)
    C = r.uniform(0, 1, (K, B)) * np.exp(2j * np.pi * r.uniform(size=(K, B)))
    return model, th, data, mc, C


@pytest.mark.parametrize("K", [5, 20])
def test_gram_matches_oracle(K):
    say(f"[batched gram] K={K}")
    model, th, data, mc, C = _case(K, 500, 20011, 4, 90 + K)
    lik = likelihood(model, data, mc).freeze(th, "f64", 8)
    Gm = lik.gram().cpu().numpy()
    ref = oracle.gram(mc, model, th)
    assert np.max(np.abs(Gm - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("K,nd,B", [(5, 3001, 7), (20, 4001, 256), (12, 777, 65)])
@pytest.mark.parametrize("fmt", ["f64", "f32", "f16x3"])
def test_batched_nll_accurate_formats(K, nd, B, fmt):
    say(f"[batched] K={K} nd={nd} B={B} {fmt}")
    model, th, data, mc, C = _case(K, nd, 8009, B, 100 + K)
    lik = likelihood(model, data, mc).freeze(th, fmt, B)
    got = lik.nll_batched(C).cpu().numpy()
    ref = oracle.nll_batched(data, mc, model, th, C)
    if fmt == "f64":
        assert np.all(np.abs(got - ref) <= 1e-10 * np.abs(ref)), np.max(np.abs(got - ref) / np.abs(ref))
    else:
        assert np.max(np.abs(got - ref)) <= 1e-3, np.max(np.abs(got - ref))


@pytest.mark.parametrize("fmt", ["bf16", "f16"])
def test_batched_nll_low_precision_formats(fmt):
    K, nd, B = 20, 3001, 64
    say(f"[batched] K={K} {fmt}")
    model, th, data, mc, C = _case(K, nd, 8009, B, 120)
    lik = likelihood(model, data, mc).freeze(th, fmt, B)
    got = lik.nll_batched(C).cpu().numpy()
    # data term of the oracle on identically rounded A and C; normalisation
    # in FP64 on unrounded MC amplitudes, as the library computes it
    F_round, _ = oracle.nll_batched(data, mc, model, th, C, fmt=fmt, parts=True)
    _, G = oracle.nll_batched(data, mc, model, th, C, parts=True)
    ref = -F_round + nd * np.log(G / len(mc[0]))
    assert np.max(np.abs(got - ref)) <= 2e-6 * nd, np.max(np.abs(got - ref))


def test_batched_matches_plain_path_at_each_start():
    """NLL_b of the batched path (FP64) equals pwa_nll with theta's couplings
    replaced by c_b (same frozen M, Gamma)."""
    K, B = 12, 9
    say("[batched] vs plain pwa_nll")
    model, th, data, mc, C = _case(K, 1501, 6007, B, 130)
    lik = likelihood(model, data, mc).freeze(th, "f64", B)
    got = lik.nll_batched(C).cpu().numpy()
    for b in range(B):
        t = th.copy()
        t[0::4], t[1::4] = C[:, b].real, C[:, b].imag
        assert abs(float(lik.nll(t)) - got[b]) <= 1e-10 * abs(got[b])

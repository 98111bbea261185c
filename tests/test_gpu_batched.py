"""Fixed-lineshape batched path on the GPU (matrix cores) against the oracle.

Tolerances:
* Gram matrix (FP64 MFMA): 1e-12 relative to its largest element.
* FP64 operands: NLL_b to 1e-10 relative (FP64 matrix cores, FP64 logs).
* FP32 operands (couplings as hi + lo): |NLL_b - oracle| <= 1e-3 absolute
  at these sizes (per-event relative error of |Z|^2 a few units of 2^-23
  from operand rounding and FP32 accumulation, summed over the data events).
* Sliced FP16: <= 1e-3 absolute against the FP64 oracle, and against the
  oracle's own sliced-format product (which carries the format's
  representation error exactly) within 2^-26 per data event: what is left
  is the kernel's FP32 rounding of the level bracket, 2^-33 of the scale of
  Z, amplified by the cancellation in Z.
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


@pytest.mark.parametrize("K,nd,B", [(5, 3001, 7), (20, 4001, 256), (12, 777, 65), (8, 1000, 1),
                                    (24, 2999, 130), (3, 1500, 40), (18, 2500, 70)])
@pytest.mark.parametrize("fmt", ["f64", "f32", "f16s"])
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
    if fmt == "f16s":
        # the format's own product; the normalisation is FP64 in the library
        F_s, _ = oracle.nll_batched(data, mc, model, th, C, fmt="f16s", parts=True)
        _, G = oracle.nll_batched(data, mc, model, th, C, parts=True)
        ref_s = -F_s + nd * np.log(G / len(mc[0]))
        say(f"  vs sliced product {np.max(np.abs(got - ref_s)):.3g}, vs FP64 {np.max(np.abs(got - ref)):.3g}")
        assert np.max(np.abs(got - ref_s)) <= 2.0 ** -26 * nd, np.max(np.abs(got - ref_s))


def test_batched_full_size_against_oracle():
    """Configuration-2 size: K = 20, 2M data events (100k MC: the
    normalisation is the FP64 Gram matrix in every format), 256 starts on
    the GPU, 32 of them (every 8th) against the oracle.  Reports two figures
    per format: the operand representation alone (oracle on the format's
    operands against the FP64 oracle) and the GPU result against the FP64
    oracle.  Bounds: FP64 1e-10 relative; sliced FP16 1e-4 absolute (its
    representation error, random over events at 2^-28 of each row's largest
    amplitude, is about 1e-5 here) and 1e-5 against its own product; FP32
    5e-3 (amplitudes rounded at 2^-24 and FP32 accumulation with
    cancellation, random over events: about 2e-3 here; this format does not
    meet 1e-3 at 2M events)."""
    W = synth.workload("k20_batched")
    nd, nm, B = W.n_data, 100_000, W.extra["n_starts"]
    data = synth.resonant_like(nd, W.channel, W.theta_true, synth.rng_for("k20_batched", synth.workloads.STREAM_DATA))
    mc = synth.uniform_phase_space(nm, synth.rng_for("k20_batched", synth.workloads.STREAM_MC))
    r = synth.rng_for("k20_batched", synth.workloads.STREAM_TEST)
    C = r.uniform(0, 1, (W.n_res, B)) * np.exp(2j * np.pi * r.uniform(size=(W.n_res, B)))
    pick = np.arange(0, B, 8)
    Cs = C[:, pick]
    model = Model(W.channel, W.spin)
    say(f"[batched full size] oracle on {nd} events x {len(pick)} starts")
    F64, G = oracle.nll_batched(data, mc, model, W.theta_true, Cs, parts=True)
    ref = -F64 + nd * np.log(G / nm)
    F_s, _ = oracle.nll_batched(data, mc, model, W.theta_true, Cs, fmt="f16s", parts=True)
    # FP32 format: amplitudes rounded to FP32, couplings carried (almost) exactly
    F_a = np.zeros(len(pick))
    for lo in range(0, nd, 100_000):
        ev = (data[0][lo:lo + 100_000], data[1][lo:lo + 100_000])
        A = np.stack(oracle.amplitudes(ev, model, W.theta_true), axis=1)
        Z = (oracle.round_to(A.real, "f32") + 1j * oracle.round_to(A.imag, "f32")) @ Cs
        F_a += np.sum(np.log(Z.real ** 2 + Z.imag ** 2), axis=0)
    rep_alone = {"f16s": float(np.max(np.abs(F_s - F64))), "f32": float(np.max(np.abs(F_a - F64)))}
    lik = likelihood(model, data, mc)
    for fmt, bound in (("f64", None), ("f16s", 1e-4), ("f32", 5e-3)):
        say(f"[batched full size] GPU {fmt}")
        lik.freeze(W.theta_true, fmt, B)
        got = lik.nll_batched(C).cpu().numpy()[pick]
        err = np.max(np.abs(got - ref))
        say(f"  {fmt}: representation alone {rep_alone.get(fmt, 0.0):.3g}, GPU vs FP64 oracle {err:.3g}")
        if fmt == "f64":
            assert np.all(np.abs(got - ref) <= 1e-10 * np.abs(ref)), err
        else:
            assert err <= bound, (fmt, err)
        if fmt == "f16s":
            own = np.max(np.abs(got - (-F_s + nd * np.log(G / nm))))
            say(f"  f16s vs its own product {own:.3g}")
            assert own <= 1e-5, own


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

"""Differentiation at scale: K = 30 resonances (120 parameters) over 4M data
and 20M MC events, FP64 and FP32 event streams.

* gradient and H v against the oracle on a 50k + 250k subsample (the FP64
  tolerance rule of the parity tests: 1e-10 of each component's
  absolute-sum scale);
* over all 24M events: the GPU FP64 NLL's central difference (Richardson,
  h = 1e-6 and 5e-7) along a random direction equals g . d, and the central
  difference of GPU gradients equals H d;
* over all 24M events, gradient and H v element by element against the
  oracle (16 worker processes over event shards, eq. (4)-(7) combine): FP64
  stream to 1e-10 of the absolute-sum scales; FP32 stream gradient to 3e-5
  of S and H v to 3e-4 of SH (the stream's s, u, g are rounded at 2^-24 and
  the H v terms carry up to three powers of w = 1/D, whose derivatives
  amplify that rounding near the narrow resonances; measured 1.3e-4, as
  the 1e-4 level of the FP32 Hessian entries);
* the FP32 stream (FP64 reductions) tracks the FP64 stream: NLL to 1e-5
  relative, gradient and H v to 1e-3 of their largest component;
* the autograd wrapper's double backward returns pwa_hvp's H v;
* memory: the workspace grows by the event stream only (18 planes), nothing
  is stored per event for the derivatives.
"""

import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_cases import Model, assert_close, likelihood, oracle_all

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def k30_diff():
    W = synth.workload("k30_diff")
    say(f"[k30_diff] generating {W.n_data} + {W.n_mc} events, K = {W.n_res}")
    mc = synth.uniform_phase_space(W.n_mc, synth.rng_for("k30_diff", synth.workloads.STREAM_MC))
    data = synth.resonant_like(W.n_data, W.channel, W.theta_true,
                               synth.rng_for("k30_diff", synth.workloads.STREAM_DATA))
    lik = likelihood(W, data, mc, streams=("f64", "f32"))
    return W, data, mc, lik


def _np(t):
    return t.detach().cpu().numpy()


def test_k30_subsample_against_oracle(k30_diff):
    W, data, mc, _ = k30_diff
    say("[k30_diff] 50k + 250k subsample vs oracle")
    d = (data[0][:50_000], data[1][:50_000])
    m = (mc[0][:250_000], mc[1][:250_000])
    model = Model(W.channel, W.spin)
    v = synth.rng_for("k30_diff", synth.workloads.STREAM_TEST).normal(size=W.n_par)
    f, g, hv, S, SH = oracle_all(model, d, m, W.theta_true, v)
    lik = likelihood(model, d, m)
    hv_g, f_g, g_g = lik.hvp(W.theta_true, v)
    assert abs(float(f_g) - f) <= 1e-10 * abs(f)
    assert_close("grad", _np(g_g), g, S, 1e-10)
    assert_close("hvp", _np(hv_g), hv, SH, 1e-10)


def test_k30_fullsize_against_oracle(k30_diff):
    import multiprocessing as mp
    import os
    from tests.oracle_workers import shard
    W, data, mc, lik = k30_diff
    th = W.theta_true
    v = synth.rng_for("k30_diff", 9).normal(size=W.n_par)
    n = 16
    nd, nm = len(data[0]), len(mc[0])
    bd = [nd * i // n for i in range(n + 1)]
    bm = [nm * i // n for i in range(n + 1)]
    jobs = [((data[0][bd[i]:bd[i + 1]], data[1][bd[i]:bd[i + 1]]),
             (mc[0][bm[i]:bm[i + 1]], mc[1][bm[i]:bm[i + 1]]), W, th, v) for i in range(n)]
    say(f"[k30_diff] grad and H v vs oracle over {nd + nm} events ({n} worker processes)")
    env = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in env:
        os.environ[k] = "1"
    try:
        with mp.get_context("spawn").Pool(n) as pool:
            res = pool.map(shard, jobs)
    finally:
        for k, val in env.items():
            if val is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = val
    ref = oracle.combine([r[0] for r in res], v=v)
    hF, gF, hG, gG = (np.sum([r[1][j] for r in res], axis=0) for j in range(4))
    G = sum(r[1][4] for r in res)
    S = gF + nd / G * gG
    SH = hF + nd / G * hG + 2.0 * nd / (G * G) * gG * np.sum(np.abs(v) * gG)
    for prec, tol_f, tol, tol_h in (("f64", 1e-10, 1e-10, 1e-10), ("f32", 1e-5, 3e-5, 3e-4)):
        lik.set_precision(prec)
        try:
            hv, f, g = [_np(x) for x in lik.hvp(th, v)]
        finally:
            lik.set_precision("f64")
        say(f"  {prec}: max |dg|/S {np.max(np.abs(g - ref['grad']) / S):.3g}, "
            f"max |dHv|/SH {np.max(np.abs(hv - ref['hv']) / SH):.3g}")
        assert abs(float(f) - ref["nll"]) <= tol_f * abs(ref["nll"])
        assert np.all(np.abs(g - ref["grad"]) <= tol * S)
        assert np.all(np.abs(hv - ref["hv"]) <= tol_h * SH)


def test_k30_central_differences(k30_diff):
    W, data, mc, lik = k30_diff
    say("[k30_diff] central differences over 24M events")
    th = W.theta_true
    d = synth.rng_for("k30_diff", 6).normal(size=W.n_par)
    hv, _, g = lik.hvp(th, d)
    g, hv = _np(g), _np(hv)

    def fcd(h):
        return (float(lik.nll(th + h * d)) - float(lik.nll(th - h * d))) / (2 * h)

    def gcd(h):
        return (_np(lik.grad(th + h * d)[1]) - _np(lik.grad(th - h * d)[1])) / (2 * h)

    h = 1e-6
    fd = (4.0 * fcd(h / 2) - fcd(h)) / 3.0
    assert abs(fd - g @ d) <= 1e-5 * np.abs(g).max() * np.abs(d).sum()
    hfd = (4.0 * gcd(h / 2) - gcd(h)) / 3.0
    assert np.max(np.abs(hfd - hv)) <= 1e-5 * np.max(np.abs(hv))


def test_k30_fp32_stream_tracks_fp64(k30_diff):
    W, data, mc, lik = k30_diff
    say("[k30_diff] FP32 stream vs FP64 stream")
    th = W.theta_true
    v = synth.rng_for("k30_diff", 7).normal(size=W.n_par)
    hv64, f64, g64 = [_np(x) for x in lik.hvp(th, v)]
    lik.set_precision("f32")
    try:
        hv32, f32, g32 = [_np(x) for x in lik.hvp(th, v)]
    finally:
        lik.set_precision("f64")
    assert abs(float(f32) - float(f64)) <= 1e-5 * abs(float(f64))
    assert np.max(np.abs(g32 - g64)) <= 1e-3 * np.max(np.abs(g64))
    assert np.max(np.abs(hv32 - hv64)) <= 1e-3 * np.max(np.abs(hv64))


def test_k30_autograd_double_backward(k30_diff):
    W, data, mc, lik = k30_diff
    say("[k30_diff] autograd double backward")
    from paper_2403_09225_amd import nll as nll_fn
    th = torch.tensor(W.theta_true, dtype=torch.float64, device="cuda", requires_grad=True)
    v = torch.tensor(synth.rng_for("k30_diff", 8).normal(size=W.n_par), dtype=torch.float64, device="cuda")
    f = nll_fn(th, lik)
    (g,) = torch.autograd.grad(f, th, create_graph=True)
    (hv,) = torch.autograd.grad(g, th, grad_outputs=v)
    hv_ref, f_ref, g_ref = lik.hvp(W.theta_true, v)
    # NLL and gradient come from the NLL and gradient passes (their own
    # summation order); the double backward is pwa_hvp itself
    assert float(f.detach()) == pytest.approx(float(f_ref), rel=1e-13)
    gs = float(torch.max(torch.abs(g_ref)))
    assert float(torch.max(torch.abs(g.detach() - g_ref))) <= 1e-11 * gs
    assert torch.equal(hv, hv_ref)


def test_k30_memory_is_the_event_stream(k30_diff):
    W, _, _, lik = k30_diff
    n = W.n_data + W.n_mc
    grow = lik.workspace_bytes(W.n_data, W.n_mc) - lik.workspace_bytes(0, 1)
    stream = 18 * (8 + 4) * n          # FP64 and FP32 planes
    # planes are padded to a multiple of 64 events and regions to 256 bytes
    assert abs(grow - stream) <= 18 * 12 * 64 + 4096

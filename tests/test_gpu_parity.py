"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs, element by element.  Sizes span many blocks and teams and
end in ragged tails; tolerances are explained in tests/gpu_cases.py."""

import math
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_cases import Model, assert_close, case, likelihood, oracle_all, rng

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _np(t):
    return t.detach().cpu().numpy()


def _check_fp64(lik, model, th, data, mc, v, tol=1e-10):
    f, g, hv, S, SH = oracle_all(model, data, mc, th, v)
    nll = float(lik.nll(th))
    nll2, g2 = lik.grad(th)
    hv3, nll3, g3 = lik.hvp(th, v)
    for val in (nll, float(nll2), float(nll3)):
        assert abs(val - f) <= tol * abs(f), (val, f)
    assert_close("grad", _np(g2), g, S, tol)
    assert_close("grad(hvp pass)", _np(g3), g, S, tol)
    assert_close("hv", _np(hv3), hv, SH, tol)


@pytest.mark.parametrize("K,nd,nm,seed,wm", [
    (1, 777, 3001, 10, 0),
    (2, 2011, 9013, 11, 0),
    (5, 1500, 6007, 12, 0),
    (6, 1999, 7001, 13, 1),
    (12, 3001, 12007, 14, 0),
    (17, 1201, 4999, 15, 0),
    (30, 1003, 4001, 16, 0),
])
def test_fp64_parity(K, nd, nm, seed, wm):
    say(f"[fp64 parity] K={K} nd={nd} nm={nm} seed={seed} width_mode={wm}")
    model, th, data, mc, v = case(K, nd, nm, seed, wm)
    lik = likelihood(model, data, mc)
    _check_fp64(lik, model, th, data, mc, v)


@pytest.mark.parametrize("shape", [(1, 4, 3), (1, 4, 4), (1, 8, 2), (1, 8, 4), (1, 16, 2),
                                   (1, 16, 4), (1, 32, 2), (2, 4, 3), (2, 3, 4), (2, 6, 2),
                                   (2, 8, 2), (2, 8, 3), (2, 8, 4), (2, 12, 2), (2, 8, 8)])
def test_every_launch_shape(shape):
    say(f"[shape] K=12 layout,groups,R={shape}")
    model, th, data, mc, v = case(12, 1777, 6001, 20)
    lik = likelihood(model, data, mc)
    lik.set_launch_shape(*shape)
    _check_fp64(lik, model, th, data, mc, v)


@pytest.mark.parametrize("K,shape", [(2, (1, 1, 2)), (2, (1, 1, 4)), (3, (1, 1, 4)), (8, (1, 2, 4)),
                                     (6, (1, 4, 2)), (16, (1, 4, 4)), (30, (1, 16, 2)),
                                     (64, (1, 32, 2)), (2, (2, 1, 2)), (3, (2, 1, 4)), (5, (2, 2, 3)),
                                     (7, (2, 2, 4)), (8, (2, 4, 2)), (16, (2, 8, 2)), (22, (2, 8, 3)),
                                     (15, (2, 5, 3)), (24, (2, 12, 2)), (12, (2, 3, 4)),
                                     (30, (2, 8, 4)), (25, (2, 8, 4)), (40, (2, 8, 8)),
                                     (64, (2, 8, 8))])
def test_small_k_shapes(K, shape):
    say(f"[shape] K={K} layout,groups,R={shape}")
    model, th, data, mc, v = case(K, 913, 3007, 21 + K)
    lik = likelihood(model, data, mc)
    lik.set_launch_shape(*shape)
    _check_fp64(lik, model, th, data, mc, v)


@pytest.mark.parametrize("K,seed", [(12, 30), (30, 31)])
def test_fp32_parity(K, seed):
    say(f"[fp32 parity] K={K}")
    model, th, data, mc, v = case(K, 2001, 8009, seed)
    lik = likelihood(model, data, mc, streams=("f64", "f32"))
    lik.set_precision("f32")
    f, g, hv, S, SH = oracle_all(model, data, mc, th, v)
    hv3, nll3, g3 = lik.hvp(th, v)
    assert abs(float(lik.nll(th)) - f) <= 1e-5 * abs(f)
    assert abs(float(nll3) - f) <= 1e-5 * abs(f)
    assert_close("grad f32", _np(g3), g, S, 3e-5)
    assert_close("hv f32", _np(hv3), hv, SH, 3e-5)


def test_bitwise_deterministic():
    say("[determinism] K=12")
    model, th, data, mc, v = case(12, 3001, 12007, 40)
    lik = likelihood(model, data, mc)
    outs = [lik.hvp(th, v) for _ in range(3)]
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert torch.equal(a, b)


def test_partials_and_virtual_shards():
    """Eq. (4)-(7) across shards: three contexts, each bound to a share of
    the events (one GPU's share in the paper's multi-GPU scheme), combined by
    pwa_combine, equal the unsharded evaluation and the oracle."""
    say("[virtual shards] K=12")
    model, th, data, mc, v = case(12, 3001, 12007, 50)
    from paper_2403_09225_amd import combine
    whole = likelihood(model, data, mc)
    hv0, f0, g0 = whole.hvp(th, v)
    cd, cm = [0, 1000, 1001, 3001], [0, 5000, 9000, 12007]
    parts = []
    for i in range(3):
        d = (data[0][cd[i]:cd[i + 1]], data[1][cd[i]:cd[i + 1]])
        m = (mc[0][cm[i]:cm[i + 1]], mc[1][cm[i]:cm[i + 1]])
        lik = likelihood(model, d, m)
        p = lik.partials(th, v)
        ref = oracle.partials(d, m, model, th, v=v)
        pp = _np(p).reshape(-1, 2).sum(axis=1)
        P = 48
        assert pp[0] == pytest.approx(ref["F"], rel=1e-12, abs=1e-9)
        assert pp[1] == pytest.approx(ref["G"], rel=1e-12)
        S = oracle.grad_scale(d, m, model, th)
        for name, sl, r in [("dF", slice(2, 2 + P), ref["dF"]), ("dG", slice(2 + P, 2 + 2 * P), ref["dG"])]:
            assert np.all(np.abs(pp[sl] - r) <= 1e-10 * (np.abs(r) + S)), name
        parts.append(p)
    f1, g1, hv1 = combine(parts, 48, len(data[0]), len(mc[0]), v)
    f, g, hv, S, SH = oracle_all(model, data, mc, th, v)
    assert float(f1) == pytest.approx(float(f0), rel=1e-13)
    assert_close("grad shards", _np(g1), _np(g0), S, 1e-12)
    assert_close("hv shards", _np(hv1), _np(hv0), SH, 1e-12)
    assert abs(float(f1) - f) <= 1e-10 * abs(f)
    assert_close("hv shards vs oracle", _np(hv1), hv, SH, 1e-10)


def test_partials_reuse_virtual_shards():
    """The sharded CG step: three contexts each take pwa_partials at theta
    with one direction, then pwa_partials_reuse with a new one; the combine
    of the reused partials equals the unsharded H w and the oracle's."""
    say("[virtual shards, reuse] K=12")
    model, th, data, mc, v = case(12, 3001, 12007, 51)
    from paper_2403_09225_amd import combine
    w = rng(52).normal(size=48)
    cd, cm = [0, 1000, 1001, 3001], [0, 5000, 9000, 12007]
    liks = []
    for i in range(3):
        d = (data[0][cd[i]:cd[i + 1]], data[1][cd[i]:cd[i + 1]])
        m = (mc[0][cm[i]:cm[i + 1]], mc[1][cm[i]:cm[i + 1]])
        lik = likelihood(model, d, m)
        lik.partials(th, v)
        liks.append(lik)
    parts = [lik.partials_reuse(w) for lik in liks]
    f1, g1, hv1 = combine(parts, 48, len(data[0]), len(mc[0]), w)
    f, g, hv, S, SH = oracle_all(model, data, mc, th, w)
    assert abs(float(f1) - f) <= 1e-10 * abs(f)
    assert_close("grad reuse shards", _np(g1), g, S, 1e-10)
    assert_close("hv reuse shards", _np(hv1), hv, SH, 1e-10)
    # equal to a full pass per shard to rounding
    full = [lik.partials(th, w) for lik in liks]
    _, _, hv2 = combine(full, 48, len(data[0]), len(mc[0]), w)
    assert np.all(np.abs(_np(hv1) - _np(hv2)) <= 1e-12 * SH)


def test_edge_cases():
    say("[edge] empty data, single events, below threshold, zero couplings")
    # no data events: NLL = 0 and gradient 0 (N_D = 0)
    model, th, data, mc, v = case(3, 0, 500, 60)
    lik = likelihood(model, data, mc)
    hv, f, g = lik.hvp(th, v)
    assert float(f) == 0.0
    assert np.all(_np(g) == 0.0) and np.all(_np(hv) == 0.0)
    # one data and one MC event
    model, th, data, mc, v = case(3, 1, 1, 61)
    lik = likelihood(model, data, mc)
    _check_fp64(lik, model, th, data, mc, v)
    # mass below its pair threshold: NLL = +inf and status bit 1
    model, th, data, mc, v = case(3, 50, 200, 62)
    lik = likelihood(model, data, mc)
    bad = th.copy()
    bad[4 * 2 + 2] = 0.25       # resonance 2 is in channel (23), threshold 0.28 GeV
    assert math.isinf(float(lik.nll(bad)))
    assert lik.device_status() & 1
    assert lik.device_status() == 0      # sticky word cleared by the read
    # all couplings zero: G = 0, NLL = +inf and status bit 2
    z = th.copy()
    z[0::4] = 0.0
    z[1::4] = 0.0
    assert math.isinf(float(lik.nll(z)))
    assert lik.device_status() & 2
    # and a normal evaluation afterwards is unaffected
    assert math.isfinite(float(lik.nll(th)))


def test_bw_integral_closed_form_on_gpu():
    """Constant width, J = 0 on a midpoint grid of 1e6 points in s12: the
    GPU's G times the grid step equals the closed-form Breit-Wigner integral
    (atan difference / (M Gamma)) to ~(h/(M Gamma))^2/12."""
    say("[bw integral] 1e6 points")
    model = Model([0], [0], width_mode=1)
    M, G = 1.1, 0.08
    th = np.array([1.0, 0.0, M, G])
    s12, s13, h = synth.midpoint_line_s12(1_000_000)
    lik = likelihood(model, (s12[:1], s13[:1]), (s12, s13))
    p = _np(lik.partials(th)).reshape(-1, 2).sum(axis=1)
    (a0, a1), _ = synth.bounding_box()
    exact = (math.atan((a1 - M * M) / (M * G)) - math.atan((a0 - M * M) / (M * G))) / (M * G)
    assert abs(p[1] * h - exact) <= 1e-9 * exact


def test_legendre_orthogonality_on_gpu():
    """S-P interference term of G vanishes on mirror-symmetric MC:
    G(c1, c2) = |c1|^2 G_SS + |c2|^2 G_PP exactly for any phase of c2."""
    say("[legendre] mirror MC")
    model = Model([0, 0], [0, 1])
    mc = synth.mirror_symmetric(*synth.uniform_phase_space(100_000, rng(70)))
    lik = likelihood(model, (mc[0][:1], mc[1][:1]), mc)
    base = np.array([1.0, 0.0, 0.9, 0.1, 0.0, 0.0, 0.892, 0.05])

    def G(c2):
        t = base.copy()
        t[4], t[5] = c2.real, c2.imag
        return _np(lik.partials(t)).reshape(-1, 2).sum(axis=1)[1]
    g0 = G(0.0 + 0.0j)
    t = base.copy()
    t[0] = 0.0
    t[4] = 1.0
    gpp = _np(lik.partials(t)).reshape(-1, 2).sum(axis=1)[1]
    for ph in (0.0, 1.0, 2.5):
        g = G(np.exp(1j * ph))
        assert abs(g - (g0 + gpp)) <= 1e-12 * (g0 + gpp)


def test_autograd_double_backward():
    say("[autograd] K=6")
    from paper_2403_09225_amd import nll as nll_fn
    model, th, data, mc, v = case(6, 1501, 6007, 80)
    lik = likelihood(model, data, mc)
    f, g, hv, S, SH = oracle_all(model, data, mc, th, v)
    t = torch.tensor(th, dtype=torch.float64, device="cuda", requires_grad=True)
    val = nll_fn(t, lik)
    (gt,) = torch.autograd.grad(val, t, create_graph=True)
    vt = torch.tensor(v, dtype=torch.float64, device="cuda")
    (hvt,) = torch.autograd.grad(gt @ vt, t)
    assert abs(float(val) - f) <= 1e-10 * abs(f)
    assert_close("autograd grad", _np(gt), g, S, 1e-10)
    assert_close("autograd hv", _np(hvt), hv, SH, 1e-10)


def test_many_iterations_per_block():
    """~230k events: every block of the benchmark's launch shape loops over
    many event batches (software-pipelined loads, LDS exchange buffers), as
    at full size; gradient and H v against the oracle."""
    say("[many iterations] K=12, 40k data + 190k MC")
    model, th, data, mc, v = case(12, 40_000, 190_000, 140)
    lik = likelihood(model, data, mc)
    _check_fp64(lik, model, th, data, mc, v)


# ------------------------------------------------- HVP reuse at a fixed theta
@pytest.mark.parametrize("K,nd,nm,seed,shape", [
    (1, 777, 3001, 60, None), (2, 2011, 9013, 61, None), (5, 1500, 6007, 62, None),
    (12, 3001, 12007, 63, None), (17, 1201, 4999, 64, None), (30, 1003, 4001, 65, None),
    (12, 1999, 7001, 66, (2, 3, 4)), (16, 913, 3007, 67, (1, 16, 2)), (40, 501, 2001, 68, None)])
def test_hvp_reuse_parity(K, nd, nm, seed, shape):
    """pwa_hvp_reuse (direction moments only, theta-only totals of the last
    pwa_hvp) against the oracle for several new directions, FP64 and FP32
    streams, and equal to a full pass to rounding, in both layouts (team
    layout: the (1, 16, 2) case and the full pass at K > 32, whose
    direction-only pass runs in 8 waves x 8)."""
    say(f"[hvp reuse] K={K} shape={shape}")
    model, th, data, mc, v = case(K, nd, nm, seed)
    lik = likelihood(model, data, mc, streams=("f64", "f32"))
    if shape:
        lik.set_launch_shape(*shape)
    f, g, _, S, _ = oracle_all(model, data, mc, th, v)
    # FP32 stream: 3e-5 of the absolute-sum scale up to K = 32; with more
    # resonances z sums more FP32-rounded terms that cancel, and the bound
    # is widened to 1e-4 (the FP64 bound does not change)
    tol32 = 3e-5 if K <= 32 else 1e-4
    for prec, tol in (("f64", 1e-10), ("f32", tol32)):
        lik.set_precision(prec)
        lik.hvp(th, v)
        for d in range(3):
            w = rng(seed * 10 + d).normal(size=4 * K)
            _, _, hvo = oracle.hvp(data, mc, model, th, w)
            SHw = oracle.hvp_scale(data, mc, model, th, w)
            hv, nll, gg = lik.hvp_reuse(w)
            assert abs(float(nll) - f) <= (1e-10 if prec == "f64" else 1e-5) * abs(f)
            assert_close(f"grad reuse {prec}", _np(gg), g, S, tol)
            assert_close(f"hv reuse {prec} dir {d}", _np(hv), hvo, SHw, tol)
            full, _, _ = lik.hvp(th, w)
            scale = SHw
            # above K = 32 the automatic shapes differ (the full pass in the
            # team layout, the direction-only pass in 8 waves x 8): their FP32
            # sums take other rounding orders, and agree to the FP32 stream's
            # bound, not to one order's last bits
            b32 = 1e-6 if (shape is not None or K <= 32) else tol32
            assert np.all(np.abs(_np(hv) - _np(full)) <= (1e-12 if prec == "f64" else b32) * scale)


def test_hvp_reuse_state():
    """Reuse needs the totals of a pwa_hvp on this context: before any, and
    after any other evaluation, it is refused; a precision change makes it
    take a full pass at the cached theta (still the right product)."""
    from paper_2403_09225_amd import _lib as L
    model, th, data, mc, v = case(6, 1001, 4001, 70)
    lik = likelihood(model, data, mc, streams=("f64", "f32"))
    w = rng(71).normal(size=24)
    with pytest.raises(L.PwaError):
        lik.hvp_reuse(w)
    ref, _, _ = lik.hvp(th, w)
    lik.hvp(th, v)
    hv, _, _ = lik.hvp_reuse(w)
    torch.testing.assert_close(hv, ref, rtol=1e-10, atol=1e-10 * float(ref.abs().max()))
    lik.nll(th)
    with pytest.raises(L.PwaError):
        lik.hvp_reuse(w)
    lik.hvp(th, v)
    lik.set_precision("f32")
    hv32, _, _ = lik.hvp_reuse(w)
    ref32, _, _ = lik.hvp(th, w)
    torch.testing.assert_close(hv32, ref32, rtol=1e-6, atol=1e-6 * float(ref32.abs().max()))
    lik.set_precision("f64")
    lik.hvp(th, v)
    lik.grad(th + 0.01)
    with pytest.raises(L.PwaError):
        lik.hvp_reuse(w)
    lik.hvp(th, v)
    lik.hessian(th)
    with pytest.raises(L.PwaError):
        lik.hvp_reuse(w)

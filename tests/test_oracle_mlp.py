"""Pins of the learned-start oracle (histogram, MLP, Adam, bf16 rounding)
against facts that do not come from its own formulas: tabulated values of
the normal distribution, symmetry identities, central finite differences,
library routines for special cases, and closed forms of Adam's first steps."""

import math

import numpy as np
import pytest
import torch

import synth
from oracle import mlp_oracle as M


def test_gelu_values_and_identities():
    # Phi(1) and Phi(2) from standard normal tables
    assert M.gelu(np.array([1.0]))[0] == pytest.approx(0.8413447460685429, rel=1e-15)
    assert M.gelu(np.array([2.0]))[0] == pytest.approx(2.0 * 0.9772498680518208, rel=1e-15)
    assert M.gelu(np.array([0.0]))[0] == 0.0
    x = np.linspace(-4, 4, 17)
    # Phi(-x) = 1 - Phi(x)  =>  GELU(-x) = GELU(x) - x
    assert np.allclose(M.gelu(-x), M.gelu(x) - x, rtol=0, atol=1e-15)
    # derivative against central differences; GELU'(0) = 1/2
    h = 1e-5
    fd = (M.gelu(x + h) - M.gelu(x - h)) / (2 * h)
    assert np.allclose(M.gelu_prime(x), fd, rtol=0, atol=1e-9)
    assert M.gelu_prime(np.array([0.0]))[0] == 0.5


def test_bf16_rounding_matches_torch():
    assert M.bf16(1.0 + 2.0 ** -8) == 1.0                       # tie -> even
    assert M.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6       # tie -> even
    assert M.bf16(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    r = np.random.Generator(np.random.PCG64(1)).normal(scale=10.0, size=5000)
    ref = torch.tensor(r, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16(r), ref)


def test_histogram_matches_numpy_and_edges():
    box = synth.bounding_box()
    s12, s13 = synth.uniform_phase_space(3000, np.random.Generator(np.random.PCG64(2)))
    h = M.histogram(s12, s13, box)
    (a0, a1), (b0, b1) = box
    ref, _, _ = np.histogram2d(s12, s13, bins=(np.linspace(a0, a1, 33), np.linspace(b0, b1, 33)))
    assert np.allclose(h, ref.ravel() / 3000, rtol=0, atol=1e-15)
    assert h.sum() == pytest.approx(1.0, abs=1e-12)
    # an event on the upper corner lands in the last bin
    e = M.histogram(np.array([a1]), np.array([b1]), box)
    assert e[-1] == 1.0 and e.sum() == 1.0


DIMS = (8, 6, 5, 3)


def _net(seed):
    r = np.random.Generator(np.random.PCG64(seed))
    p = r.normal(scale=0.5, size=M.n_params(DIMS))
    x = r.normal(size=(4, DIMS[0]))
    t = r.normal(size=(4, DIMS[3]))
    return p, x, t


def test_gradient_against_central_differences():
    p, x, t = _net(3)
    loss, g = M.loss_and_grad(p, DIMS, x, t)
    h = 1e-6
    fd = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        fd[i] = (M.loss_and_grad(p + e, DIMS, x, t)[0] - M.loss_and_grad(p - e, DIMS, x, t)[0]) / (2 * h)
    assert np.max(np.abs(g - fd)) <= 1e-8 * max(1.0, np.max(np.abs(g)))


def test_zero_weights_give_the_bias_and_closed_form_loss():
    p, x, t = _net(4)
    W1, b1, W2, b2, W3, b3 = M.unpack(p, DIMS)
    q = p.copy()
    n = DIMS[2] * DIMS[3]
    start = M.n_params(DIMS) - DIMS[3] - n
    q[start:start + n] = 0.0        # W3 = 0: y = b3 for every sample
    y, _ = M.forward(q, DIMS, x)
    assert np.array_equal(y, np.tile(b3, (4, 1)))
    loss, g = M.loss_and_grad(q, DIMS, x, t)
    assert loss == pytest.approx(np.mean((b3 - t) ** 2), rel=1e-14)
    # dL/db3 = 2 mean over the batch of (b3 - t) / P
    assert np.allclose(g[-DIMS[3]:], 2.0 * np.sum(b3 - t, axis=0) / (4 * DIMS[3]), rtol=1e-13, atol=0)


def test_adam_first_steps_closed_form():
    r = np.random.Generator(np.random.PCG64(5))
    w = r.normal(size=50)
    g = r.normal(size=50)
    m = np.zeros(50)
    v = np.zeros(50)
    lr = 1e-3
    w1, m, v = M.adam(w, m, v, g, 1, lr, eps=0.0)
    # bias correction makes the first step exactly lr * sign(g)
    assert np.allclose(w1 - w, -lr * np.sign(g), rtol=0, atol=1e-15)
    w2, m, v = M.adam(w1, m, v, g, 2, lr, eps=0.0)
    assert np.allclose(w2 - w1, -lr * np.sign(g), rtol=0, atol=1e-15)
    # an opposite gradient on step 2: m-hat = (0.09 g - 0.1 g)/0.19, v-hat = g^2
    w3, _, _ = M.adam(w1, 0.1 * g, 0.001 * g * g, -g, 2, lr, eps=0.0)
    mh = (0.9 * 0.1 - 0.1) / (1 - 0.81)
    assert np.allclose(w3 - w1, -lr * mh * np.sign(g), rtol=0, atol=1e-15)


def test_adam_weight_decay_alone_shrinks_geometrically():
    # zero gradient from zero moments: only the decoupled decay acts
    w = np.linspace(-1, 1, 11)
    z = np.zeros_like(w)
    w1, m, v = M.adam(w, z, z, z, 1, 0.01, wd=0.1)
    assert np.allclose(w1, w * (1 - 0.01 * 0.1), rtol=1e-15, atol=0)
    assert not m.any() and not v.any()

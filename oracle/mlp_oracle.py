"""FP64 CPU oracle for the learned start-point proposal: the binned Dalitz
histogram, the MLP 1024 -> 512 -> 512 -> P with GELU, its mean-squared-error
loss and gradient, and the Adam update.

TEST INFRASTRUCTURE ONLY: used by the test suite and the package smoke
check; never by the product path.  Shares no code with the HIP library.

The proposal network is an addition to the paper's method: the paper starts
Newton-CG from random points and counts how many reach the global minimum
(Sec. 3, the fit-success study); here a network maps the binned data to a
start point, with random multi-start as the fallback.

Definitions written out:
* histogram: 32 x 32 bins over the Dalitz bounding box (s12 along rows,
  s13 along columns), counts divided by the number of events; an event on
  an upper edge falls in the last bin.
* GELU(x) = x Phi(x) = x (1 + erf(x / sqrt 2)) / 2, the exact form.
* layers: h1 = GELU(W1 x + b1), h2 = GELU(W2 h1 + b2), y = W3 h2 + b3, with
  W[out][in] row-major.
* loss L = sum over the batch and outputs of (y - t)^2 / (B * P).
* Adam (Kingma and Ba): m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
  w <- w - lr [(m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps) + wd w], the
  last term being decoupled weight decay (Loshchilov and Hutter).
* BF16 emulation (optional): the points where the GPU rounds to bfloat16
  (inputs, weights, hidden activations, back-propagated signals) are rounded
  here the same way, round to nearest even, so that the difference from the
  GPU is accumulation order only.
"""

import math

import numpy as np

NBINS = 32


def histogram(s12, s13, box):
    """Normalised 32 x 32 counts (flattened, s12-major) by plain counting."""
    (a0, a1), (b0, b1) = box
    out = np.zeros(NBINS * NBINS)
    n = len(s12)
    for x, y in zip(s12, s13):
        i = min(NBINS - 1, max(0, int((x - a0) / (a1 - a0) * NBINS)))
        j = min(NBINS - 1, max(0, int((y - b0) / (b1 - b0) * NBINS)))
        out[i * NBINS + j] += 1.0
    return out / max(n, 1)


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(x):
    return 0.5 * x * (1.0 + np.vectorize(math.erf)(x / math.sqrt(2.0)))


def gelu_prime(x):
    """d/dx [x Phi(x)] = Phi(x) + x phi(x)."""
    Phi = 0.5 * (1.0 + np.vectorize(math.erf)(x / math.sqrt(2.0)))
    phi = np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)
    return Phi + x * phi


def unpack(params, dims):
    """Split the packed parameter vector [W1, b1, W2, b2, W3, b3]."""
    n_in, h1, h2, n_out = dims
    shapes = [(h1, n_in), (h1,), (h2, h1), (h2,), (n_out, h2), (n_out,)]
    out, o = [], 0
    for s in shapes:
        n = int(np.prod(s))
        out.append(np.asarray(params[o:o + n], dtype=np.float64).reshape(s))
        o += n
    return out


def n_params(dims):
    n_in, h1, h2, n_out = dims
    return h1 * n_in + h1 + h2 * h1 + h2 + n_out * h2 + n_out


def forward(params, dims, x, emulate_bf16=False):
    """Outputs y (B x P) and the saved activations."""
    W1, b1, W2, b2, W3, b3 = unpack(params, dims)
    r = bf16 if emulate_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    x = r(x)
    z1 = x @ r(W1).T + b1
    h1 = r(gelu(z1))
    z2 = h1 @ r(W2).T + b2
    h2 = r(gelu(z2))
    y = h2 @ r(W3).T + b3
    return y, (x, z1, h1, z2, h2)


def loss_and_grad(params, dims, x, t, emulate_bf16=False):
    """Mean-squared-error loss and its gradient (packed like params),
    by the chain rule through the three layers."""
    W1, b1, W2, b2, W3, b3 = unpack(params, dims)
    r = bf16 if emulate_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    y, (x, z1, h1, z2, h2) = forward(params, dims, x, emulate_bf16)
    B, P = y.shape
    loss = float(np.sum((y - t) ** 2) / (B * P))
    dy = r(2.0 * (y - t) / (B * P))
    gW3 = dy.T @ h2
    gb3 = dy.sum(0)
    dz2 = r((dy @ r(W3)) * gelu_prime(z2))
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(0)
    dz1 = r((dz2 @ r(W2)) * gelu_prime(z1))
    gW1 = dz1.T @ x
    gb1 = dz1.sum(0)
    g = np.concatenate([a.ravel() for a in (gW1, gb1, gW2, gb2, gW3, gb3)])
    return loss, g


def adam(w, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8, wd=0.0):
    """One Adam step at step number t >= 1; returns (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return w - lr * (mh / (np.sqrt(vh) + eps) + wd * w), m, v

"""Learned start-point proposal for Newton-CG fits.

The paper fits from random start points and counts how many fits reach the
global minimum (Sec. 3, the fit-success study: a few per cent to about a
third of random starts, depending on the convergence tolerance).  Here a
small network maps the binned data of a fit -- a 32 x 32 histogram of the
events over the Dalitz plane -- to a start point.  It is trained on fits that
the likelihood library performs on toy data drawn from the model, with
random multi-start as the fallback and the exact NLL deciding success.

Everything runs on the GPU through the library: toys (accept-reject on the
per-event intensity), histograms (pwa_hist2d), fits (pwa_fit), and the MLP's
forward pass, backward pass and Adam step (pwa_mlp_*, bfloat16 matrix cores
with FP32 master weights).

Parameter coding.  The NLL is invariant under a global phase and scale of
the couplings (eq. (3): the normalisation divides out |c|^2) and resonances
with the same channel and spin are interchangeable, so a label is made
canonical before it is learned: such resonances are ordered by mass, the
couplings are rotated so that c_0 is real positive and scaled to unit
r.m.s. modulus, and M, Gamma are mapped affinely from the prior's ranges
onto [-1, 1].
"""

import ctypes
import math
import os
import threading
import time

import numpy as np
import torch

from . import _lib as L
from .api import DAUGHTER_MASSES, PARENT_MASS, Likelihood, _ptr, _stream
from .toys import ToyGenerator

NBINS = 32
PAIRS = ((0, 1), (0, 2), (1, 2))     # daughters of channels (12), (13), (23)

# wide prior: the ranges of the random multi-start of a model-free search
M_RANGE = (0.6, 1.6)
G_RANGE = (0.03, 0.3)
C_RANGE = (0.2, 1.0)


def threshold(ch, masses=DAUGHTER_MASSES):
    a, b = PAIRS[ch]
    return masses[a] + masses[b]


class Prior:
    """Parameter prior of the toys' true parameters and of the random starts.

    Each resonance has a nominal mass and width (the model hypothesis of an
    analysis) and a relative spread around them; couplings have |c| uniform
    in c_range and a uniform phase.  A mass is redrawn while it is below the
    channel threshold + 20 MeV.  `Prior.wide` spans M in [0.6, 1.6] GeV and
    Gamma in [0.03, 0.3] GeV for every resonance."""

    def __init__(self, channel, m_nom, g_nom, m_spread, g_spread, c_range=C_RANGE,
                 masses=DAUGHTER_MASSES):
        self.channel = list(channel)
        K = len(self.channel)
        self.m_nom = np.broadcast_to(np.asarray(m_nom, dtype=np.float64), (K,)).copy()
        self.g_nom = np.broadcast_to(np.asarray(g_nom, dtype=np.float64), (K,)).copy()
        self.m_spread = np.broadcast_to(np.asarray(m_spread, dtype=np.float64), (K,)).copy()
        self.g_spread = np.broadcast_to(np.asarray(g_spread, dtype=np.float64), (K,)).copy()
        self.c_range = c_range
        self.thr = np.array([threshold(c, masses) for c in self.channel])

    @classmethod
    def wide(cls, channel, masses=DAUGHTER_MASSES):
        mc, gc = 0.5 * sum(M_RANGE), 0.5 * sum(G_RANGE)
        return cls(channel, mc, gc, 0.5 * (M_RANGE[1] - M_RANGE[0]) / mc,
                   0.5 * (G_RANGE[1] - G_RANGE[0]) / gc, C_RANGE, masses)

    def draw(self, rng):
        th = np.empty(4 * len(self.channel))
        for k in range(len(self.channel)):
            m = self.m_nom[k] * (1.0 + rng.uniform(-self.m_spread[k], self.m_spread[k]))
            while m < self.thr[k] + 0.02:
                m = self.m_nom[k] * (1.0 + rng.uniform(-self.m_spread[k], self.m_spread[k]))
            g = self.g_nom[k] * (1.0 + rng.uniform(-self.g_spread[k], self.g_spread[k]))
            mag, ph = rng.uniform(*self.c_range), rng.uniform(0.0, 2.0 * np.pi)
            th[4 * k:4 * k + 4] = (mag * np.cos(ph), mag * np.sin(ph), m, g)
        return th

    def code(self, m, g):
        return (m / self.m_nom - 1.0) / self.m_spread, (g / self.g_nom - 1.0) / self.g_spread

    def uncode(self, ym, yg):
        return self.m_nom * (1.0 + self.m_spread * ym), self.g_nom * (1.0 + self.g_spread * yg)


def draw_start(channel, rng, masses=DAUGHTER_MASSES):
    """A random start from the wide prior."""
    return Prior.wide(channel, masses).draw(rng)


class StartCoder:
    """Canonical form and the affine coding of parameter vectors: couplings
    rotated and scaled as described above, M and Gamma by the prior's
    nominal values and spreads (the prior's range maps onto [-1, 1])."""

    def __init__(self, channel, spin, prior=None, masses=DAUGHTER_MASSES):
        self.channel, self.spin = list(channel), list(spin)
        self.K = len(channel)
        self.P = 4 * self.K
        self.prior = prior if prior is not None else Prior.wide(channel, masses)
        groups = {}
        for k, key in enumerate(zip(channel, spin)):
            groups.setdefault(key, []).append(k)
        self.groups = [g for g in groups.values() if len(g) > 1]
        self.thr = np.array([threshold(c, masses) for c in channel])

    def canonical(self, theta):
        th = np.asarray(theta, dtype=np.float64).reshape(self.K, 4).copy()
        for g in self.groups:
            # interchangeable resonances: the k-th lightest takes the slot of
            # the k-th lightest nominal mass (by mass alone for equal nominals)
            by_mass = sorted(g, key=lambda k: th[k, 2])
            slots = sorted(g, key=lambda k: self.prior.m_nom[k])
            th[slots] = th[by_mass]
        c = th[:, 0] + 1j * th[:, 1]
        if abs(c[0]) > 0:
            c = c * np.exp(-1j * np.angle(c[0]))
        rms = np.sqrt(np.mean(np.abs(c) ** 2))
        if rms > 0:
            c = c / rms
        th[:, 0], th[:, 1] = c.real, c.imag
        return th.reshape(-1)

    def encode(self, theta):
        th = self.canonical(theta).reshape(self.K, 4)
        y = th.copy()
        y[:, 2], y[:, 3] = self.prior.code(th[:, 2], th[:, 3])
        return y.reshape(-1)

    def decode(self, y):
        y = np.asarray(y, dtype=np.float64).reshape(self.K, 4)
        th = y.copy()
        th[:, 2], th[:, 3] = self.prior.uncode(y[:, 2], y[:, 3])
        th[:, 2] = np.maximum(th[:, 2], self.thr + 0.02)
        th[:, 3] = np.maximum(th[:, 3], 0.25 * self.prior.g_nom * (1.0 - self.prior.g_spread) + 1e-3)
        c = th[:, 0] + 1j * th[:, 1]
        c = np.where(np.abs(c) > 1e-3, c, 1e-3)    # keep every coupling alive
        th[:, 0], th[:, 1] = c.real, c.imag
        return th.reshape(-1)


def histograms(s12, s13, offsets, parent=PARENT_MASS, masses=DAUGHTER_MASSES):
    """Normalised 32 x 32 Dalitz histograms of event sets (pwa_hist2d).
    s12, s13: FP64 device tensors; offsets: n_sets + 1 int64 boundaries."""
    lib = L.load()
    s12 = s12.to(dtype=torch.float64).contiguous()
    s13 = s13.to(dtype=torch.float64).contiguous()
    off = torch.as_tensor(offsets, dtype=torch.int64, device=s12.device).contiguous()
    n_sets = int(off.numel()) - 1
    out = torch.empty(n_sets, NBINS * NBINS, dtype=torch.float32, device=s12.device)
    m = (ctypes.c_double * 3)(*masses)
    L.check("pwa_hist2d", lib.pwa_hist2d(_ptr(s12), _ptr(s13), _ptr(off), n_sets, parent, m,
                                         _ptr(out), _stream()))
    return out


class MLP:
    """n_in -> n_h1 -> n_h2 -> n_out with GELU, trained with Adam in bf16 on
    the matrix cores (FP32 master weights and moments)."""

    def __init__(self, dims=(1024, 512, 512, 48), seed=0, device="cuda"):
        self.lib = L.load()
        self.dims = L.PwaMlpDims(*dims)
        self.n_in, self.n_h1, self.n_h2, self.n_out = dims
        self.device = torch.device(device)
        n = int(self.lib.pwa_mlp_n_params(ctypes.byref(self.dims)))
        if n == 0:
            raise ValueError("layer widths n_in, n_h1, n_h2 must be multiples of 16")
        self.n_params = n
        g = torch.Generator(device="cpu")
        g.manual_seed(seed)
        parts = []
        for fan_out, fan_in, gain in ((self.n_h1, self.n_in, 2.0), (self.n_h2, self.n_h1, 2.0),
                                      (self.n_out, self.n_h2, 1.0)):
            parts.append(torch.randn(fan_out * fan_in, generator=g) * np.sqrt(gain / fan_in))
            parts.append(torch.zeros(fan_out))
        self.w = torch.cat(parts).to(device=self.device, dtype=torch.float32).contiguous()
        assert self.w.numel() == n
        self.m = torch.zeros_like(self.w)
        self.v = torch.zeros_like(self.w)
        self.wbf = torch.empty(n, dtype=torch.int16, device=self.device)
        nt = int(self.lib.pwa_mlp_n_transposed(ctypes.byref(self.dims)))
        self.wtbf = torch.empty(nt, dtype=torch.int16, device=self.device)
        self.step = 0
        self._ws, self._ws_batch = None, 0
        self.cast()

    def save(self, path, **meta):
        """FP32 master weights, the layer widths and `meta` (numbers, arrays
        or strings) to an .npz file."""
        np.savez_compressed(path, w=self.w.cpu().numpy(),
                            dims=np.array([self.n_in, self.n_h1, self.n_h2, self.n_out]),
                            **{k: np.asarray(v) for k, v in meta.items()})

    @classmethod
    def load(cls, path, device="cuda"):
        """(network, meta dict) from a file written by save."""
        d = np.load(path, allow_pickle=False)
        net = cls(tuple(int(x) for x in d["dims"]), device=device)
        w = torch.as_tensor(d["w"], dtype=torch.float32, device=net.device)
        if w.numel() != net.n_params:
            raise ValueError("weight file does not match the layer widths")
        net.w.copy_(w)
        net.cast()
        return net, {k: d[k] for k in d.files if k not in ("w", "dims")}

    def cast(self):
        L.check("pwa_mlp_cast", self.lib.pwa_mlp_cast(ctypes.byref(self.dims), _ptr(self.w),
                                                      _ptr(self.wbf), _ptr(self.wtbf), _stream()))

    def _workspace(self, batch):
        nb = int(self.lib.pwa_mlp_workspace_bytes(ctypes.byref(self.dims), batch))
        if self._ws is None or self._ws.numel() < nb + 256:
            self._ws = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
        off = (-self._ws.data_ptr()) % 256
        return ctypes.c_void_p(self._ws.data_ptr() + off), nb

    def forward(self, x):
        x = torch.as_tensor(x, dtype=torch.float32, device=self.device).contiguous()
        B = int(x.shape[0])
        ws, nb = self._workspace(B)
        y = torch.empty(B, self.n_out, dtype=torch.float32, device=self.device)
        L.check("pwa_mlp_forward", self.lib.pwa_mlp_forward(
            ctypes.byref(self.dims), _ptr(self.w), _ptr(self.wbf), _ptr(x), B, _ptr(y), ws, nb,
            _stream()))
        return y

    def loss_grad(self, x, t):
        """Loss (FP64 scalar tensor) and gradient (packed FP32) on a batch."""
        x = torch.as_tensor(x, dtype=torch.float32, device=self.device).contiguous()
        t = torch.as_tensor(t, dtype=torch.float32, device=self.device).contiguous()
        y = self.forward(x)
        B = int(x.shape[0])
        ws, nb = self._workspace(B)
        grad = torch.empty_like(self.w)
        loss = torch.empty(1, dtype=torch.float64, device=self.device)
        L.check("pwa_mlp_backward", self.lib.pwa_mlp_backward(
            ctypes.byref(self.dims), _ptr(self.wtbf), _ptr(y), _ptr(t), B, ws, nb, _ptr(grad),
            _ptr(loss), _stream()))
        return loss[0], grad

    def adam(self, grad, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
        self.step += 1
        L.check("pwa_mlp_adam", self.lib.pwa_mlp_adam(
            ctypes.byref(self.dims), _ptr(self.w), _ptr(self.m), _ptr(self.v), _ptr(grad),
            self.step, lr, beta1, beta2, eps, weight_decay, _ptr(self.wbf), _ptr(self.wtbf),
            _stream()))

    def loss(self, x, t):
        """Mean-squared error of the network on (x, t) (forward only)."""
        t = torch.as_tensor(t, dtype=torch.float32, device=self.device)
        return float(((self.forward(x) - t) ** 2).mean())

    def train(self, x, t, epochs=100, batch=256, lr=1e-3, seed=0, lr_end=None,
              weight_decay=0.0, x_val=None, t_val=None):
        """Mini-batch Adam over (x, t); returns the per-epoch mean losses.
        With a validation set, the weights of the epoch with the lowest
        validation loss are kept (early stopping)."""
        x = torch.as_tensor(x, dtype=torch.float32, device=self.device)
        t = torch.as_tensor(t, dtype=torch.float32, device=self.device)
        n = int(x.shape[0])
        g = torch.Generator(device="cpu")
        g.manual_seed(seed)
        hist = []
        self.val_history = []
        best = (float("inf"), None)
        for ep in range(epochs):
            rate = lr if lr_end is None else lr * (lr_end / lr) ** (ep / max(1, epochs - 1))
            perm = torch.randperm(n, generator=g).to(self.device)
            tot = []
            for i in range(0, n - batch + 1 if n >= batch else 1, batch):
                idx = perm[i:i + batch]
                loss, grad = self.loss_grad(x[idx], t[idx])
                self.adam(grad, lr=rate, weight_decay=weight_decay)
                tot.append(loss)
            hist.append(float(torch.stack(tot).mean()))
            if x_val is not None:
                v = self.loss(x_val, t_val)
                self.val_history.append(v)
                if v < best[0]:
                    best = (v, self.w.clone())
        if best[1] is not None:
            self.w.copy_(best[1])
            self.cast()
        return hist


# ---------------------------------------------------------------------------
# Toy fits: training data and evaluation.
# ---------------------------------------------------------------------------
def fit(lik, start, xtol=1e-6, maxiter=100, time_cap_s=5.0):
    th, rep = lik.fit(start, xtol=xtol, maxiter=maxiter, time_cap_s=time_cap_s,
                      forcing="relative")
    return th.cpu().numpy(), rep


class ToyStudy:
    """Toys of one resonance layout with a shared MC sample."""

    def __init__(self, channel, spin, n_mc, prior=None, seed=0, device="cuda", mc=None):
        self.channel, self.spin = list(channel), list(spin)
        self.prior = prior if prior is not None else Prior.wide(channel)
        self.coder = StartCoder(channel, spin, self.prior)
        self.gen = torch.Generator(device=device)
        self.gen.manual_seed(seed)
        self.rng = np.random.Generator(np.random.PCG64(seed))
        self.toys = ToyGenerator(channel, spin, batch=1 << 19, scan=1 << 18, device=device)
        if mc is None:
            from .toys import uniform_dalitz
            mc = uniform_dalitz(n_mc, self.gen, device=device)
        self.mc = mc
        self.device = device

    def toy(self, n_events):
        """(true canonical theta, events) of one toy."""
        th = self.coder.canonical(self.prior.draw(self.rng))
        ev = self.toys.draw(th, n_events, self.gen)
        return th, ev

    def likelihood(self, ev):
        lik = Likelihood(self.channel, self.spin, device=self.device)
        return lik.bind(ev[0], ev[1], self.mc[0], self.mc[1])

    @staticmethod
    def transform(h):
        """Network input from normalised histograms: the square root of the
        density scaled by the bin count (a flat distribution over the box
        gives 1 per bin; the square root evens out the Poisson noise of the
        bins)."""
        return torch.sqrt(h * float(NBINS * NBINS))

    def features(self, ev, n_events):
        """Network input of one event set."""
        return self.transform(histograms(ev[0], ev[1], [0, n_events]))

    def resampled_features(self, ev, n_events, n_rep):
        """Features of n_rep bootstrap resamples of one event set (the
        statistical fluctuation of a toy of the same size), for augmentation."""
        idx = torch.randint(0, n_events, (n_rep * n_events,), generator=self.gen,
                            device=ev[0].device)
        off = torch.arange(0, n_rep + 1, dtype=torch.int64, device=ev[0].device) * n_events
        return self.transform(histograms(ev[0][idx], ev[1][idx], off))

    def training_set(self, n_toys, n_events, log_every=0, label_bound=4.0, n_rep=0):
        """Features and coded labels of toy fits started at the truth (the
        fit's best point, also when it stops before meeting xtol).  A coded
        mass or width beyond +-label_bound (a resonance the toy does not
        constrain wandering off) is clipped to it; a fit whose couplings end
        beyond it is left out.  With n_rep > 0, each toy also contributes n_rep
        bootstrap resamples of its events with the same label; the toy index
        of every row is returned so that a validation split can keep whole
        toys apart."""
        hs, ys, ids = [], [], []
        t0 = time.time()
        for i in range(n_toys):
            th, ev = self.toy(n_events)
            lik = self.likelihood(ev)
            th_fit, rep = fit(lik, th)
            if not np.all(np.isfinite(th_fit)) or not np.isfinite(rep["nll"]):
                continue
            y = self.coder.encode(th_fit).reshape(-1, 4)
            if np.max(np.abs(y[:, :2])) > label_bound:
                continue
            y[:, 2:] = np.clip(y[:, 2:], -label_bound, label_bound)
            y = y.reshape(-1)
            f = self.features(ev, n_events)
            if n_rep:
                f = torch.cat([f, self.resampled_features(ev, n_events, n_rep)])
            hs.append(f)
            ys.extend([y] * int(f.shape[0]))
            ids.extend([i] * int(f.shape[0]))
            if log_every and (i + 1) % log_every == 0:
                print(f"[learned-start] {i + 1}/{n_toys} toy fits, {time.time() - t0:.1f} s",
                      flush=True)
        x = torch.cat(hs)
        y = torch.as_tensor(np.stack(ys), dtype=torch.float32, device=self.device)
        return x, y, np.asarray(ids)

    def propose(self, net, hists):
        y = net.forward(hists).cpu().numpy().astype(np.float64)
        return [self.coder.decode(r) for r in y]

    def evaluate(self, net, n_toys, n_events, n_random, tol=0.01, log_every=0, blind=None):
        """(summary, rows) of evaluate_rows on n_toys toys."""
        rows = self.evaluate_rows(net, n_toys, n_events, n_random, tol, log_every, blind)
        return summarize(rows, n_events, n_random, tol), rows

    def evaluate_rows(self, net, n_toys, n_events, n_random, tol=0.01, log_every=0, blind=None,
                      net_lock=None):
        """Proposal-started fits against random multi-start on held-out toys.

        Per toy, NLL_min is the lowest NLL of all its fits (from the truth,
        the proposal, the blind start and every random start); a fit
        succeeds when its NLL is within `tol` of it.  Random multi-start is
        priced as the expected cost until its first success over a random
        order of its starts (failures before the first success count in
        full); a single-start strategy (the proposal, or the blind start
        `blind` -- one fixed start that ignores the data, e.g. the decoded
        mean training label) costs its own fit plus, when that fails, the
        random strategy's expected cost.  One row per toy.  With net_lock
        (workers sharing one network), the proposal is taken under it."""
        rows = []
        t0 = time.time()
        for i in range(n_toys):
            th, ev = self.toy(n_events)
            lik = self.likelihood(ev)
            feats = self.features(ev, n_events)
            if net_lock is None:
                start = self.propose(net, feats)[0]
            else:
                with net_lock:   # the network's workspace is shared
                    start = self.propose(net, feats)[0]
            fits = {"truth": fit(lik, th), "proposal": fit(lik, start)}
            if blind is not None:
                fits["blind"] = fit(lik, blind)
            rnd = [fit(lik, self.prior.draw(self.rng)) for _ in range(n_random)]
            nlls = [f[1]["nll"] for f in list(fits.values()) + rnd]
            nmin = min(x for x in nlls if np.isfinite(x))
            ok = lambda rep: np.isfinite(rep["nll"]) and rep["nll"] <= nmin + tol  # noqa: E731
            succ = [ok(r[1]) for r in rnd]
            S = sum(succ)

            def expected(key):
                costs = [r[1][key] for r in rnd]
                if S == 0:
                    return float(sum(costs)), False
                fail = sum(c for c, s in zip(costs, succ) if not s)
                good = sum(c for c, s in zip(costs, succ) if s)
                return fail / (S + 1) + good / S, True

            row = {"random_success_fraction": S / max(1, n_random)}
            for name in ("proposal", "blind"):
                if name not in fits:
                    continue
                s_ok = ok(fits[name][1])
                row[f"{name}_success"] = bool(s_ok)
                for key in ("iterations", "seconds"):
                    e_rnd, found = expected(key)
                    row[f"random_{key}"] = e_rnd
                    row["random_found"] = found
                    row[f"{name}_{key}"] = fits[name][1][key] + (0.0 if s_ok else e_rnd)
            rows.append(row)
            if log_every and (i + 1) % log_every == 0:
                print(f"[learned-start] evaluated {i + 1}/{n_toys} toys, {time.time() - t0:.1f} s",
                      flush=True)
        return rows


def summarize(rows, n_events, n_random, tol):
    """Success rates, expected costs, the paired proposal-vs-blind comparison
    and 95% intervals over the evaluation rows."""
    n_toys = len(rows)
    summary = {
        "toys": n_toys, "events_per_toy": n_events, "random_starts": n_random, "tol": tol,
        "random_start_success_rate": float(np.mean([r["random_success_fraction"] for r in rows])),
        "random_found_fraction": float(np.mean([r["random_found"] for r in rows])),
        "mean_iterations_random_strategy": float(np.mean([r["random_iterations"] for r in rows])),
        "mean_seconds_random_strategy": float(np.mean([r["random_seconds"] for r in rows])),
    }
    for name in ("proposal", "blind"):
        if f"{name}_success" in rows[0]:
            summary[f"{name}_success_rate"] = float(np.mean([r[f"{name}_success"] for r in rows]))
            summary[f"mean_iterations_{name}_strategy"] = float(np.mean([r[f"{name}_iterations"] for r in rows]))
            summary[f"mean_seconds_{name}_strategy"] = float(np.mean([r[f"{name}_seconds"] for r in rows]))
    if "blind_success" in rows[0]:
        summary["proposal_vs_blind"] = paired_comparison(rows, "proposal", "blind")
    if "proposal_success" in rows[0]:
        summary["proposal_vs_random"] = paired_costs(rows, "proposal", "random")
    # 95% intervals: Wilson for the success rates (the random rate pools
    # every random start), mean +- 1.96 standard errors for the costs
    n = len(rows)
    summary["ci95"] = {
        "random_start_success_rate": wilson_interval(
            round(summary["random_start_success_rate"] * n * n_random), n * n_random),
        "mean_iterations_random_strategy": mean_interval([r["random_iterations"] for r in rows])}
    for name in ("proposal", "blind"):
        if f"{name}_success" in rows[0]:
            summary["ci95"][f"{name}_success_rate"] = wilson_interval(
                sum(r[f"{name}_success"] for r in rows), n)
            summary["ci95"][f"mean_iterations_{name}_strategy"] = mean_interval(
                [r[f"{name}_iterations"] for r in rows])
    return summary


def split_counts(n, parts):
    """n items over `parts` workers, as even as possible."""
    return [n // parts + (1 if w < n % parts else 0) for w in range(parts)]


def run_workers(n_workers, make_study, work):
    """work(study, w) for w = 0 .. n_workers-1, each in a host thread of its
    own with its own HIP stream (default priority) and its own ToyStudy
    (make_study(w), built on that stream).  The library's calls release the
    interpreter lock, so the workers' fits -- many small kernels and host
    round trips each -- overlap on the GPU.  Returns the results in worker
    order; tensors in them may be used on the caller's stream."""
    main = torch.cuda.current_stream()
    main.synchronize()   # inputs shared by the workers (the MC sample) are ready
    results, errors = [None] * n_workers, []

    def run(w):
        try:
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                results[w] = work(make_study(w), w)
            st.synchronize()
        except BaseException as e:   # re-raised in the caller
            errors.append(e)

    threads = [threading.Thread(target=run, args=(w,)) for w in range(n_workers)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    if errors:
        raise errors[0]
    for res in results:
        for x in (res if isinstance(res, tuple) else ()):
            if isinstance(x, torch.Tensor) and x.is_cuda:
                x.record_stream(main)
    return results


def parallel_training_set(channel, spin, prior, mc, n_toys, n_events, n_workers, seed, n_rep=0,
                          log_every=0):
    """ToyStudy.training_set over n_workers workers (toy streams seeded
    seed * 1000 + w), merged with the toy index made unique per worker."""
    counts = split_counts(n_toys, n_workers)
    res = run_workers(
        n_workers,
        lambda w: ToyStudy(channel, spin, 0, prior=prior, seed=seed * 1000 + w, mc=mc),
        lambda st, w: st.training_set(counts[w], n_events, log_every=log_every, n_rep=n_rep))
    off = np.cumsum([0] + counts)
    x = torch.cat([r[0] for r in res])
    y = torch.cat([r[1] for r in res])
    ids = np.concatenate([r[2] + off[w] for w, r in enumerate(res)])
    return x, y, ids


def parallel_evaluate(channel, spin, prior, mc, net, n_toys, n_events, n_random, n_workers, seed,
                      blind=None, tol=0.01, log_every=0):
    """ToyStudy.evaluate over n_workers workers (toy streams seeded
    seed * 1000 + w); (summary, rows)."""
    counts = split_counts(n_toys, n_workers)
    lock = threading.Lock()
    res = run_workers(
        n_workers,
        lambda w: ToyStudy(channel, spin, 0, prior=prior, seed=seed * 1000 + w, mc=mc),
        lambda st, w: st.evaluate_rows(net, counts[w], n_events, n_random, tol, log_every, blind,
                                       net_lock=lock))
    rows = [r for part in res for r in part]
    return summarize(rows, n_events, n_random, tol), rows


def wilson_interval(k, n, z=1.959963984540054):
    """Wilson score interval for a binomial proportion k / n."""
    if n == 0:
        return [0.0, 1.0]
    p = k / n
    den = 1.0 + z * z / n
    c = (p + z * z / (2 * n)) / den
    h = z * math.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / den
    return [max(0.0, c - h), min(1.0, c + h)]


def mean_interval(x, z=1.959963984540054):
    """Mean +- z standard errors."""
    x = np.asarray(x, dtype=np.float64)
    m = float(np.mean(x))
    se = float(np.std(x, ddof=1) / math.sqrt(len(x))) if len(x) > 1 else float("inf")
    return [m - z * se, m + z * se]


def sign_test(n_a, n_b):
    """Two-sided exact sign test on n_a + n_b discordant pairs (n_a where
    only the first strategy succeeds, n_b where only the second does)."""
    n = n_a + n_b
    if n == 0:
        return 1.0
    k = min(n_a, n_b)
    tail = sum(math.comb(n, j) for j in range(k + 1)) / 2.0 ** n
    return min(1.0, 2.0 * tail)


def paired_comparison(rows, a, b):
    """Per-toy comparison of two single-start strategies on the same toys:
    the discordant successes with an exact sign test, and the per-toy
    difference of expected Newton iterations to the global minimum with a
    Wilcoxon signed-rank test (scipy)."""
    sa = np.array([r[f"{a}_success"] for r in rows], dtype=bool)
    sb = np.array([r[f"{b}_success"] for r in rows], dtype=bool)
    n_a, n_b = int(np.sum(sa & ~sb)), int(np.sum(~sa & sb))
    d = np.array([r[f"{a}_iterations"] - r[f"{b}_iterations"] for r in rows], dtype=np.float64)
    p_w = 1.0
    if np.any(d != 0):
        from scipy.stats import wilcoxon
        p_w = float(wilcoxon(d, zero_method="wilcox", alternative="two-sided").pvalue)
    return {"toys": len(rows), "both": int(np.sum(sa & sb)), "neither": int(np.sum(~sa & ~sb)),
            f"only_{a}": n_a, f"only_{b}": n_b, "sign_test_p": sign_test(n_a, n_b),
            "mean_iteration_difference": float(np.mean(d)),
            "median_iteration_difference": float(np.median(d)), "wilcoxon_p": p_w}


def paired_costs(rows, a, b):
    """Per-toy difference of the expected Newton iterations and seconds to
    the global minimum of strategy a minus strategy b (e.g. the proposal
    strategy against random multi-start), with Wilcoxon signed-rank tests."""
    out = {"toys": len(rows)}
    for key in ("iterations", "seconds"):
        d = np.array([r[f"{a}_{key}"] - r[f"{b}_{key}"] for r in rows], dtype=np.float64)
        p_w = 1.0
        if np.any(d != 0):
            from scipy.stats import wilcoxon
            p_w = float(wilcoxon(d, zero_method="wilcox", alternative="two-sided").pvalue)
        out[f"mean_{key}_difference"] = float(np.mean(d))
        out[f"median_{key}_difference"] = float(np.median(d))
        out[f"{key}_wilcoxon_p"] = p_w
    out[f"toys_{a}_cheaper"] = int(sum(r[f"{a}_iterations"] < r[f"{b}_iterations"] for r in rows))
    return out


DATA = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")


def load_proposal(path=None, device="cuda"):
    """A trained start proposal: (network, prior, blind start, metadata).
    The default is the K = 12 network shipped in data/ (trained by this
    module's main() on 18000 toy fits of 50k events; see its metadata)."""
    net, meta = MLP.load(path or os.path.join(DATA, "start_proposal_k12.npz"), device=device)
    K = int(meta["K"])
    ch, _ = resonance_layout(K)
    prior = Prior(ch, meta["m_nom"], meta["g_nom"], meta["m_spread"], meta["g_spread"],
                  tuple(float(c) for c in meta["c_range"]))
    return net, prior, np.asarray(meta["blind"], dtype=np.float64), meta


def resonance_layout(K):
    """Resonance k in channel k mod 3 with spin floor(k / 3) mod 3."""
    return [k % 3 for k in range(K)], [(k // 3) % 3 for k in range(K)]


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description="Train and evaluate the start-point proposal")
    ap.add_argument("--K", type=int, default=12)
    ap.add_argument("--train", type=int, default=2000, help="training toys")
    ap.add_argument("--events", type=int, default=20000, help="events per training toy")
    ap.add_argument("--mc", type=int, default=200000)
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--rep", type=int, default=4, help="bootstrap resamples per training toy")
    ap.add_argument("--wd", default="1e-4", help="decoupled weight decay; a comma-separated "
                    "list trains one network per value and keeps the lowest validation loss")
    ap.add_argument("--val", type=float, default=0.1, help="fraction of toys held for validation")
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--eval", type=int, default=40, help="held-out toys")
    ap.add_argument("--eval-events", type=int, default=100000)
    ap.add_argument("--random", type=int, default=32, help="random starts per held-out toy")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--m-spread", type=float, default=0.03,
                    help="relative mass spread around the nominal masses (0: wide prior)")
    ap.add_argument("--g-spread", type=float, default=0.2, help="relative width spread")
    ap.add_argument("--out", default="")
    ap.add_argument("--save-net", default="", help="save the trained network and its prior "
                    "to this .npz")
    ap.add_argument("--save-set", default="", help="save the training features (one row per "
                    "toy, float16) and labels to this .npz")
    ap.add_argument("--threads", type=int, default=1, help="host threads (each with its own "
                    "HIP stream) running toy fits side by side; 1 keeps the single-stream order")
    ap.add_argument("--evaluate-shipped", action="store_true",
                    help="only evaluate the shipped proposal (data/) on --eval fresh toys of "
                    "--eval-events events, seeded by --seed")
    ap.add_argument("--net", default="", help="with --evaluate-shipped: evaluate this saved "
                    "network (.npz from --save-net) instead of the shipped one")
    a = ap.parse_args(argv)
    if a.threads < 1:
        ap.error("--threads must be at least 1")

    def shared_mc(seed):
        from .toys import uniform_dalitz
        g = torch.Generator(device="cuda")
        g.manual_seed(seed)
        return uniform_dalitz(a.mc, g)

    def evaluate(ch, sp, prior, net, blind, seed, log_every):
        if a.threads == 1:
            ev = ToyStudy(ch, sp, a.mc, prior=prior, seed=seed)
            return ev.evaluate(net, a.eval, a.eval_events, a.random, log_every=log_every,
                               blind=blind)
        return parallel_evaluate(ch, sp, prior, shared_mc(seed), net, a.eval, a.eval_events,
                                 a.random, a.threads, seed, blind=blind, log_every=log_every)

    if a.evaluate_shipped:
        net, prior, blind, meta = load_proposal(a.net or None)
        ch, sp = resonance_layout(int(meta["K"]))
        summary, rows = evaluate(ch, sp, prior, net, blind, a.seed,
                                 max(1, min(10, a.eval // (10 * a.threads))))
        print(json.dumps(summary), flush=True)
        if a.out:
            with open(a.out, "w") as f:
                json.dump({"summary": summary, "rows": rows}, f, indent=1)
        return summary
    ch, sp = resonance_layout(a.K)
    if a.m_spread > 0:
        # the analysis model: nominal masses and widths drawn once from the wide prior
        nom = Prior.wide(ch).draw(np.random.Generator(np.random.PCG64(a.seed + 7)))
        prior = Prior(ch, nom[2::4], nom[3::4], a.m_spread, a.g_spread)
    else:
        prior = Prior.wide(ch)
    t0 = time.time()
    study = ToyStudy(ch, sp, a.mc, prior=prior, seed=a.seed)
    if a.threads == 1:
        x, y, ids = study.training_set(a.train, a.events, log_every=max(1, min(50, a.train // 10)),
                                       n_rep=a.rep)
    else:
        x, y, ids = parallel_training_set(ch, sp, prior, study.mc, a.train, a.events, a.threads,
                                          a.seed, n_rep=a.rep,
                                          log_every=max(1, min(200, a.train // (10 * a.threads))))
    t_data = time.time() - t0
    if a.save_set:
        first = np.concatenate([[True], ids[1:] != ids[:-1]])
        np.savez_compressed(a.save_set, x=x[torch.as_tensor(first, device=x.device)].cpu().numpy().astype(np.float16),
                            y=y[torch.as_tensor(first, device=y.device)].cpu().numpy(), toy=ids[first])
    toys = np.unique(ids)
    n_val = int(round(a.val * len(toys)))
    val_toys = set(np.random.Generator(np.random.PCG64(a.seed)).choice(toys, n_val, replace=False))
    is_val = torch.as_tensor([i in val_toys for i in ids], device=x.device)
    xv, yv = x[is_val], y[is_val]
    x, y = x[~is_val], y[~is_val]
    yc = y.cpu().numpy()
    print(f"[learned-start] {x.shape[0]} labels: mean |y| {np.mean(np.abs(yc)):.3f}, "
          f"std {yc.std():.3f}, max |y| {np.max(np.abs(yc)):.3f}", flush=True)
    t1 = time.time()
    best = None
    for wd in [float(w) for w in str(a.wd).split(",")]:
        cand = MLP((NBINS * NBINS, 512, 512, 4 * a.K), seed=a.seed)
        losses = cand.train(x, y, epochs=a.epochs, batch=min(a.batch, int(x.shape[0])), lr=a.lr,
                            lr_end=a.lr * 0.05, seed=a.seed, weight_decay=wd,
                            x_val=xv if n_val else None, t_val=yv if n_val else None)
        vh = cand.val_history
        vbest = min(vh) if vh else float("nan")
        print(f"[learned-start] weight decay {wd:g}: loss {losses[0]:.4f} -> {losses[-1]:.4f}; "
              f"validation {vh[0] if vh else float('nan'):.4f} -> best {vbest:.4f} "
              f"(epoch {int(np.argmin(vh)) + 1 if vh else 0})", flush=True)
        if best is None or (vh and vbest < best[0]):
            best = (vbest, wd, cand, losses, vh)
    _, wd_best, net, losses, vh = best
    torch.cuda.synchronize()
    t_train = time.time() - t1
    blind = study.coder.decode(y.mean(0).cpu().numpy().astype(np.float64))
    if a.save_net:
        net.save(a.save_net, K=a.K, blind=blind, m_nom=prior.m_nom, g_nom=prior.g_nom, m_spread=prior.m_spread,
                 g_spread=prior.g_spread, c_range=np.asarray(prior.c_range),
                 train_toys=int(len(toys) - n_val), train_events=a.events, mc=a.mc,
                 val_loss_best=min(vh) if vh else np.nan, seed=a.seed)
    if a.eval > 0:
        summary, _ = evaluate(ch, sp, prior, net, blind, a.seed + 1000,
                              max(1, min(5, a.eval // (10 * a.threads))))
    else:
        summary = {}
    summary.update({"K": a.K, "m_spread": a.m_spread, "g_spread": a.g_spread, "weight_decay": wd_best, "train_toys": int(len(toys) - n_val), "val_toys": n_val,
                    "train_rows": int(x.shape[0]), "train_events": a.events, "mc": a.mc,
                    "epochs": a.epochs, "loss_first_epoch": losses[0], "loss_last_epoch": losses[-1],
                    "val_loss_first_epoch": vh[0] if vh else None,
                    "val_epoch_best": int(np.argmin(vh)) + 1 if vh else None,
                    "val_loss_best": min(vh) if vh else None,
                    "seconds_training_set": round(t_data, 1), "seconds_training": round(t_train, 1)})
    print(json.dumps(summary), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(summary, f, indent=1)


if __name__ == "__main__":
    main()

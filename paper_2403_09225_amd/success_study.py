"""Fit-success study of random multi-start Newton-CG (and of the
gradient-only BFGS comparator) on a synthetic model.

The paper's central experiment (Sec. 3) fits one data sample from 300
random starting points and counts how often a fit reaches the global
minimum: a fit succeeds if its -ln L is within 1 of the lowest value found.
It finds the success rate of Newton-CG rising from a few per cent at
xtol = 1e-5 to about a third at xtol = 1e-8, and caps each fit's wall time
(early stopping) at little cost in success.

Here the same study runs on a model of this library's family: K resonances
(channel k mod 3, spin floor(k/3) mod 3), one data sample drawn from the
model on the GPU, a uniform MC sample, random starts from the wide prior
(M in [0.6, 1.6] GeV, Gamma in [0.03, 0.3] GeV, |c| in [0.2, 1], uniform
phase) and `pwa_fit` at each xtol with a wall-time cap; the same starts are
fitted by `pwa_fit_bfgs`, the gradient-only arm of the paper's comparison.
The lowest NLL is taken over every fit and a fit from the generating point.

    python -m paper_2403_09225_amd.success_study --K 6 --events 10000 \\
        --mc 1000000 --starts 300 --xtol 1e-5 1e-8 --time-cap 10 --out study.json
"""

import sys
import time

import numpy as np
import torch

from .api import Likelihood
from .learned_start import Prior, resonance_layout
from .toys import ToyGenerator, uniform_dalitz


def run(K=6, n_events=10_000, n_mc=1_000_000, n_starts=300, xtols=(1e-5, 1e-8), time_cap_s=10.0,
        maxiter=1000, forcing="scipy", tol=1.0, seed=0, log_every=0, device="cuda",
        precondition=False, early_caps=(0.05, 0.1, 0.2, 0.5, 1.0), methods=("newton-cg", "bfgs"),
        return_sample=False):
    """Run the study; returns (summary dict, per-fit rows dict of arrays) and,
    with return_sample, the (data, mc, truth, model layout) it fitted.
    methods: "newton-cg" (pwa_fit; rows "xtol_<x>") and the gradient-only
    comparator "bfgs" (pwa_fit_bfgs; rows "bfgs_xtol_<x>"), the two arms of
    the paper's comparison (Sec. 3: Newton-CG against gradient-only Migrad)."""
    ch, sp = resonance_layout(K)
    prior = Prior.wide(ch)
    rng = np.random.Generator(np.random.PCG64(seed))
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    truth = prior.draw(rng)
    data = ToyGenerator(ch, sp, device=device).draw(truth, n_events, gen)
    mc = uniform_dalitz(n_mc, gen, device=device)
    lik = Likelihood(ch, sp, device=device).bind(data[0], data[1], mc[0], mc[1])
    sample = None
    if return_sample:
        sample = ((data[0].cpu().numpy(), data[1].cpu().numpy()),
                  (mc[0].cpu().numpy(), mc[1].cpu().numpy()), truth, (ch, sp))
    del data, mc
    starts = np.stack([prior.draw(rng) for _ in range(n_starts)])

    _, rep_t = lik.fit(truth, xtol=1e-10, maxiter=maxiter, forcing="relative")
    nll_truth_fit = rep_t["nll"]
    rows = {"start": starts}
    t_all = time.perf_counter()
    for method, xt in [(m, x) for m in methods for x in xtols]:
        key = f"xtol_{xt:g}" if method == "newton-cg" else f"{method}_xtol_{xt:g}"
        nll = np.empty(n_starts)
        sec = np.empty(n_starts)
        it = np.empty(n_starts, dtype=np.int64)
        hvp = np.empty(n_starts, dtype=np.int64)
        code = np.empty(n_starts, dtype=np.int64)
        conv = np.empty(n_starts, dtype=np.int64)
        ngr = np.empty(n_starts, dtype=np.int64)
        ths = np.empty((n_starts, 4 * K))
        for i in range(n_starts):
            th_i, rep = lik.fit(starts[i], xtol=xt, maxiter=maxiter, time_cap_s=time_cap_s,
                                forcing=forcing, precondition=precondition, method=method)
            ths[i] = th_i.cpu().numpy()
            nll[i], sec[i], it[i] = rep["nll"], rep["seconds"], rep["iterations"]
            hvp[i], code[i], conv[i] = rep["n_hvp"], rep["code"], rep["converged"]
            ngr[i] = rep["n_grad"]
            if log_every and (i + 1) % log_every == 0:
                print(f"[study] {method} xtol {xt:g}: {i + 1}/{n_starts} fits, "
                      f"{time.perf_counter() - t_all:.1f} s", file=sys.stderr, flush=True)
        rows[key] = {"nll": nll, "seconds": sec, "iterations": it, "n_hvp": hvp,
                     "n_grad": ngr, "code": code, "converged": conv, "theta": ths}
    finite = [r["nll"][np.isfinite(r["nll"])] for k, r in rows.items() if k != "start"]
    nll_min = float(min([nll_truth_fit] + [float(f.min()) for f in finite if f.size]))
    summary = {"K": K, "n_par": 4 * K, "n_events": n_events, "n_mc": n_mc, "n_starts": n_starts,
               "time_cap_s": time_cap_s, "forcing": forcing, "precondition": bool(precondition),
               "tol": tol, "seed": seed,
               "nll_min": nll_min, "nll_truth_fit": nll_truth_fit,
               "truth_fit_is_global": bool(nll_truth_fit <= nll_min + tol)}
    for key, r in rows.items():
        if key == "start":
            continue
        ok = np.isfinite(r["nll"]) & (r["nll"] <= nll_min + tol)
        r["success"] = ok
        rate = float(ok.mean())
        mean_s = float(r["seconds"].mean())
        summary[key] = {
            "success_rate": rate,
            "n_success": int(ok.sum()),
            "mean_seconds": round(mean_s, 4),
            "median_seconds": round(float(np.median(r["seconds"])), 4),
            "max_seconds": round(float(r["seconds"].max()), 4),
            "mean_iterations": round(float(r["iterations"].mean()), 2),
            "mean_hvps": round(float(r["n_hvp"].mean()), 1),
            "mean_grads": round(float(r["n_grad"].mean()), 1),
            "converged_rate": float((r["converged"] == 1).mean()),
            "hit_time_cap": int(((r["converged"] != 1) & (r["seconds"] >= time_cap_s)).sum()),
            # random multi-start until the first success: expected fits
            # 1/p, each taking the mean time
            "expected_seconds_to_global": (round(mean_s / rate, 3) if rate > 0 else None),
        }
        # early stopping at a cap c, from the recorded times: the successes
        # that finished within c (a lower bound) and the capped mean time
        caps = {}
        for c in early_caps:
            ok_c = ok & (r["seconds"] <= c)
            t_c = float(np.minimum(r["seconds"], c).mean())
            caps[f"{c:g}s"] = {"success_rate": float(ok_c.mean()),
                               "mean_seconds": round(t_c, 4),
                               "expected_seconds_to_global":
                                   (round(t_c / ok_c.mean(), 3) if ok_c.any() else None)}
        summary[key]["early_stop"] = caps
    if return_sample:
        return summary, rows, sample
    return summary, rows


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description="Random multi-start Newton-CG success study")
    ap.add_argument("--K", type=int, default=6)
    ap.add_argument("--events", type=int, default=10_000)
    ap.add_argument("--mc", type=int, default=1_000_000)
    ap.add_argument("--starts", type=int, default=300)
    ap.add_argument("--xtol", type=float, nargs="+", default=[1e-5, 1e-8])
    ap.add_argument("--time-cap", type=float, default=10.0)
    ap.add_argument("--forcing", choices=["scipy", "relative"], default="scipy")
    ap.add_argument("--precondition", action="store_true",
                    help="CG preconditioned with |H|^-1 (pwa_fit_opts.precondition)")
    ap.add_argument("--methods", nargs="+", default=["newton-cg", "bfgs"],
                    choices=["newton-cg", "bfgs"])
    ap.add_argument("--tol", type=float, default=1.0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default="")
    a = ap.parse_args(argv)
    summary, rows = run(a.K, a.events, a.mc, a.starts, tuple(a.xtol), a.time_cap, forcing=a.forcing,
                        tol=a.tol, seed=a.seed, log_every=25, precondition=a.precondition,
                        methods=tuple(a.methods))
    text = json.dumps(summary)
    print(text, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text + "\n")
        flat = {"start": rows["start"]}
        for key, r in rows.items():
            if key != "start":
                for name, arr in r.items():
                    flat[f"{key}_{name}"] = arr
        np.savez(a.out.rsplit(".", 1)[0] + ".npz", **flat)


if __name__ == "__main__":
    main()

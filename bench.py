"""Benchmark of the PWA hot path on one MI355X.

    python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--no-fit] [--no-cpu]

Workload: the GPU-scale model -- K = 12 resonances over the channels (12),
(13), (23) with J in {0, 1, 2}, 1M data-like events and 5M uniform
phase-space MC events (synthetic, seeded), FP64.  One step is one fused
NLL + gradient + Hessian-vector-product evaluation over all 6M events (the
Newton-CG inner-loop call).  Inputs and the parameter-free event stream are
resident in HBM before timing starts.

Prints one JSON line with events/s, the roofline of the dominant kernel
(the per-event pass; timed by HIP events recorded on its stream), the CPU
oracle timed on a bounded sample, and Newton-CG time-to-minimum with FP64
and with mixed precision (FP32 HVPs inside CG).
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
HBM_PEAK_GBS = 8000.0


def hvp_flops_per_event(K, data_fraction):
    """Algorithmic FP64 flops of one fused NLL + gradient + HVP per event.

    Counted from the factorised amplitude (add, sub, mul = 1; a fused
    multiply-add = 2; reciprocal and logarithm = 1), with no recomputation:
    per resonance 55 for a, z, zdot; 48 for the four gradient terms; 126 for
    the second derivatives and four HVP terms: 229.  Per event: |z|^2 and the
    sum (4), plus for data events the log, reciprocal and weights (16)."""
    return 229.0 * K + 4.0 + 16.0 * data_fraction


def stream_bytes_per_event(n_planes, real_bytes=8):
    return n_planes * real_bytes


def make_workload():
    import synth
    W = synth.workload(1)
    mc = synth.uniform_phase_space(W.n_mc, synth.rng_for(1, synth.configs.STREAM_MC))
    data = synth.resonant_like(W.n_data, W.channel, W.theta_true,
                               synth.rng_for(1, synth.configs.STREAM_DATA))
    return W, data, mc


def cpu_baseline(W, data, mc, n_data=100_000, n_mc=500_000):
    """The oracle, as it is, on a bounded sample (same 1:5 data:MC mix)."""
    import oracle
    try:
        from threadpoolctl import threadpool_limits
        limiter = threadpool_limits(limits=1)
    except Exception:  # pragma: no cover
        limiter = None
    d = (data[0][:n_data], data[1][:n_data])
    m = (mc[0][:n_mc], mc[1][:n_mc])
    v = np.random.Generator(np.random.PCG64(5)).normal(size=W.n_par)
    t0 = time.perf_counter()
    oracle.hvp(d, m, W, W.theta_true, v)
    dt = time.perf_counter() - t0
    if limiter is not None:
        limiter.unregister()
    return {"value": (n_data + n_mc) / dt, "unit": "events/s", "cores": 1, "kind": "oracle",
            "sample": f"one NLL+grad+HVP of the oracle (NumPy FP64, single thread) over "
                      f"{n_data} data + {n_mc} MC events of the same workload; {dt:.2f} s",
            "host_cores_available": len(os.sched_getaffinity(0))}


def fit_compare(lik, W, cap_s=60.0):
    """Newton-CG time to minimum from a fixed start: FP64 HVPs vs FP32 HVPs
    (line search and convergence test in FP64 in both)."""
    import synth
    start = W.theta_true + synth.rng_for(1, synth.configs.STREAM_TEST).normal(
        scale=np.tile([0.02, 0.02, 0.002, 0.002], W.n_res))
    out = {}
    for prec in ("f64", "f32"):
        th, rep = lik.fit(start, xtol=1e-8, maxiter=200, time_cap_s=cap_s, hvp_precision=prec)
        out[prec] = {"seconds": round(rep["seconds"], 4), "nll": rep["nll"],
                     "iterations": rep["iterations"], "hvps": rep["n_hvp"],
                     "grads": rep["n_grad"], "converged": rep["converged"]}
    out["speedup_mixed_vs_fp64"] = round(out["f64"]["seconds"] / max(out["f32"]["seconds"], 1e-9), 3)
    out["nll_diff_mixed_minus_fp64"] = out["f32"]["nll"] - out["f64"]["nll"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-fit", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--precision", default="f64", choices=["f64", "f32"])
    ap.add_argument("--shape", default="", help="lanes_per_event,res_per_lane override")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build runs the likelihood on a single MI355X "
              "(multi-GPU sharding is described in DESIGN.md but not launched). Use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2403_09225_amd import Likelihood

    torch.cuda.set_device(0)
    W, data, mc = make_workload()
    print(f"[bench] workload ready: {W.n_data} data + {W.n_mc} MC events, K={W.n_res}",
          file=sys.stderr, flush=True)
    lik = Likelihood(W.channel, W.spin, streams=("f64", "f32"))
    lik.bind(data[0], data[1], mc[0], mc[1])
    if args.shape:
        lik.set_launch_shape(*[int(x) for x in args.shape.split(",")])
    lik.set_precision(args.precision)
    th = torch.tensor(W.theta_true, dtype=torch.float64, device="cuda")
    v = torch.tensor(np.random.Generator(np.random.PCG64(9)).normal(size=W.n_par),
                     dtype=torch.float64, device="cuda")
    for _ in range(args.warmup):
        lik.hvp(th, v)
    torch.cuda.synchronize()
    lik.set_kernel_timing(True)
    lik.kernel_time()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        lik.hvp(th, v)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    k_ms, k_n = lik.kernel_time()
    lik.set_kernel_timing(False)
    print(f"[bench] timed {args.steps} steps in {dt:.4f} s", file=sys.stderr, flush=True)

    n_ev = W.n_data + W.n_mc
    value = n_ev * args.steps / dt
    k_avg_s = k_ms / max(k_n, 1) / 1e3
    frac_d = W.n_data / n_ev
    flops = hvp_flops_per_event(W.n_res, frac_d) * n_ev
    n_planes = 18
    rbytes = 8 if args.precision == "f64" else 4
    bytes_launch = stream_bytes_per_event(n_planes, rbytes) * n_ev
    achieved = flops / k_avg_s / 1e12
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4), "traffic": None,
            "kernel": f"eval_kernel HVP ({args.precision})", "kernel_avg_us": round(k_avg_s * 1e6, 2),
            "algorithmic_flops_per_launch": flops, "algorithmic_bytes_per_launch": bytes_launch,
            "hbm_frac_at_algorithmic_bytes": round(bytes_launch / k_avg_s / 1e9 / HBM_PEAK_GBS, 4)}
    result = {
        "metric": "events/s for NLL+grad+HVP (one fused evaluation)",
        "value": round(value, 1), "unit": "events/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "f64" else "f32", "data": "synthetic",
        "config": {"workload": "K=12 resonances over (12),(13),(23), J in {0,1,2}; "
                               "1M data-like + 5M uniform MC events; Newton-CG HVP step",
                   "n_res": W.n_res, "n_data": W.n_data, "n_mc": W.n_mc,
                   "launch_shape": args.shape or "auto", "grid_blocks": lik.grid_blocks()},
        "roofline": roof,
    }
    if args.calib_copy:
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        result["calib_copy_bytes_each_way"] = src.numel() * 8
        del src, dst
    if not args.no_fit:
        result["newton_cg_time_to_min"] = fit_compare(lik, W)
        print("[bench] fits done", file=sys.stderr, flush=True)
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(W, data, mc)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

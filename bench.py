"""Benchmark of the PWA hot path on one MI355X.

    python bench.py [--gpus 1] [--steps 200] [--warmup 20] [--no-fit] [--no-cpu]
                    [--no-batched] [--precision f64|f32]

Workload: the GPU-scale model -- K = 12 resonances over the channels (12),
(13), (23) with J in {0, 1, 2}, 1M events drawn from the model by
accept-reject and 5M uniform phase-space MC events (synthetic, seeded),
FP64.  One step is one fused
NLL + gradient + Hessian-vector-product evaluation over all 6M events (the
Newton-CG inner-loop call).  Inputs and the parameter-free event stream are
resident in HBM before timing starts.

Prints one JSON line with events/s, the roofline of the dominant kernel
(the per-event pass; timed by HIP events recorded on its stream), the CPU
oracle timed on a bounded sample, per-entry-point timings, Newton-CG
time-to-minimum with FP64 and with mixed precision (FP32 HVPs inside CG), and
the fixed-lineshape batched multi-start path (K = 20, 2M data, 10M MC, 256
coupling vectors) per operand format against the plain FP64 path.
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
WARM_SECONDS = 1.5        # minimum untimed warm-up (clock ramp), see main()


def hvp_flops_per_event(K, data_fraction):
    """Algorithmic FP64 flops of one fused NLL + gradient + HVP per event in
    the moment formulation (add, sub, mul = 1; fused multiply-add = 2;
    reciprocal, logarithm = 1; nothing recomputed).  Per resonance: 46 for
    u, D, w = 1/D, u w, u w^2 and the z, zdot terms; 57 for the nine complex
    moments (the chains p = x u w, q = p w, r = q w for x = gamma, alpha and
    their accumulation): 103.  Per event: |z|^2 and its sum (4), plus for data
    events the log, reciprocal and the weights gamma, alpha (15)."""
    return 103.0 * K + 4.0 + 15.0 * data_fraction


def stream_bytes_per_event(n_planes, real_bytes=8):
    return n_planes * real_bytes


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "hvp_k12_6M_hbm_traffic.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2403_09225_amd", "csrc", "pwa_kernels.hip")


def measured_traffic(kernel):
    """HBM bytes per dispatch of `kernel` from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary (each counter scaled by what it reads for
    a plain copy of known size), or None when there is no summary for this
    kernel or the kernel source has changed since the counters were taken."""
    import hashlib
    try:
        fields = {}
        for line in open(TRAFFIC_PROFILE):
            if ":" in line:
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
        src = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    except OSError:
        return None
    if fields.get("kernel") != kernel or fields.get("source_sha256") != src:
        return None
    return (float(fields["fetch_kib_per_dispatch"]) * 1024.0 * float(fields["fetch_calibration"])
            + float(fields["write_kib_per_dispatch"]) * 1024.0 * float(fields["write_calibration"]))


def measured_valu_instructions(kernel):
    """VALU instructions per dispatch of `kernel` from the same committed
    counter summary (SQ_INSTS_VALU), or None under the same conditions as
    measured_traffic."""
    import hashlib
    try:
        fields = {}
        for line in open(TRAFFIC_PROFILE):
            if ":" in line:
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
        src = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    except OSError:
        return None
    if fields.get("kernel") != kernel or fields.get("source_sha256") != src:
        return None
    v = fields.get("valu_instructions_per_dispatch")
    return float(v) if v else None


def make_workload():
    """MC: uniform phase space (seeded NumPy).  Data: drawn from the model at
    the generating parameters by accept-reject on the GPU (seeded torch
    generator), so a fit from near the truth has a minimum to converge to."""
    import torch
    import synth
    from paper_2403_09225_amd.toys import ToyGenerator
    W = synth.workload("k12_hvp")
    mc = synth.uniform_phase_space(W.n_mc, synth.rng_for("k12_hvp", synth.workloads.STREAM_MC))
    gen = torch.Generator(device="cuda")
    wl = synth.workloads
    gen.manual_seed(wl.BASE_SEED + 100 * wl.SEED_INDEX["k12_hvp"] + wl.STREAM_DATA)
    d12, d13 = ToyGenerator(W.channel, W.spin).draw(W.theta_true, W.n_data, gen)
    data = (d12.cpu().numpy(), d13.cpu().numpy())
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


def cpu_baseline_general(n_data=20_000, n_mc=80_000):
    """The oracle, as it is, on the general physics path's three models
    (K = 12 layout; a Flatte scalar, a spin-1 parent, both), single thread,
    one NLL+grad+HVP over a bounded sample of the same kind of events as the
    GPU section (uniform over phase space and orientation)."""
    import types
    import oracle
    import synth
    try:
        from threadpoolctl import threadpool_limits
        limiter = threadpool_limits(limits=1)
    except Exception:  # pragma: no cover
        limiter = None
    ch, sp = synth.resonance_layout(12)
    kf = next(k for k in range(len(ch)) if ch[k] == 2 and sp[k] == 0)
    rng = np.random.Generator(np.random.PCG64(21))
    ev = []
    for n in (n_data, n_mc):
        s12, s13 = synth.uniform_phase_space(n, rng)
        cb, g = synth.uniform_orientation(n, rng)
        ev.append((s12, s13, cb, g))
    th0 = synth.draw_theta(ch, sp, np.random.Generator(np.random.PCG64(12)))
    v = np.random.Generator(np.random.PCG64(13)).normal(size=4 * len(ch))
    out = {}
    for name, flatte, ps in (("flatte", True, 0), ("spin1", False, 1), ("spin1_flatte", True, 1)):
        model = types.SimpleNamespace(
            channel=list(ch), spin=list(sp), width_mode=0, parent_mass=synth.PARENT_MASS,
            masses=synth.DAUGHTER_MASSES, r=synth.R_BARRIER, n_res=len(ch),
            lineshape=[1 if (flatte and k == kf) else 0 for k in range(len(ch))],
            flatte_masses=synth.FLATTE_MASSES, flatte_ratio=synth.FLATTE_RATIO, parent_spin=ps)
        th = th0.copy()
        if flatte:
            th[4 * kf + 2:4 * kf + 4] = synth.FLATTE_F0
        d, m = (ev[0], ev[1]) if ps == 1 else (ev[0][:2], ev[1][:2])
        t0 = time.perf_counter()
        oracle.hvp(d, m, model, th, v)
        dt = time.perf_counter() - t0
        out[name] = {"value": round((n_data + n_mc) / dt, 1), "unit": "events/s", "cores": 1,
                     "kind": "oracle", "sample": f"one NLL+grad+HVP over {n_data} data + {n_mc} MC "
                                                 f"events; {dt:.2f} s"}
    if limiter is not None:
        limiter.unregister()
    return out


def _oracle_shard(args):
    import oracle
    d, m, W, theta, v = args
    return oracle.partials(d, m, W, theta, v=v)


def cpu_all_cores(W, data, mc, n_data=200_000, n_mc=1_000_000):
    """The oracle on all host cores: a process pool over contiguous event
    shards, combined by eq. (4)-(7) (the oracle's own combine); the same 1:5
    data:MC mix as the workload, one NLL+grad+HVP."""
    import multiprocessing as mp
    import oracle
    cores = len(os.sched_getaffinity(0))
    v = np.random.Generator(np.random.PCG64(5)).normal(size=W.n_par)
    nd, nm = n_data // cores, n_mc // cores
    jobs = [((data[0][i * nd:(i + 1) * nd], data[1][i * nd:(i + 1) * nd]),
             (mc[0][i * nm:(i + 1) * nm], mc[1][i * nm:(i + 1) * nm]), W, W.theta_true, v)
            for i in range(cores)]
    env = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in env:
        os.environ[k] = "1"
    try:
        # fresh interpreters: the workers never inherit this process's GPU state
        ctx = mp.get_context("spawn")
        t0 = time.perf_counter()
        with ctx.Pool(cores) as pool:
            parts = pool.map(_oracle_shard, jobs)
        oracle.combine(parts, v=v)
        dt = time.perf_counter() - t0
    finally:
        for k, val in env.items():
            if val is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = val
    n = cores * (nd + nm)
    return {"value": n / dt, "unit": "events/s", "cores": cores, "kind": "oracle",
            "sample": f"one NLL+grad+HVP of the oracle over {cores * nd} data + {cores * nm} MC events "
                      f"in {cores} processes (eq. (4)-(7) combine); {dt:.2f} s"}


def fit_compare(lik, W, cap_s=60.0, n_starts=5):
    """Newton-CG time to minimum from seeded starts near the generating
    parameters, with FP64 HVPs and with FP32 HVPs inside CG (line search and
    convergence test in FP64 in both), for scipy's forcing term (the paper's
    fits) and for the relative one, each with plain and with reconjugated CG
    (every direction H-conjugated to the earlier ones of its solve), and
    with CG preconditioned by |H|^-1.
    Per variant: the first start in detail, and the totals over n_starts
    starts."""
    import synth
    rng = synth.rng_for("k12_hvp", synth.workloads.STREAM_TEST)
    starts = [W.theta_true + rng.normal(scale=np.tile([0.02, 0.02, 0.002, 0.002], W.n_res))
              for _ in range(n_starts)]
    out = {}
    for forcing, rc in (("relative", False), ("scipy", False), ("relative", True), ("scipy", True)):
        rec = {}
        for prec in ("f64", "f32"):
            runs = []
            for i, start in enumerate(starts):
                th, rep = lik.fit(start, xtol=1e-8, maxiter=200, time_cap_s=cap_s,
                                  hvp_precision=prec, forcing=forcing, reconjugate=rc)
                runs.append(rep)
            r0 = runs[0]
            rec[prec] = {"seconds": round(r0["seconds"], 4), "nll": r0["nll"],
                         "iterations": r0["iterations"], "hvps": r0["n_hvp"],
                         "grads": r0["n_grad"], "nlls": r0["n_nll"], "converged": r0["converged"],
                         f"seconds_total_{n_starts}_starts": round(sum(r["seconds"] for r in runs), 4),
                         f"iterations_total_{n_starts}_starts": int(sum(r["iterations"] for r in runs)),
                         f"converged_{n_starts}_starts": int(sum(r["converged"] for r in runs)),
                         "nll_spread": float(max(r["nll"] for r in runs) - min(r["nll"] for r in runs))}
        rec["speedup_mixed_vs_fp64"] = round(rec["f64"]["seconds"] / max(rec["f32"]["seconds"], 1e-9), 3)
        key = f"seconds_total_{n_starts}_starts"
        rec[f"speedup_mixed_vs_fp64_{n_starts}_starts"] = round(rec["f64"][key] / max(rec["f32"][key], 1e-9), 3)
        rec["nll_diff_mixed_minus_fp64"] = rec["f32"]["nll"] - rec["f64"]["nll"]
        out[f"forcing_{forcing}" + ("_reconjugated" if rc else "")] = rec
    # CG preconditioned with |H|^-1 (relative forcing), FP64 and FP32 HVPs
    for prec in ("f64", "f32"):
        runs = [lik.fit(start, xtol=1e-8, maxiter=200, time_cap_s=cap_s, forcing="relative",
                        precondition=True, hvp_precision=prec)[1] for start in starts]
        r0 = runs[0]
        out[f"forcing_relative_preconditioned_{prec}"] = {
            "seconds": round(r0["seconds"], 4), "nll": r0["nll"], "iterations": r0["iterations"],
            "hvps": r0["n_hvp"], "grads": r0["n_grad"], "converged": r0["converged"],
            f"seconds_total_{n_starts}_starts": round(sum(r["seconds"] for r in runs), 4),
            f"iterations_total_{n_starts}_starts": int(sum(r["iterations"] for r in runs)),
            f"converged_{n_starts}_starts": int(sum(r["converged"] for r in runs)),
            "nll_spread": float(max(r["nll"] for r in runs) - min(r["nll"] for r in runs)),
            "nll_diff_vs_plain_f64": r0["nll"] - out["forcing_relative"]["f64"]["nll"]}
    return out


def k30_bench(steps=20):
    """The differentiation workload (K = 30, 4M data drawn from the model on
    the GPU + 20M MC): fused NLL+grad+HVP events/s on the FP64 and FP32
    streams, and the direction-only HVP of the CG inner step."""
    import torch
    import synth
    from paper_2403_09225_amd import Likelihood
    from paper_2403_09225_amd.toys import ToyGenerator
    W = synth.workload("k30_diff")
    mc = synth.uniform_phase_space(W.n_mc, synth.rng_for("k30_diff", synth.workloads.STREAM_MC))
    wl = synth.workloads
    gen = torch.Generator(device="cuda")
    gen.manual_seed(wl.BASE_SEED + 100 * wl.SEED_INDEX["k30_diff"] + wl.STREAM_DATA)
    data = ToyGenerator(W.channel, W.spin).draw(W.theta_true, W.n_data, gen)
    lik = Likelihood(W.channel, W.spin, streams=("f64", "f32")).bind(data[0], data[1], mc[0], mc[1])
    del data, mc
    th = torch.tensor(W.theta_true, dtype=torch.float64, device="cuda")
    v = torch.tensor(np.random.Generator(np.random.PCG64(3)).normal(size=W.n_par),
                     dtype=torch.float64, device="cuda")
    n = W.n_data + W.n_mc
    out = {"workload": f"K={W.n_res} (P={W.n_par}), {W.n_data} data + {W.n_mc} MC events"}
    for prec in ("f64", "f32"):
        lik.set_precision(prec)
        for _ in range(3):
            lik.hvp(th, v)
        torch.cuda.synchronize()
        lik.set_kernel_timing(True)
        lik.kernel_time()
        t0 = time.perf_counter()
        for _ in range(steps):
            lik.hvp(th, v)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        k_ms, k_n = lik.kernel_time()
        lik.set_kernel_timing(False)
        out[prec] = {"ms_per_step": round(dt * 1e3, 4), "events_per_s": round(n / dt, 1),
                     "kernel_us": round(k_ms / max(k_n, 1) * 1e3, 2),
                     "hbm_frac_kernel": round(n * 18 * (8 if prec == "f64" else 4)
                                              / (k_ms / max(k_n, 1) / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
        lik.hvp(th, v)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            lik.hvp_reuse(v)
        torch.cuda.synchronize()
        out[prec]["reuse_ms_per_step"] = round((time.perf_counter() - t0) / steps * 1e3, 4)
    return out


def general_bench(reps=20, models=("flatte", "spin1", "spin1_flatte")):
    """The general physics path on the GPU-scale layout (K = 12, 1M data +
    5M MC events, uniform over phase space and parent orientation, FP64
    stream): a Flatte f0(980)-like scalar in the (23) channel (Sec. 3's
    model), a spin-1 parent with two helicity amplitudes per event (eq. (1),
    mu = +1, -1), and both.  Per-event kernel time of the fused
    NLL+grad+HVP, NLL+grad and NLL passes, events/s, and the HBM fraction of
    the stream bytes (planes x 8 B per event, read once per pass)."""
    import torch
    import synth
    from paper_2403_09225_amd import Likelihood
    ch, sp = synth.resonance_layout(12)
    nd, nm = 1_000_000, 5_000_000
    rng = np.random.Generator(np.random.PCG64(11))
    ev = []
    for n in (nd, nm):
        s12, s13 = synth.uniform_phase_space(n, rng)
        cb, g = synth.uniform_orientation(n, rng)
        ev.append((s12, s13, cb, g))
    th0 = synth.draw_theta(ch, sp, np.random.Generator(np.random.PCG64(12)))
    kf = next(k for k in range(len(ch)) if ch[k] == 2 and sp[k] == 0)
    ls = [1 if k == kf else 0 for k in range(len(ch))]
    v = torch.tensor(np.random.Generator(np.random.PCG64(13)).normal(size=4 * len(ch)),
                     dtype=torch.float64, device="cuda")
    out = {"workload": f"K=12, {nd} data + {nm} MC events (uniform), FP64 stream; Flatte "
                       f"resonance {kf} (channel (23), J = 0)"}
    for name, lshape, ps in (("flatte", ls, 0), ("spin1", None, 1), ("spin1_flatte", ls, 1)):
        if name not in models:
            continue
        lik = Likelihood(ch, sp, lineshape=lshape, flatte_masses=synth.FLATTE_MASSES,
                         flatte_ratio=synth.FLATTE_RATIO, parent_spin=ps)
        if ps == 1:
            lik.bind_oriented(ev[0], ev[1])
        else:
            lik.bind(ev[0][0], ev[0][1], ev[1][0], ev[1][1])
        th = th0.copy()
        if lshape:
            th[4 * kf + 2:4 * kf + 4] = synth.FLATTE_F0
        th = torch.tensor(th, dtype=torch.float64, device="cuda")
        fields = lik.stream_fields()
        rec = {"stream_fields": fields}
        for mode, fn in (("hvp", lambda: lik.hvp(th, v)), ("grad", lambda: lik.grad(th)),
                         ("nll", lambda: lik.nll(th))):
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            lik.set_kernel_timing(True)
            lik.kernel_time()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            k_ms, k_n = lik.kernel_time()
            lik.set_kernel_timing(False)
            us = k_ms / max(k_n, 1) * 1e3
            rec[mode] = {"kernel_us": round(us, 2), "events_per_s": round((nd + nm) / us * 1e6, 1),
                         "hbm_frac": round((nd + nm) * fields * 8 / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}
        out[name] = rec
        del lik
        torch.cuda.empty_cache()
    return out


def entry_point_times(lik, th, v, reps=20):
    """Per-call time of pwa_nll, pwa_grad, pwa_hvp and pwa_hvp_reuse (an HVP
    at the theta of the last pwa_hvp, as inside CG) on the FP64 and FP32
    event streams: wall time per call over `reps` back-to-back calls and the
    average duration of the per-event kernel (HIP events on its stream)."""
    import torch
    out = {}
    for prec in ("f64", "f32"):
        lik.set_precision(prec)
        for name, fn in (("nll", lambda: lik.nll(th)), ("grad", lambda: lik.grad(th)),
                         ("hvp", lambda: lik.hvp(th, v)), ("hvp_reuse", lambda: lik.hvp_reuse(v))):
            if name == "hvp_reuse":
                lik.hvp(th, v)   # the theta-only totals the reuse pass starts from
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            lik.set_kernel_timing(True)
            lik.kernel_time()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            k_ms, k_n = lik.kernel_time()
            lik.set_kernel_timing(False)
            out[f"{name}_{prec}"] = {"call_us": round(dt * 1e6, 2),
                                     "kernel_us": round(k_ms / max(k_n, 1) * 1e3, 2)}
    return out


def at_minimum_times(lik, th, reps=3):
    """Wall time of the quantities read off at a minimum on the same events:
    the full Hessian (pwa_hessian, P Hessian-vector passes), the fit
    fractions with their gradients (pwa_fit_fractions, K + 1 MC-only
    gradient passes) and the fraction matrix with interference terms
    (pwa_fraction_matrix, one MC Gram pass), FP64 event stream."""
    import torch
    lik.set_precision("f64")
    out = {}
    for name, fn in (("hessian", lambda: lik.hessian(th)),
                     ("fit_fractions", lambda: lik.fit_fractions(th)),
                     ("fraction_matrix", lambda: lik.fraction_matrix(th))):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        out[f"{name}_ms"] = round((time.perf_counter() - t0) / reps * 1e3, 3)
    return out


def batched_bench(reps=5):
    """Fixed-lineshape batched multi-start (K = 20, 2M data, 10M MC, 256
    coupling vectors): time per batch and NLL error per operand format (vs
    the FP64-operand batched result, itself checked against the oracle), and
    the plain FP64 GPU path (pwa_nll once per start) for the speed-up."""
    import torch
    import synth
    from paper_2403_09225_amd import Likelihood
    W = synth.workload("k20_batched")
    mc = synth.uniform_phase_space(W.n_mc, synth.rng_for("k20_batched", synth.workloads.STREAM_MC))
    data = synth.resonant_like(W.n_data, W.channel, W.theta_true,
                               synth.rng_for("k20_batched", synth.workloads.STREAM_DATA))
    B = W.extra["n_starts"]
    r = synth.rng_for("k20_batched", synth.workloads.STREAM_TEST)
    C = r.uniform(0, 1, (W.n_res, B)) * np.exp(2j * np.pi * r.uniform(size=(W.n_res, B)))
    lik = Likelihood(W.channel, W.spin).bind(data[0], data[1], mc[0], mc[1])
    del data, mc
    out = {"workload": f"K={W.n_res} frozen masses/widths, {W.n_data} data + {W.n_mc} MC, "
                       f"B={B} coupling vectors", "formats": {}}
    ref = None
    for fmt in ("f64", "f32", "f16s", "f16", "bf16"):
        lik.freeze(W.theta_true, fmt, B)
        nll = lik.nll_batched(C)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            nll = lik.nll_batched(C)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / reps * 1e3
        v = nll.cpu().numpy()
        if ref is None:
            ref = v
        out["formats"][fmt] = {"ms_per_batch": round(ms, 4), "us_per_start": round(ms * 1e3 / B, 3),
                               "max_abs_nll_err_vs_f64": float(np.max(np.abs(v - ref)))}
    # plain FP64 path: one full NLL pass per start at the frozen M, Gamma
    th = torch.tensor(W.theta_true, dtype=torch.float64, device="cuda")
    thetas = []
    for b in range(B):
        t = th.clone()
        t[0::4] = torch.tensor(C[:, b].real, device="cuda")
        t[1::4] = torch.tensor(C[:, b].imag, device="cuda")
        thetas.append(t)
    lik.nll(thetas[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain = [lik.nll(t) for t in thetas]
    torch.cuda.synchronize()
    plain_ms = (time.perf_counter() - t0) * 1e3
    pv = np.array([float(x) for x in plain])
    out["plain_fp64_ms_per_batch"] = round(plain_ms, 3)
    out["plain_vs_batched_f64_max_abs_diff"] = float(np.max(np.abs(pv - ref)))
    for fmt, rec in out["formats"].items():
        rec["speedup_vs_plain_fp64"] = round(plain_ms / rec["ms_per_batch"], 2)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-fit", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--precision", default="f64", choices=["f64", "f32"])
    ap.add_argument("--shape", default="", help="layout,groups,res_per_group override (layout 0: lanes per event, 1: waves per block)")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-k30", action="store_true", help="skip the K = 30, 24M-event section")
    ap.add_argument("--no-general", action="store_true",
                    help="skip the general physics path section (Flatte, spin-1 parent)")
    ap.add_argument("--general-model", default="all",
                    choices=["all", "flatte", "spin1", "spin1_flatte"],
                    help="run the general physics path section for one model only")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the sharded evaluation (pwa_partials on each rank, "
              "one exchange, pwa_combine) is not launched by it. Use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2403_09225_amd import Likelihood

    torch.cuda.set_device(0)
    W, data, mc = make_workload()
    print(f"[bench] workload ready: {W.n_data} data + {W.n_mc} MC events, K={W.n_res}",
          file=sys.stderr, flush=True)
    lik = Likelihood(W.channel, W.spin, streams=("f64", "f32"))
    dev = [torch.as_tensor(x, device="cuda") for x in (data[0], data[1], mc[0], mc[1])]
    torch.cuda.synchronize()
    t_bind = time.perf_counter()
    lik.bind(*dev)
    torch.cuda.synchronize()
    t_bind = time.perf_counter() - t_bind
    del dev
    if args.shape:
        lik.set_launch_shape(*[int(x) for x in args.shape.split(",")])
    lik.set_precision(args.precision)
    th = torch.tensor(W.theta_true, dtype=torch.float64, device="cuda")
    v = torch.tensor(np.random.Generator(np.random.PCG64(9)).normal(size=W.n_par),
                     dtype=torch.float64, device="cuda")
    for _ in range(args.warmup):
        lik.hvp(th, v)
    torch.cuda.synchronize()
    # Clock ramp: the first few hundred milliseconds of sustained load run at
    # lower clocks, so untimed steps continue until the warm-up has lasted
    # WARM_SECONDS of wall time whatever --warmup says.
    t_w = time.perf_counter()
    while time.perf_counter() - t_w < WARM_SECONDS:
        for _ in range(50):
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
    # The pass reads the event stream once (bytes) and does `flops` of FP64
    # work; at these intensities (~8.5 flop/B for FP64, below the 9.8 flop/B
    # ridge) the binding roofline is HBM; the ALU fraction is reported beside.
    gbs = bytes_launch / k_avg_s / 1e9
    tfl = flops / k_avg_s / 1e12
    hbm_bound = flops / bytes_launch < FP64_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    traffic = valu = None
    if args.precision == "f64" and not args.shape:
        traffic = measured_traffic("wg_kernel<double, 2, 4, 3>")
        valu = measured_valu_instructions("wg_kernel<double, 2, 4, 3>")
    # VALU-issue floor: one wave64 instruction per SIMD every 4 cycles, 1024
    # SIMDs at the 2.4 GHz peak clock
    valu_floor_s = valu * 4 / (1024 * 2.4e9) if valu else None
    roof = {"bound": "hbm" if hbm_bound else "alu",
            "achieved": round(gbs if hbm_bound else tfl, 3),
            "peak": HBM_PEAK_GBS if hbm_bound else FP64_PEAK_TFLOPS,
            "unit": "GB/s" if hbm_bound else "TFLOP/s",
            "frac": round(gbs / HBM_PEAK_GBS if hbm_bound else tfl / FP64_PEAK_TFLOPS, 4),
            "traffic": traffic,
            "traffic_source": "profiles/hvp_k12_6M_hbm_traffic.md" if traffic else None,
            "kernel": f"wg_kernel HVP ({args.precision}), per-event pass",
            "kernel_avg_us": round(k_avg_s * 1e6, 2),
            "algorithmic_bytes_per_launch": bytes_launch, "algorithmic_flops_per_launch": flops,
            "alu_achieved_tflops": round(tfl, 3), "alu_frac": round(tfl / FP64_PEAK_TFLOPS, 4),
            "valu_instructions_per_launch": valu,
            "valu_issue_floor_us": round(valu_floor_s * 1e6, 1) if valu_floor_s else None,
            "valu_issue_frac": round(valu_floor_s / k_avg_s, 4) if valu_floor_s else None}
    result = {
        "metric": "events/s for NLL+grad+HVP (one fused evaluation)",
        "value": round(value, 1), "unit": "events/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "f64" else "f32", "data": "synthetic",
        "config": {"workload": "K=12 resonances over (12),(13),(23), J in {0,1,2}; "
                               "1M events drawn from the model + 5M uniform MC events; "
                               "one fused NLL+grad+HVP pass (Newton-CG inner step)",
                   "n_res": W.n_res, "n_data": W.n_data, "n_mc": W.n_mc,
                   "launch_shape": args.shape or "auto", "grid_blocks": lik.grid_blocks(),
                   "workspace_bytes": lik.workspace_bytes(W.n_data, W.n_mc),
                   "bind_precompute_ms": round(t_bind * 1e3, 3),
                   "workspace_bytes_per_event": round(lik.workspace_bytes(W.n_data, W.n_mc)
                                                      / (W.n_data + W.n_mc), 1)},
        "roofline": roof,
    }
    result["entry_points"] = entry_point_times(lik, th, v)
    result["at_minimum"] = at_minimum_times(lik, th)
    lik.set_precision(args.precision)
    # A plain 1 GiB device-to-device copy: the practical HBM ceiling (read +
    # write bytes / time) and the reference for the HBM byte counters.
    src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5 if args.calib_copy else 10):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * src.numel() * 8 * (5 if args.calib_copy else 10) / (e0.elapsed_time(e1) / 1e3) / 1e9
    roof["hbm_copy_measured_GBs"] = round(copy_gbs, 1)
    roof["frac_of_measured_copy"] = round(gbs / copy_gbs, 4)
    result["calib_copy_bytes_each_way"] = src.numel() * 8
    del src, dst
    if not args.no_fit:
        result["newton_cg_time_to_min"] = fit_compare(lik, W)
        print("[bench] fits done", file=sys.stderr, flush=True)
    if not args.no_batched or not args.no_k30 or not args.no_general:
        del lik
        torch.cuda.empty_cache()
    if not args.no_batched:
        result["batched_multistart"] = batched_bench()
        torch.cuda.empty_cache()
        print("[bench] batched path done", file=sys.stderr, flush=True)
    if not args.no_k30:
        result["k30_differentiation"] = k30_bench()
        torch.cuda.empty_cache()
        print("[bench] K = 30 workload done", file=sys.stderr, flush=True)
    if not args.no_general:
        result["general_physics_path"] = general_bench(
            models=("flatte", "spin1", "spin1_flatte") if args.general_model == "all"
            else (args.general_model,))
        torch.cuda.empty_cache()
        print("[bench] general physics path done", file=sys.stderr, flush=True)
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(W, data, mc)
        result["cpu_all_cores"] = cpu_all_cores(W, data, mc)
        if not args.no_general:
            result["cpu_baseline_general_path"] = cpu_baseline_general()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

#!/usr/bin/env python
"""Throughput of FSM-scheduled multi-chain MCMC on one MI355X.

Headline workload (value): elliptical slice sampling of a D = 1024 latent
Gaussian process (inputs uniform on [0, 1], squared-exponential prior,
lengthscale 0.05, jitter 1e-5) with a Bernoulli-logistic likelihood whose
labels come from a seeded prior draw; 8192 chains x 2000 draws, FP32,
ellipse directions L z on FP32 MFMA.  One step = one complete sampling job
(init_chains + every chain to 2000 draws) through the C ABI; inputs (L,
labels) are resident in HBM before the timed region.

Reported beside it, on the same box and run:
  * the synchronized runtime on the same job (vmap semantics and the
    compacted variant), the FSM/synchronized speed-ups and bit-exactness;
  * NUTS on Bayesian logistic regression (N = 10000, D = 100, step 0.05,
    depth 10, Laplace starts), 8192 chains x 1000 draws, FSM vs synchronized;
  * R(m) of each job estimated from its own loop counts;
  * the live roofline figure of the dominant kernel (HIP events);
  * the FP64 CPU oracle timed on a bounded sample of the ESS workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "draws/sec FSM vs synchronized (ESS, NUTS, 8192 chains); p50/p99 job latency"
PEAK_MFMA_F32 = 157.3  # TFLOP/s, MI355X dense FP32 MFMA


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def checksum(out, m_chunk=256):
    """Exact integer checksum of a float32 tensor (bit patterns summed in int64)."""
    import torch
    s = 0
    for i in range(0, out.shape[0], m_chunk):
        s += int(out[i:i + m_chunk].view(torch.int32).to(torch.int64).sum().item())
    return s


def timed_jobs(make, run, steps, warmup):
    import torch
    for i in range(warmup):
        job = make()
        run(job)
        job.free()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = None
    for i in range(steps):
        if last is not None:
            last.free()
        last = make()
        run(last)
        log("  job %d: %.3f s" % (i, time.perf_counter() - t0))
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    return dt, last


def bench_ess(F, ctx, args):
    import torch

    from oracle import diagnostics as Dg
    from paper_2503_17405_amd import inputs
    m, n, D = args.chains, args.draws, 1024
    w = inputs.gp_logistic(dim=D, lengthscale=0.05, jitter=1e-5, seed=2001)
    seed = 2002
    L = torch.tensor(w["L"], dtype=torch.float32, device="cuda")
    y = torch.tensor(w["y"], dtype=torch.float32, device="cuda")
    out = torch.empty((m, n, D), dtype=torch.float32, device="cuda")
    target, sampler = F.gp_target(L, y), F.ess_sampler(F.F32)
    make = lambda: F.Job(ctx, target, sampler, m, n, seed, out=out, window=args.window, timing=True)

    log("ESS FSM")
    t_fsm, job = timed_jobs(make, lambda j: j.step_fsm(0), args.steps, args.warmup)
    st = job.stats()
    counts = job.counts()
    job.free()
    ref = checksum(out)
    res = dict(seconds=t_fsm, draws_per_s=m * n / t_fsm, steps=st["steps"],
               kernel_ms=st["kernel_ms"], kernel_launches=st["kernel_launches"],
               mean_loop=float(counts.mean()), mean_max_loop=float(counts.max(axis=0).mean()),
               R_hat_m=Dg.r_hat_m(counts, m))
    g_ms, g_n = st["kernel_ms"][0], st["kernel_launches"][0]
    flops = float(m) * n * D * (D + 1)
    res["gemm"] = dict(kernel="nu_gemm_mfma_kernel<4>", ms=g_ms, launches=g_n, avg_us=1e3 * g_ms / max(g_n, 1),
                       tflops=flops / (g_ms * 1e-3) / 1e12, flop_per_column=D * (D + 1))
    sync = {}
    if not args.no_sync:
        for name, mode in (("vmap", F.SYNC_VMAP), ("compact", F.SYNC_COMPACT)):
            log("ESS sync %s" % name)
            dt, job = timed_jobs(make, lambda j, mode=mode: j.step_synchronized(n, mode), args.sync_steps, 0)
            s2 = job.stats()
            job.free()
            sync[name] = dict(seconds=dt, draws_per_s=m * n / dt, steps=s2["steps"],
                              padded_steps=s2["padded_steps"], kernel_ms=s2["kernel_ms"],
                              bit_exact_vs_fsm=bool(checksum(out) == ref), speedup_fsm=dt / t_fsm)
    res["sync"] = sync
    del out
    torch.cuda.empty_cache()
    return res, w, seed


def bench_nuts(F, ctx, args):
    import numpy as np
    import torch

    from oracle import diagnostics as Dg
    from paper_2503_17405_amd import inputs
    m, n, N, D = args.nuts_chains, args.nuts_draws, 10000, 100
    d = inputs.logreg(n_data=N, dim=D, seed=3001)
    lap = inputs.logreg_laplace(d["X"], d["y"], m, seed=3002)
    X = torch.tensor(d["X"], dtype=torch.float32, device="cuda")
    y = torch.tensor(d["y"], dtype=torch.float32, device="cuda")
    x0 = torch.tensor(lap["x0"], dtype=torch.float32, device="cuda")
    out = torch.empty((m, n, D), dtype=torch.float32, device="cuda")
    target, sampler = F.logreg_target(X, y), F.nuts_sampler(0.05, 10)
    seed = 3003
    make = lambda: F.Job(ctx, target, sampler, m, n, seed, x0=x0, out=out, timing=True)
    log("NUTS FSM")
    t_fsm, job = timed_jobs(make, lambda j: j.step_fsm(0), args.nuts_steps, args.nuts_warmup)
    st = job.stats()
    counts = job.counts()
    job.free()
    ref = checksum(out)
    res = dict(seconds=t_fsm, draws_per_s=m * n / t_fsm, steps=st["steps"],
               kernel_ms=st["kernel_ms"], kernel_launches=st["kernel_launches"],
               mean_loop=float(counts.mean()), mean_max_loop=float(counts.max(axis=0).mean()),
               R_hat_m=Dg.r_hat_m(counts, m), divergent_free=bool(np.isfinite(counts).all()))
    g_ms = st["kernel_ms"][0]
    flops = 4.0 * N * D * st["steps"]  # X Theta and X^T r per requested gradient
    res["gradient"] = dict(kernel="logreg_grad_kernel<4> + logreg_reduce_kernel", ms=g_ms,
                           launches=st["kernel_launches"][0],
                           tflops=flops / (g_ms * 1e-3) / 1e12, flop_per_gradient=4 * N * D)
    sync = {}
    if not args.no_sync:
        for name, mode in (("vmap", F.SYNC_VMAP), ("compact", F.SYNC_COMPACT)):
            log("NUTS sync %s" % name)
            dt, job = timed_jobs(make, lambda j, mode=mode: j.step_synchronized(n, mode), 1, 0)
            s2 = job.stats()
            job.free()
            sync[name] = dict(seconds=dt, draws_per_s=m * n / dt, steps=s2["steps"],
                              padded_steps=s2["padded_steps"], kernel_ms=s2["kernel_ms"],
                              bit_exact_vs_fsm=bool(checksum(out) == ref), speedup_fsm=dt / t_fsm)
    res["sync"] = sync
    del out
    torch.cuda.empty_cache()
    return res


def cpu_baseline(w, seed, chains, draws, threads):
    from oracle import oracle as O
    tg = O.gp_target(w["y"])
    sp = O.ess_sampler(w["L"])
    t0 = time.perf_counter()
    O.run_chains(tg, sp, seed, range(chains), draws, threads=threads)
    dt = time.perf_counter() - t0
    return dict(value=chains * draws / dt, unit="draws/s", cores=threads, kind="oracle",
                sample="ESS workload: %d chains x first %d draws, FP64, %d threads, %.1f s"
                       % (chains, draws, threads, dt))


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sync-steps", type=int, default=1)
    ap.add_argument("--chains", type=int, default=8192)
    ap.add_argument("--draws", type=int, default=2000)
    ap.add_argument("--window", type=int, default=0)
    ap.add_argument("--nuts-chains", type=int, default=8192)
    ap.add_argument("--nuts-draws", type=int, default=1000)
    ap.add_argument("--nuts-steps", type=int, default=1)
    ap.add_argument("--nuts-warmup", type=int, default=1)
    ap.add_argument("--no-nuts", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sync", action="store_true")
    ap.add_argument("--cpu-draws", type=int, default=2000)
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU: the chains are independent and this build runs on a "
              "single MI355X (--gpus %d is not supported)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2503_17405_amd import fsmmc as F

    ctx = F.Context(0)
    ess, w, seed = bench_ess(F, ctx, args)
    log("ESS: FSM %.3g draws/s" % ess["draws_per_s"])
    nuts = None
    if not args.no_nuts:
        nuts = bench_nuts(F, ctx, args)
        log("NUTS: FSM %.3g draws/s" % nuts["draws_per_s"])
    cpu = None
    if not args.no_cpu_baseline:
        threads = min(os.cpu_count() or 1, 16)
        cpu = cpu_baseline(w, seed, 4 * threads, args.cpu_draws, threads)
        log("cpu oracle: %.3g draws/s (%s)" % (cpu["value"], cpu["sample"]))
    ctx.close()

    g = ess["gemm"]
    line = {
        "metric": METRIC,
        "value": ess["draws_per_s"],
        "unit": "draws/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ess["seconds"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "ESS GP-logistic D=1024 (SE lengthscale 0.05, jitter 1e-5), "
                               "%d chains x %d draws, FP32; one step = one whole sampling job"
                               % (args.chains, args.draws),
                   "chains": args.chains, "draws": args.draws, "dim": 1024},
        "roofline": {"bound": "mfma", "kernel": g["kernel"], "achieved": g["tflops"],
                     "peak": PEAK_MFMA_F32, "unit": "TFLOP/s", "frac": g["tflops"] / PEAK_MFMA_F32,
                     "traffic": None, "avg_launch_us": g["avg_us"], "launches": g["launches"]},
        "ess": ess,
        "speedup_vs_sync_vmap": ess["sync"].get("vmap", {}).get("speedup_fsm"),
        "speedup_vs_sync_compact": ess["sync"].get("compact", {}).get("speedup_fsm"),
        "nuts": nuts,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()

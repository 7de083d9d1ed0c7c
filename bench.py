#!/usr/bin/env python
"""Throughput of FSM-scheduled multi-chain MCMC on one MI355X.

Workload (the headline configuration): elliptical slice sampling of a
D = 1024 latent Gaussian process (inputs uniform on [0, 1], squared-
exponential prior, lengthscale 0.05, jitter 1e-5) with a Bernoulli-logistic
likelihood whose labels come from a seeded prior draw; 8192 chains x 2000
draws, FP32, ellipse directions L z on FP32 MFMA.

One step = one complete sampling job (init_chains + every chain to 2000
draws) through the C ABI; inputs (L, labels) are resident in HBM before the
timed region.  The synchronized runtime (vmap semantics and the compacted
variant) is timed on the same job and reported beside it, with the FSM/sync
speed-up, the efficiency bound R(m) estimated from the job's own loop counts,
the live roofline figure of the dominant kernel, and the FP64 CPU oracle
timed on a bounded sample of the same workload.
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
PEAK_HBM = 8000.0      # GB/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def checksum(out, m_chunk=256):
    """Exact integer checksum of a float32 tensor (bit patterns summed in int64)."""
    import torch
    s = 0
    for i in range(0, out.shape[0], m_chunk):
        s += int(out[i:i + m_chunk].view(torch.int32).to(torch.int64).sum().item())
    return s


def cpu_baseline(w, seed, chains, draws, threads):
    from oracle import oracle as O
    tg = O.gp_target(w["y"])
    sp = O.ess_sampler(w["L"])
    t0 = time.perf_counter()
    O.run_chains(tg, sp, seed, range(chains), draws, threads=threads)
    dt = time.perf_counter() - t0
    return dict(value=chains * draws / dt, unit="draws/s", cores=threads, kind="oracle",
                sample="%d chains x first %d draws of the same workload, FP64, %d threads, %.1f s"
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
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sync", action="store_true")
    ap.add_argument("--cpu-draws", type=int, default=2000)
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU: the chains are independent and this build runs on a "
              "single MI355X (--gpus %d is not supported)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from oracle import diagnostics as Dg
    from paper_2503_17405_amd import fsmmc as F
    from paper_2503_17405_amd import inputs

    m, n, D = args.chains, args.draws, 1024
    w = inputs.gp_logistic(dim=D, lengthscale=0.05, jitter=1e-5, seed=2001)
    seed = 2002
    L = torch.tensor(w["L"], dtype=torch.float32, device="cuda")
    y = torch.tensor(w["y"], dtype=torch.float32, device="cuda")
    out = torch.empty((m, n, D), dtype=torch.float32, device="cuda")
    ctx = F.Context(0)
    target = F.gp_target(L, y)
    sampler = F.ess_sampler(F.F32)
    torch.cuda.synchronize()

    def job_fsm():
        job = F.Job(ctx, target, sampler, m, n, seed, out=out, window=args.window, timing=True)
        job.step_fsm(0)
        st = job.stats()
        return job, st

    def job_sync(mode):
        job = F.Job(ctx, target, sampler, m, n, seed, out=out, window=args.window, timing=True)
        job.step_synchronized(n, mode)
        st = job.stats()
        return job, st

    for i in range(args.warmup):
        job, _ = job_fsm()
        job.free()
        log("warmup %d done" % i)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for i in range(args.steps):
        job, st = job_fsm()
        stats.append(st)
        if i < args.steps - 1:
            job.free()
        log("step %d: %.3f s" % (i, time.perf_counter() - t0))
    torch.cuda.synchronize()
    t_fsm = (time.perf_counter() - t0) / args.steps
    counts = job.counts()
    job.free()
    sum_fsm = checksum(out)
    value = m * n / t_fsm
    log("FSM: %.3f s/job, %.3g draws/s" % (t_fsm, value))

    # efficiency bound from the job's own loop counts (Sec. 4.2)
    emax_emp = float(counts.max(axis=0).mean())
    mean_n = float(counts.mean())
    r_hat = Dg.r_hat_m(counts, m)

    st = stats[-1]
    g_ms, g_n = st["kernel_ms"][0], st["kernel_launches"][0]
    f_ms, f_n = st["kernel_ms"][1], st["kernel_launches"][1]
    flops = float(m) * n * D * (D + 1)  # triangular L z per (chain, draw)
    gemm_tflops = flops / (g_ms * 1e-3) / 1e12
    res = {}
    if not args.no_sync:
        for name, mode in (("vmap", F.SYNC_VMAP), ("compact", F.SYNC_COMPACT)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(args.sync_steps):
                job, sst = job_sync(mode)
                job.free()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / args.sync_steps
            res[name] = dict(seconds=dt, draws_per_s=m * n / dt, steps=sst["steps"],
                             padded_steps=sst["padded_steps"], kernel_ms=sst["kernel_ms"],
                             bit_exact_vs_fsm=bool(checksum(out) == sum_fsm))
            log("sync %s: %.3f s/job, %.3g draws/s, bit-exact=%s" % (name, dt, m * n / dt,
                                                                    res[name]["bit_exact_vs_fsm"]))

    cpu = None
    if not args.no_cpu_baseline:
        threads = min(os.cpu_count() or 1, 16)
        cpu = cpu_baseline(w, seed, 4 * threads, args.cpu_draws, threads)
        log("cpu oracle: %.3g draws/s (%s)" % (cpu["value"], cpu["sample"]))

    dominant = "ellipse_gemm" if g_ms >= f_ms else "ess_fsm_loop"
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "draws/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_fsm * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "ESS GP-logistic D=1024 (SE lengthscale 0.05, jitter 1e-5), "
                               "8192 chains x 2000 draws, FP32; one step = one whole job",
                   "chains": m, "draws": n, "dim": D},
        "roofline": {"bound": "mfma", "kernel": "nu_gemm_mfma_kernel", "achieved": gemm_tflops,
                     "peak": PEAK_MFMA_F32, "unit": "TFLOP/s", "frac": gemm_tflops / PEAK_MFMA_F32,
                     "traffic": None,
                     "per_launch": {"columns": m * st.get("window", 0) if False else None,
                                    "avg_ms": g_ms / max(g_n, 1), "launches": g_n},
                     "dominant_kernel": dominant},
        "kernel_time_ms_per_job": {"ellipse_gemm": g_ms, "fsm_loop": f_ms},
        "fsm": {"steps": st["steps"], "mean_evals_per_draw": mean_n,
                "mean_max_evals_per_draw": emax_emp, "R_hat_m": r_hat},
        "sync": {k: {kk: vv for kk, vv in v.items()} for k, v in res.items()},
        "speedup_vs_sync_vmap": (res["vmap"]["seconds"] / t_fsm) if "vmap" in res else None,
        "speedup_vs_sync_compact": (res["compact"]["seconds"] / t_fsm) if "compact" in res else None,
        "cpu_baseline": cpu,
    }
    ctx.close()
    print(json.dumps(line))


if __name__ == "__main__":
    main()

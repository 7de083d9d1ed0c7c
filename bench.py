#!/usr/bin/env python
"""Throughput of FSM-scheduled multi-chain MCMC on one MI355X.

Headline workload (value): elliptical slice sampling of a D = 1024 latent
Gaussian process (inputs uniform on [0, 1], squared-exponential prior,
lengthscale 0.05, jitter 1e-5) with a Bernoulli-logistic likelihood whose
labels come from a seeded prior draw; 8192 chains x 2000 draws, FP32,
ellipse directions L z to FP32 accuracy on the bf16 matrix cores (exact
three-piece bf16 splits of z and L, six piece products per FP32 product,
FP32 accumulation).  One step = one complete sampling job
(init_chains + every chain to 2000 draws) through the C ABI; inputs (L,
labels) are resident in HBM before the timed region.

Reported beside it, on the same box and run:
  * the synchronized runtime on the same job (vmap semantics and the
    compacted variant), the FSM/synchronized speed-ups and bit-exactness;
  * NUTS on Bayesian logistic regression (N = 10000, D = 100, step 0.05,
    depth 10, Laplace starts), 8192 chains x 1000 draws, FSM vs synchronized;
  * R(m) of each job estimated from its own loop counts, chain transitions
    per second, and effective samples per second (multi-chain ESS of the
    first coordinates on a subsample of the chains);
  * batching: 32 GP-logistic ESS targets of uneven dim / chains / draws plus a
    65536-chain D=10 funnel under 3-stage delayed rejection, in one batch
    (one graph replay per round, autotuned), against the same jobs run one
    after another; bit-identical outputs checked;
  * serving: a Poisson stream of ESS-GP and NUTS jobs of random sizes through
    the continuous-batching server, against one-job-at-a-time on the same
    stream: p50/p99 latency and draws/s, bit-identical outputs checked;
  * the live roofline figure of the dominant kernel (HIP events);
  * the FP64 CPU oracle timed on a bounded sample of the ESS workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "draws/sec FSM vs synchronized (ESS, NUTS, 8192 chains); p50/p99 job latency"
PEAK_MFMA_F32 = 157.3  # TFLOP/s, MI355X dense FP32 MFMA
PEAK_MFMA_BF16 = 2500.0  # TFLOP/s, MI355X dense bf16 MFMA
# The D = 1024 ellipse GEMM and the NUTS gradient compute each FP32 product as
# six bf16 piece products (exact three-piece splits of both operands), so their
# ceiling in FP32-equivalent flops is the bf16 peak over six.
PIECE_PRODUCTS = 6
PEAK_GEMM = PEAK_MFMA_BF16 / PIECE_PRODUCTS


def gemm_source_digest():
    """SHA-256 of the ellipse GEMM's device code (the "ellipse GEMM" section of ess_device.h)."""
    src = open(os.path.join(ROOT, "paper_2503_17405_amd", "csrc", "ess_device.h")).read()
    a = src.index("// ------------------------------------------------------------ ellipse GEMM")
    b = src.index("// ------------------------------------------------------------ ESS blocks", a)
    return hashlib.sha256(src[a:b].encode()).hexdigest()


def stored_traffic():
    """HBM bytes per full-window launch of the ellipse GEMM, from the committed rocprofv3
    counter summary -- None if the kernel source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "nu_gemm_d1024_traffic.md")
    try:
        txt = open(path).read()
        cur = gemm_source_digest()
    except (OSError, ValueError):
        return None
    m1 = re.search(r"traffic_bytes_per_launch: (\d+)", txt)
    m2 = re.search(r"ellipse GEMM source sha256: ([0-9a-f]{64})", txt)
    if not (m1 and m2) or m2.group(1) != cur:
        return None
    return int(m1.group(1))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def checksum(out, m_chunk=256):
    """Exact integer checksum of a float32 tensor (bit patterns summed in int64)."""
    import torch
    s = 0
    for i in range(0, out.shape[0], m_chunk):
        s += int(out[i:i + m_chunk].view(torch.int32).to(torch.int64).sum().item())
    return s


def ess_report(out, seconds, chains=256, coords=4):
    """Effective samples per second of the first `coords` coordinates, from the
    draws of the first `chains` chains (chains are i.i.d., so the sum over all
    chains scales by m / chains); the minimum over the coordinates is reported."""
    from paper_2503_17405_amd import diagnostics as Dx
    m = out.shape[0]
    c = min(chains, m)
    sub = out[:c, :, :coords].double().cpu().numpy()
    e = Dx.ess(sub) * (m / c)
    return dict(ess_per_s=float(e.min() / seconds), ess_min=float(e.min()), ess_mean=float(e.mean()),
                sample="chains 0..%d, coordinates 0..%d, all draws" % (c - 1, coords - 1))


def timed_jobs(make, run, steps, warmup):
    import torch
    for i in range(warmup):
        job = make()
        run(job)
        job.free()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = None
    marks = [t0]
    for i in range(steps):
        if last is not None:
            last.free()
        last = make()
        run(last)
        torch.cuda.synchronize()
        marks.append(time.perf_counter())
        log("  job %d: %.3f s" % (i, marks[-1] - t0))
    dt = (marks[-1] - t0) / steps
    STEP_TIMES.append([b - a for a, b in zip(marks[:-1], marks[1:])])
    return dt, last


STEP_TIMES = []  # per-step wall times of every timed_jobs call (the last one is read by the caller)


def spread(times):
    import numpy as np
    t = np.asarray(times, dtype=np.float64)
    return dict(median_s=float(np.median(t)), min_s=float(t.min()), max_s=float(t.max()), repeats=int(t.size))


def bench_ess(F, ctx, args):
    import torch

    from paper_2503_17405_amd import diagnostics as Dx
    from paper_2503_17405_amd import inputs
    m, n, D = args.chains, args.draws, 1024
    w = inputs.gp_logistic(dim=D, lengthscale=0.05, jitter=1e-5, seed=2001)
    seed = 2002
    L = torch.tensor(w["L"], dtype=torch.float32, device="cuda")
    y = torch.tensor(w["y"], dtype=torch.float32, device="cuda")
    out = torch.empty((m, n, D), dtype=torch.float32, device="cuda")
    target, sampler = F.gp_target(L, y), F.ess_sampler(F.F32)
    def make(timing=True):
        return F.Job(ctx, target, sampler, m, n, seed, out=out, window=args.window, timing=timing)

    # the FSM job is timed with HIP events around its launches (63 windows: the
    # live roofline of the GEMM); the synchronized baselines issue thousands of
    # launches, so they are timed without events and their kernel breakdown
    # comes from one more run with events
    log("ESS FSM")
    t_fsm, job = timed_jobs(make, lambda j: j.step_fsm(0), args.steps, args.warmup)
    st = job.stats()
    counts = job.counts()
    job.free()
    ref = checksum(out)
    res = dict(seconds=t_fsm, draws_per_s=m * n / t_fsm, steps=st["steps"],
               transitions_per_s=st["steps"] / t_fsm, timing=spread(STEP_TIMES[-1]),
               kernel_ms=st["kernel_ms"], kernel_launches=st["kernel_launches"],
               mean_loop=float(counts.mean()), mean_max_loop=float(counts.max(axis=0).mean()),
               R_hat_m=Dx.r_of_m(counts, m))
    res["effective"] = ess_report(out, t_fsm)
    res["_moments"] = Dx.moments(out[:, :, :4].double().cpu().numpy())
    res["_sample"] = out[:64, :100].double().cpu().numpy()
    g_ms, g_n = st["kernel_ms"][0], st["kernel_launches"][0]
    flops = float(m) * n * D * (D + 1)
    # in the job, each window's GEMM shares the chip with the previous window's FSM kernel
    res["gemm"] = dict(kernel="nu_gemm_mfma_kernel<4>", ms=g_ms, launches=g_n, avg_us=1e3 * g_ms / max(g_n, 1),
                       tflops=flops / (g_ms * 1e-3) / 1e12, flop_per_column=D * (D + 1),
                       flop_per_launch=flops / max(g_n, 1))
    # the same job with a finite step budget runs its windows one after another:
    # the GEMM launches then have the chip to themselves
    log("ESS FSM, windows not overlapped")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    job = make()
    while not job.step_fsm(1 << 40):
        pass
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    si = job.stats()
    job.free()
    gi_ms, gi_n = si["kernel_ms"][0], si["kernel_launches"][0]
    res["gemm_isolated"] = dict(ms=gi_ms, launches=gi_n, avg_us=1e3 * gi_ms / max(gi_n, 1),
                                tflops=flops / (gi_ms * 1e-3) / 1e12,
                                bit_exact_vs_fsm=bool(checksum(out) == ref),
                                job_seconds=t_seq)
    sync = {}
    if not args.no_sync:
        for name, mode in (("vmap", F.SYNC_VMAP), ("compact", F.SYNC_COMPACT)):
            log("ESS sync %s" % name)
            dt, job = timed_jobs(lambda: make(False), lambda j, mode=mode: j.step_synchronized(n, mode),
                                 args.sync_steps, 0)
            s2 = job.stats()
            job.free()
            exact = bool(checksum(out) == ref)
            job = make(True)
            job.step_synchronized(n, mode)
            kms = job.stats()["kernel_ms"]
            job.free()
            sync[name] = dict(seconds=dt, draws_per_s=m * n / dt, steps=s2["steps"],
                              padded_steps=s2["padded_steps"], kernel_ms=kms,
                              bit_exact_vs_fsm=exact, speedup_fsm=dt / t_fsm)
    res["sync"] = sync
    del out
    torch.cuda.empty_cache()
    return res, w, seed


def bench_nuts(F, ctx, args, m=None, light=False):
    """NUTS on the logistic-regression workload (N = 10000, D = 100, step
    0.05, depth 10, Laplace starts).  light: FSM and synchronized timings
    only (no kernel breakdown or oracle samples)."""
    import numpy as np
    import torch

    from paper_2503_17405_amd import diagnostics as Dx
    from paper_2503_17405_amd import inputs
    m = args.nuts_chains if m is None else m
    n, N, D = args.nuts_draws, 10000, 100
    d = inputs.logreg(n_data=N, dim=D, seed=3001)
    lap = inputs.logreg_laplace(d["X"], d["y"], m, seed=3002)
    X = torch.tensor(d["X"], dtype=torch.float32, device="cuda")
    y = torch.tensor(d["y"], dtype=torch.float32, device="cuda")
    x0 = torch.tensor(lap["x0"], dtype=torch.float32, device="cuda")
    out = torch.empty((m, n, D), dtype=torch.float32, device="cuda")
    target, sampler = F.logreg_target(X, y), F.nuts_sampler(0.05, 10)
    seed = 3003
    def make(timing=False):
        return F.Job(ctx, target, sampler, m, n, seed, x0=x0, out=out, timing=timing)

    # timed without per-launch events (thousands of steps); the kernel
    # breakdown comes from one more FSM run with events
    log("NUTS FSM")
    t_fsm, job = timed_jobs(make, lambda j: j.step_fsm(0), args.nuts_steps, args.nuts_warmup)
    st = job.stats()
    counts = job.counts()
    job.free()
    ref = checksum(out)
    job = make(True)
    job.step_fsm(0)
    st_t = job.stats()
    job.free()
    st["kernel_ms"], st["kernel_launches"] = st_t["kernel_ms"], st_t["kernel_launches"]
    res = dict(seconds=t_fsm, draws_per_s=m * n / t_fsm, steps=st["steps"],
               transitions_per_s=st["steps"] / t_fsm,
               kernel_ms=st["kernel_ms"], kernel_launches=st["kernel_launches"],
               mean_loop=float(counts.mean()), mean_max_loop=float(counts.max(axis=0).mean()),
               R_hat_m=Dx.r_of_m(counts, m), divergent_free=bool(np.isfinite(counts).all()))
    res["effective"] = ess_report(out, t_fsm)
    if light:
        job = None
        sync = {}
        if not args.no_sync:
            for name, mode in (("vmap", F.SYNC_VMAP), ("compact", F.SYNC_COMPACT)):
                log("NUTS sync %s (%d chains)" % (name, m))
                dt, job = timed_jobs(make, lambda j, mode=mode: j.step_synchronized(n, mode), 1, 0)
                job.free()
                sync[name] = dict(seconds=dt, draws_per_s=m * n / dt, bit_exact_vs_fsm=bool(checksum(out) == ref),
                                  speedup_fsm=dt / t_fsm)
        res.update(chains=m, draws=n, sync=sync)
        del out
        torch.cuda.empty_cache()
        return res
    res["_check"] = dict(moments=Dx.moments(out[:, :100, :4].double().cpu().numpy()),
                         sample=out[:64, :100].double().cpu().numpy(), X=d["X"], y=d["y"],
                         x0=lap["x0"][:64].astype(np.float32).astype(np.float64), seed=seed, eps=0.05, depth=10)
    g_ms = st["kernel_ms"][0]
    flops = 4.0 * N * D * st["steps"]  # X Theta and X^T r per requested gradient
    g_tf = flops / (g_ms * 1e-3) / 1e12
    res["gradient"] = dict(kernel="logreg_grad_bf16_kernel<4, 13>", ms=g_ms,
                           launches=st["kernel_launches"][0],
                           avg_us=g_ms * 1e3 / max(1, st["kernel_launches"][0]),
                           tflops=g_tf, flop_per_gradient=4 * N * D,
                           roofline=dict(bound="mfma", achieved=g_tf, peak=PEAK_GEMM, unit="TFLOP/s",
                                         frac=g_tf / PEAK_GEMM,
                                         note="FP32 products run as six bf16 piece products: ceiling "
                                              "2500 / 6 TFLOP/s (FP32 MFMA peak 157.3 for scale)"))
    sync = {}
    if not args.no_sync:
        for name, mode in (("vmap", F.SYNC_VMAP), ("compact", F.SYNC_COMPACT)):
            log("NUTS sync %s" % name)
            dt, job = timed_jobs(make, lambda j, mode=mode: j.step_synchronized(n, mode), 1, 0)
            s2 = job.stats()
            job.free()
            sync[name] = dict(seconds=dt, draws_per_s=m * n / dt, steps=s2["steps"],
                              padded_steps=s2["padded_steps"],
                              bit_exact_vs_fsm=bool(checksum(out) == ref), speedup_fsm=dt / t_fsm)
    res["sync"] = sync
    del out
    torch.cuda.empty_cache()
    return res


# Step size of NUTS on the correlated mixture: the paper pre-tunes it to an
# acceptance rate of about 0.85; the value below is the dual-averaging result
# of tune_mog_step_size (run with --tune-mog-eps: 512 chains, 400 iterations,
# averaged step 0.04728, acceptance 0.84-0.86 over the last iterations;
# recorded here so that every run samples the same target with the same step).
MOG_EPS = 0.0473


def tune_mog_step_size(F, ctx, m=512, iters=400, delta=0.85, eps0=0.05, seed=6100):
    """Dual averaging (Hoffman & Gelman 2014, Sec. 3.2) of one step size shared
    by m chains of the 100-D mixture: iteration t draws once from every chain at
    step exp(log_eps_t) and feeds the mean acceptance statistic (sum over all
    leapfrogs of min(1, e^(H0 - H)) / leapfrogs, from fsmmc_job_stats) into
    the averaged iterate.  Constants gamma = 0.05, t0 = 10, kappa = 0.75,
    mu = log(10 eps0)."""
    import math

    import torch

    from paper_2503_17405_amd import inputs
    w = inputs.mog(dim=100, n_chains=m, seed=seed)
    target = F.mog_target(torch.tensor(w["means"], device="cuda"), torch.tensor(w["log_weights"], device="cuda"),
                          torch.tensor(w["prec"], device="cuda"))
    x = torch.tensor(w["x0"], dtype=torch.float32, device="cuda")
    mu, gamma, t0, kappa = math.log(10 * eps0), 0.05, 10.0, 0.75
    hbar, log_eps, log_eps_bar = 0.0, math.log(eps0), 0.0
    for t in range(1, iters + 1):
        job = F.Job(ctx, target, F.nuts_sampler(math.exp(log_eps), 10), m, 1, seed + 17 * t, x0=x)
        job.step_fsm(0)
        st = job.stats()
        x = torch.tensor(job.samples()[:, 0, :], device="cuda")
        job.free()
        alpha = st["accept_sum"] / max(st["steps"], 1)
        hbar = (1 - 1 / (t + t0)) * hbar + (delta - alpha) / (t + t0)
        log_eps = mu - math.sqrt(t) / gamma * hbar
        eta = t ** (-kappa)
        log_eps_bar = eta * log_eps + (1 - eta) * log_eps_bar
        if t % 50 == 0:
            log("  dual averaging %d: eps %.5f, averaged %.5f, acceptance %.3f" %
                (t, math.exp(log_eps), math.exp(log_eps_bar), alpha))
    return math.exp(log_eps_bar)


def bench_mog(F, ctx, args):
    """NUTS on the 100-D correlated mixture (rho 0.99, modes -10 1, 0, +10 1),
    n = 1000 draws, depth 10, FSM vs synchronized for several chain counts."""
    import numpy as np
    import torch

    from paper_2503_17405_amd import inputs
    eps = args.mog_eps
    res = dict(workload="NUTS on a 100-D mixture of three Gaussians sharing Sigma = 0.01 I + 0.99 1 1^T, "
                        "means -10 1, 0, +10 1, equal weights; step %.4g, depth 10, identity mass, "
                        "exact mixture draws as starts, %d draws, FP32" % (eps, args.mog_draws),
               step_size=eps, runs={})
    n, D = args.mog_draws, 100
    for m in args.mog_chains:
        w = inputs.mog(dim=D, n_chains=m, seed=6001)
        target = F.mog_target(torch.tensor(w["means"], device="cuda"),
                              torch.tensor(w["log_weights"], device="cuda"), torch.tensor(w["prec"], device="cuda"))
        x0 = torch.tensor(w["x0"], dtype=torch.float32, device="cuda")
        out = torch.empty((m, n, D), dtype=torch.float32, device="cuda")
        sampler = F.nuts_sampler(eps, 10)

        def make(timing=False):
            return F.Job(ctx, target, sampler, m, n, 6002, x0=x0, out=out, timing=timing)

        log("MoG NUTS FSM, m=%d" % m)
        t_fsm, job = timed_jobs(make, lambda j: j.step_fsm(0), 1, 1)
        st = job.stats()
        counts = job.counts()
        job.free()
        ref = checksum(out)
        r = dict(chains=m, seconds=t_fsm, draws_per_s=m * n / t_fsm, leapfrogs=st["steps"],
                 leapfrogs_per_s=st["steps"] / t_fsm, mean_loop=st["mean_loops"],
                 mean_max_loop=st["mean_max_loops"], R_hat_m=st["r_hat"],
                 p_loop_over_1000=float((counts > 1000).mean()),
                 p_loop_under_20=float((counts < 20).mean()),
                 acceptance=st["accept_sum"] / max(st["steps"], 1))
        r["effective"] = ess_report(out, t_fsm, chains=min(m, 256))
        sync = {}
        if not args.no_sync:
            for name, mode in (("vmap", F.SYNC_VMAP), ("compact", F.SYNC_COMPACT)):
                log("MoG NUTS sync %s, m=%d" % (name, m))
                dt, job = timed_jobs(make, lambda j, mode=mode: j.step_synchronized(n, mode), 1, 0)
                s2 = job.stats()
                job.free()
                sync[name] = dict(seconds=dt, draws_per_s=m * n / dt, leapfrogs=s2["steps"],
                                  padded=s2["padded_steps"], bit_exact_vs_fsm=bool(checksum(out) == ref),
                                  speedup_fsm=dt / t_fsm)
        r["sync"] = sync
        if sync:
            r["speedup_vs_vmap"] = sync["vmap"]["speedup_fsm"]
            r["speedup_vs_compact"] = sync["compact"]["speedup_fsm"]
        log("  m=%d: FSM %.3f s (%.3g draws/s), R(m) %.2f%s" %
            (m, t_fsm, m * n / t_fsm, st["r_hat"],
             "" if not sync else ", vmap %.2fx, compact %.2fx" % (r["speedup_vs_vmap"], r["speedup_vs_compact"])))
        res["runs"][str(m)] = r
        del out
        torch.cuda.empty_cache()
    return res


def _lane_runs(F, ctx, target, sampler, m, n, seed, D, args, fsm_variants):
    """FSM (one or more FSM shapes) vs synchronized runs of one lane-per-chain job."""
    import torch
    out = torch.empty((m, n, D), dtype=torch.float32, device="cuda")

    def make(states=0):
        return F.Job(ctx, target, sampler, m, n, seed, out=out, fsm_states=states)

    r = dict(chains=m, draws=n)
    ref = None
    for name, states in fsm_variants:
        t, job = timed_jobs(lambda: make(states), lambda j: j.step_fsm(0), 1, 1)
        st = job.stats()
        job.free()
        cs = checksum(out)
        ref = cs if ref is None else ref
        r[name] = dict(seconds=t, draws_per_s=m * n / t, steps=st["steps"], mean_loop=st["mean_loops"],
                       mean_max_loop=st["mean_max_loops"], R_hat_m=st["r_hat"],
                       lane_occupancy=st["active_lanes"] / max(st["lane_slots"], 1),
                       bit_exact_vs_first=bool(cs == ref))
    t_fsm = r[fsm_variants[0][0]]["seconds"]
    if not args.no_sync:
        for name, mode in (("vmap", F.SYNC_VMAP), ("compact", F.SYNC_COMPACT)):
            t, job = timed_jobs(make, lambda j, mode=mode: j.step_synchronized(n, mode), 1, 0)
            st = job.stats()
            job.free()
            r["sync_" + name] = dict(seconds=t, draws_per_s=m * n / t, steps=st["steps"],
                                     padded_steps=st["padded_steps"],
                                     lane_occupancy=st["active_lanes"] / max(st["lane_slots"], 1),
                                     bit_exact_vs_fsm=bool(checksum(out) == ref), speedup_fsm=t / t_fsm)
    del out
    torch.cuda.empty_cache()
    return r


def bench_drsym(F, ctx, args):
    """Symmetric delayed rejection on N(0, 1) (M = 100 tries, N(., 0.1^2)
    re-centred proposals, 10^4 draws per chain): condensed FSM, the four-state
    FSM, and the synchronized runtime."""
    import torch
    tg = F.gauss_target(torch.ones(1, device="cuda"))
    sampler = F.drsym_sampler(100, 0.1)
    res = dict(workload="symmetric DR on N(0,1), M=100 tries, proposal sd 0.1 re-centred on the last "
                        "rejection, %d draws per chain, FP32, lane per chain" % args.drsym_draws, runs={})
    for m in args.drsym_chains:
        log("DRSYM m=%d" % m)
        r = _lane_runs(F, ctx, tg, sampler, m, args.drsym_draws, 7001, 1, args,
                       [("fsm_condensed", 1), ("fsm_4state", 4)])
        r["bundling_gain"] = r["fsm_4state"]["seconds"] / r["fsm_condensed"]["seconds"]
        log("  condensed %.3f s, 4-state %.3f s (bundling %.2fx)%s" % (
            r["fsm_condensed"]["seconds"], r["fsm_4state"]["seconds"], r["bundling_gain"],
            "" if "sync_vmap" not in r else ", vmap %.2fx, compact %.2fx, R(m) %.2f" % (
                r["sync_vmap"]["speedup_fsm"], r["sync_compact"]["speedup_fsm"], r["fsm_condensed"]["R_hat_m"])))
        res["runs"][str(m)] = r
    return res


def bench_slice(F, ctx, args):
    """Slice sampling along random directions on the D = 10 funnel (width 1)."""
    tg = F.funnel_target(10)
    sampler = F.slice_sampler(1.0)
    res = dict(workload="slice sampling along random directions (stepping out + shrinkage, width 1) on the "
                        "D=10 Neal funnel, %d draws per chain, FP32, lane per chain, FSM transition "
                        "generated from the sample program" % args.slice_draws, runs={})
    for m in args.slice_chains:
        log("SLICE m=%d" % m)
        r = _lane_runs(F, ctx, tg, sampler, m, args.slice_draws, 8001, 10, args, [("fsm", 0)])
        log("  FSM %.3f s (%.3g draws/s)%s" % (
            r["fsm"]["seconds"], r["fsm"]["draws_per_s"],
            "" if "sync_vmap" not in r else ", vmap %.2fx, compact %.2fx, R(m) %.2f" % (
                r["sync_vmap"]["speedup_fsm"], r["sync_compact"]["speedup_fsm"], r["fsm"]["R_hat_m"])))
        res["runs"][str(m)] = r
    return res


def bench_gphyper(F, ctx, args):
    """ESS on GP-regression hyperparameters (tau, lambda, sigma), N(0, I) prior,
    marginal likelihood through an FP64 Cholesky of the n x n kernel matrix
    inside every loop iteration; FSM vs synchronized for n in args.gph_obs."""
    import torch

    from paper_2503_17405_amd import inputs
    res = dict(workload="ESS on GP-regression hyperparameters: n observations with 6 inputs (synthetic "
                        "stand-in for the 6-feature regression data), N(0,I) prior on (tau, lambda, sigma), "
                        "FP64 Cholesky per likelihood, %d chains x %d draws (%d draws for n > 128); the "
                        "chain's wave factors each matrix for n <= 96, a block of four waves above"
                        % (args.gph_chains, args.gph_draws, args.gph_big_draws),
               runs={})
    m = args.gph_chains
    for nobs in args.gph_obs:
        n = args.gph_draws if nobs <= 128 else args.gph_big_draws
        w = inputs.gp_hyper(n=nobs, n_chains=m, seed=9001)
        tg = F.gp_hyper_target(torch.tensor(w["X"], device="cuda"), torch.tensor(w["y"], device="cuda"),
                               w["jitter"])
        x0 = torch.tensor(w["x0"], device="cuda")
        out = torch.empty((m, n, 3), dtype=torch.float64, device="cuda")
        sampler = F.ess_sampler(F.F64)

        def make():
            return F.Job(ctx, tg, sampler, m, n, 9002, x0=x0, out=out)

        log("GP hyper n=%d" % nobs)
        t_fsm, job = timed_jobs(make, lambda j: j.step_fsm(0), 1, 1)
        st = job.stats()
        job.free()
        ref = checksum(out.view(torch.float32))
        r = dict(obs=nobs, draws=n, seconds=t_fsm, draws_per_s=m * n / t_fsm, likelihoods=st["steps"],
                 likelihoods_per_s=st["steps"] / t_fsm, cholesky_flop_per_likelihood=nobs ** 3 / 3.0,
                 mean_loop=st["mean_loops"], mean_max_loop=st["mean_max_loops"], R_hat_m=st["r_hat"])
        sync = {}
        if not args.no_sync:
            for name, mode in (("vmap", F.SYNC_VMAP), ("compact", F.SYNC_COMPACT)):
                dt, job = timed_jobs(make, lambda j, mode=mode: j.step_synchronized(n, mode), 1, 0)
                s2 = job.stats()
                job.free()
                sync[name] = dict(seconds=dt, draws_per_s=m * n / dt, padded=s2["padded_steps"],
                                  bit_exact_vs_fsm=bool(checksum(out.view(torch.float32)) == ref),
                                  speedup_fsm=dt / t_fsm)
        r["sync"] = sync
        log("  n=%d: FSM %.3f s, R(m) %.2f%s" % (nobs, t_fsm, st["r_hat"], "" if not sync else
            ", vmap %.2fx, compact %.2fx" % (sync["vmap"]["speedup_fsm"], sync["compact"]["speedup_fsm"])))
        res["runs"][str(nobs)] = r
        del out
        torch.cuda.empty_cache()
    return res


def _ess_job_data(F, D, ds, cache):
    import torch

    from paper_2503_17405_amd import inputs
    if (D, ds) not in cache:
        w = inputs.gp_logistic(dim=D, lengthscale=0.05, jitter=1e-5, seed=ds)
        cache[(D, ds)] = (torch.tensor(w["L"], dtype=torch.float32, device="cuda"),
                          torch.tensor(w["y"], dtype=torch.float32, device="cuda"))
    L, y = cache[(D, ds)]
    return F.gp_target(L, y)


def bench_batch(F, ctx, args):
    """Uneven batch: 32 ESS GP-logistic targets + the 65536-chain funnel."""
    import torch

    from paper_2503_17405_amd import inputs
    spec = inputs.ess_uneven_targets()
    cache = {}
    jobs_spec = [("ess", s["dim"], s["n_chains"], s["n_draws"], s["data_seed"], s["chain_seed"]) for s in spec]
    jobs_spec.append(("dr", 10, args.funnel_chains, 1000, 0, 4002))
    outs = [torch.empty((m, n, D), dtype=torch.float32, device="cuda") for _, D, m, n, _, _ in jobs_spec]
    draws = sum(m * n for _, _, m, n, _, _ in jobs_spec)

    def make(k):
        kind, D, m, n, ds, cs = jobs_spec[k]
        if kind == "ess":
            return F.Job(ctx, _ess_job_data(F, D, ds, cache), F.ess_sampler(), m, n, cs, out=outs[k])
        return F.Job(ctx, F.funnel_target(D), F.dr_sampler((1.0, 0.3, 0.1)), m, n, cs, out=outs[k])

    log("C4 batch (%d jobs, %d draws)" % (len(jobs_spec), draws))
    jobs = [make(k) for k in range(len(jobs_spec))]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = F.Batch(ctx, jobs, autotune=True)
    b.run(0)
    t_batch = time.perf_counter() - t0
    st = b.stats()
    b.free()
    for j in jobs:
        j.free()
    sums = [checksum(o) for o in outs]
    from paper_2503_17405_amd import diagnostics as Dx
    check = dict(moments=Dx.moments(outs[-1][:, :200, :4].double().cpu().numpy()),
                 sample=outs[-1][:64, :200].double().cpu().numpy(), seed=jobs_spec[-1][5], dim=10)
    log("C4 one job at a time")
    t_alone = 0.0
    for k in range(len(jobs_spec)):
        j = make(k)
        j.sync()
        t1 = time.perf_counter()
        while not j.step_fsm(0):
            pass
        t_alone += time.perf_counter() - t1
        j.free()
    same = all(checksum(o) == s for o, s in zip(outs, sums))
    del outs
    torch.cuda.empty_cache()
    return dict(workload="32 GP-logistic ESS targets (D~U{64..1024}, m~U{256..2048}, n~U{200..2000}) + "
                         "3-stage DR on the D=10 funnel (%d chains x 1000 draws), FP32" % args.funnel_chains,
                jobs=len(jobs_spec), draws=draws, batch_s=t_batch, alone_s=t_alone,
                draws_per_s_batch=draws / t_batch, draws_per_s_alone=draws / t_alone,
                speedup=t_alone / t_batch, bit_exact_vs_alone=bool(same), rounds=st["rounds"],
                captures=st["captures"], gpu_ms=st["gpu_ms"], _check=check, tuned=dict(window=st["window"],
                dr_chunk=st["dr_chunk"], gemm_cols=st["gemm_cols"], trials=st["tune_trials"],
                tune_ms=st["tune_ms"]))


def serve_stream(n_jobs, seed):
    """Job list of the serving stream: Poisson arrivals at 50 jobs/s, half
    ESS GP-logistic (D~U{64..1024}), half NUTS logistic regression
    (D~U{10..100}, N~U{1000..10000}), m~U{16..1024}, n~U{200..2000}."""
    import numpy as np
    g = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for k in range(n_jobs):
        t += g.exponential(0.02)
        m = int(g.integers(16, 1025))
        n = int(g.integers(200, 2001))
        if g.uniform() < 0.5:
            out.append(dict(kind="ess", t=t, m=m, n=n, D=int(g.integers(64, 1025)),
                            data_seed=int(g.integers(1 << 31)), seed=int(g.integers(1 << 62))))
        else:
            out.append(dict(kind="nuts", t=t, m=m, n=n, D=int(g.integers(10, 101)),
                            N=int(g.integers(1000, 10001)), data_seed=int(g.integers(1 << 31)),
                            seed=int(g.integers(1 << 62))))
    return out


def nuts_step_cost(F):
    """Microseconds per NUTS runtime step (transition, compaction, gradient)
    for small logistic-regression jobs of the serving mix, alone (single-job
    API) and as the only job of a server (its batch rounds of 16 steps);
    wall time over the steps issued, same draws both ways."""
    import numpy as np
    import torch

    from paper_2503_17405_amd import inputs
    ctx = F.Context(0)
    res = []
    for m, D, N, n in [(16, 10, 1000, 40), (128, 50, 5000, 20), (1024, 20, 2000, 20)]:
        d = inputs.logreg(n_data=N, dim=D, seed=7)
        lap = inputs.logreg_laplace(d["X"], d["y"], m, seed=8)
        eps = min(0.05, 1.0 / np.sqrt(float(np.linalg.eigvalsh(lap["hessian"])[-1])))
        X = torch.tensor(d["X"], dtype=torch.float32, device="cuda")
        y = torch.tensor(d["y"], dtype=torch.float32, device="cuda")
        x0 = torch.tensor(lap["x0"], dtype=torch.float32, device="cuda")
        tg, smp = F.logreg_target(X, y), F.nuts_sampler(eps, 10)
        outs = []
        for timing in (True, False):  # the timed run counts the steps, the untimed one is clocked
            out = torch.empty((m, n, D), dtype=torch.float32, device="cuda")
            j = F.Job(ctx, tg, smp, m, n, 11, x0=x0, out=out, timing=timing)
            t0 = time.perf_counter()
            while not j.step_fsm(0):
                pass
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            st = j.stats()
            j.free()
            if timing:
                steps = st["kernel_launches"][0]
            outs.append(out)
        srv = F.Server(ctx)
        out_s = torch.empty_like(outs[1])
        srv.submit(tg, smp, m, n, 11, out_s, x0=x0)
        while not srv.wait(10.0):
            pass
        rec = srv.poll(8)[0]
        sst = srv.stats()
        srv.close()
        ssteps = 16 * sst["rounds"]
        res.append(dict(m=m, D=D, N=N, n=n, steps_alone=int(steps), us_per_step_alone=wall / steps * 1e6,
                        steps_server=int(ssteps), us_per_step_server=(rec["t_done"] - rec["t_admit"]) / ssteps * 1e6,
                        same=bool(torch.equal(outs[1], out_s) and torch.equal(outs[0], outs[1]))))
        log("  NUTS step m=%d D=%d N=%d: %.1f us alone (%d steps), %.1f us in the server (%d steps)"
            % (m, D, N, res[-1]["us_per_step_alone"], steps, res[-1]["us_per_step_server"], ssteps))
    ctx.close()
    return res


def bench_serve(F, args):
    import numpy as np
    import torch

    from paper_2503_17405_amd import inputs
    step_cost = nuts_step_cost(F)
    stream = serve_stream(args.serve_jobs, 5001)
    log("C5 stream: %d jobs, preparing inputs" % len(stream))
    t0 = time.perf_counter()
    cache, data = {}, []
    for js in stream:
        if js["kind"] == "ess":
            tgt = _ess_job_data(F, js["D"], js["data_seed"], cache)
            data.append((tgt, F.ess_sampler(), None))
        else:
            d = inputs.logreg(n_data=js["N"], dim=js["D"], seed=js["data_seed"])
            lap = inputs.logreg_laplace(d["X"], d["y"], js["m"], seed=js["data_seed"] + 1)
            lam = float(np.linalg.eigvalsh(lap["hessian"])[-1])
            eps = min(0.05, 1.0 / np.sqrt(lam))
            X = torch.tensor(d["X"], dtype=torch.float32, device="cuda")
            y = torch.tensor(d["y"], dtype=torch.float32, device="cuda")
            x0 = torch.tensor(lap["x0"], dtype=torch.float32, device="cuda")
            data.append((F.logreg_target(X, y), F.nuts_sampler(eps, 10), x0))
            js["eps"] = eps
    outs = [torch.empty((js["m"], js["n"], js["D"]), dtype=torch.float32, device="cuda") for js in stream]
    torch.cuda.synchronize()
    prep_s = time.perf_counter() - t0
    draws = sum(js["m"] * js["n"] for js in stream)

    def latencies(lat):
        lat = np.sort(np.asarray(lat))
        return dict(p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                    mean_s=float(lat.mean()), max_s=float(lat.max()))

    log("C5 server")
    ctx = F.Context(0, hbm_budget_bytes=args.serve_budget_gib << 30)
    srv = F.Server(ctx)
    ids = []
    start = F.clock()
    for k, js in enumerate(stream):
        while F.clock() - start < js["t"]:
            time.sleep(min(0.002, max(0.0, js["t"] - (F.clock() - start))))
        tgt, smp, x0 = data[k]
        ids.append(srv.submit(tgt, smp, js["m"], js["n"], js["seed"], outs[k], x0=x0))
    log("  all %d jobs submitted after %.2f s" % (len(stream), F.clock() - start))
    while not srv.wait(10.0):
        st = srv.stats()
        log("  server: %d/%d done, %d live, %d pending, %.1f s" % (st["completed"], len(stream), st["live_jobs"],
                                                                  st["pending_jobs"], F.clock() - start))
    recs = {r["job_id"]: r for r in srv.poll(len(stream) + 8)}
    sst = srv.stats()
    srv.close()
    ctx.close()
    ok = all(recs[i]["status"] == F.OK for i in ids)
    lat_srv = [recs[i]["t_done"] - recs[i]["t_submit"] for i in ids]
    # submission to admission (state allocated, initialisation queued): the
    # request loop admits while the device runs its queued rounds, so this is
    # the wait for the loop plus any wait for HBM budget; the job then joins
    # the batch at the next round boundary
    adm = np.sort(np.asarray([recs[i]["t_admit"] - recs[i]["t_submit"] for i in ids]))
    span_srv = max(recs[i]["t_done"] for i in ids) - start
    log("  server: span %.2f s, p50 %.2f s, p99 %.2f s" % (span_srv, np.percentile(lat_srv, 50),
                                                        np.percentile(lat_srv, 99)))
    sums = [checksum(o) for o in outs]

    log("C5 one job at a time")
    ctx = F.Context(0)
    start = F.clock()
    lat_one, t_done = [], 0.0
    for k, js in enumerate(stream):
        now = F.clock() - start
        if now < js["t"]:
            time.sleep(js["t"] - now)
        tgt, smp, x0 = data[k]
        j = F.Job(ctx, tgt, smp, js["m"], js["n"], js["seed"], x0=x0, out=outs[k], window=16)
        while not j.step_fsm(0):
            pass
        j.free()
        t_done = F.clock() - start
        lat_one.append(t_done - js["t"])
        log("  job %d (%s m=%d n=%d D=%d): done at %.2f s" % (k, js["kind"], js["m"], js["n"], js["D"], t_done))
    ctx.close()
    same = all(checksum(o) == s for o, s in zip(outs, sums))
    del outs
    torch.cuda.empty_cache()
    return dict(workload="%d jobs, Poisson arrivals at 50 jobs/s; ESS GP-logistic D~U{64..1024} or NUTS "
                         "logistic regression D~U{10..100}, N~U{1000..10000}; m~U{16..1024}, "
                         "n~U{200..2000}; FP32" % len(stream),
                prefix="the first %d jobs of the configured 2000-job stream (same generator and seed); "
                       "the one-job-at-a-time leg of the whole stream would take about %.0f minutes at "
                       "this prefix's rate" % (len(stream), t_done / len(stream) * 2000 / 60.0)
                       if len(stream) < 2000 else None,
                jobs=len(stream), draws=draws, host_prep_s=prep_s, all_ok=bool(ok), nuts_step_us=step_cost,
                bit_exact_vs_alone=bool(same), hbm_budget_gib=args.serve_budget_gib,
                server=dict(draws_per_s=draws / span_srv, span_s=span_srv, **latencies(lat_srv),
                            rounds=sst["rounds"], gpu_ms=sst["gpu_ms"], peak_live_jobs=sst["peak_live_jobs"],
                            admit_wait_p50_s=float(np.percentile(adm, 50)),
                            admit_wait_p99_s=float(np.percentile(adm, 99)),
                            peak_state_gib=sst["peak_bytes"] / 2 ** 30),
                one_at_a_time=dict(draws_per_s=draws / t_done, span_s=t_done, **latencies(lat_one)),
                throughput_gain=(draws / span_srv) / (draws / t_done))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, seed, chains, draws, threads, gpu_moments=None):
    """The FP64 oracle on the host cores: chains x draws of the ESS workload
    (the first chains of the benchmark job, same seed).  Its draws also give
    the posterior-moment check: first four coordinates, GPU (all chains) vs
    oracle, in units of the combined Monte Carlo standard error."""
    from oracle import oracle as O
    from paper_2503_17405_amd import diagnostics as Dx
    tg = O.gp_target(w["y"])
    sp = O.ess_sampler(w["L"])
    t0 = time.perf_counter()
    R, _, _ = O.run_chains(tg, sp, seed, range(chains), draws, threads=threads)
    dt = time.perf_counter() - t0
    res = dict(value=chains * draws / dt, unit="draws/s", cores=threads, kind="oracle",
               sample="ESS workload: %d chains x first %d draws, FP64, %d threads, %.1f s"
                      % (chains, draws, threads, dt),
               host_cpus=os.cpu_count(), cpu_model=cpu_model(),
               threads_note="one GPU's share of the box's host cores is 16; the oracle uses one "
                            "thread per core of that share")
    if gpu_moments is not None:
        om = Dx.moments(R[:, :, :4])
        z = Dx.z_scores(gpu_moments, om)
        res["posterior_moments_vs_gpu"] = dict(
            coordinates=[0, 1, 2, 3], gpu_mean=[float(v) for v in gpu_moments["mean"]],
            oracle_mean=[float(v) for v in om["mean"]], gpu_var=[float(v) for v in gpu_moments["var"]],
            oracle_var=[float(v) for v in om["var"]], **z,
            note="GPU: every chain of the FP32 job; oracle: the FP64 chains above; |z| in units of "
                 "the combined MCSE")
    return res, R


def parted_fraction(G, R, tol=1e-4):
    """Fraction of chains whose GPU draws leave the oracle's (relative error
    above tol at some draw of the window): the flip fraction of the parity
    tests, where a chain parts at a near-tie accept/reject decision."""
    import numpy as np
    num = np.linalg.norm(G - R, axis=2)
    den = np.maximum(np.linalg.norm(R, axis=2), 1e-30)
    bad = (num / den > tol).any(axis=1)
    return dict(chains=int(G.shape[0]), draws=int(G.shape[1]), parted=int(bad.sum()),
                flip_frac=float(bad.mean()), tol=tol)


def oracle_checks(ess_sample, R_ess, nuts_check, batch_check, threads):
    """Posterior moments against the FP64 oracle in MCSE units and the flip
    fraction, for the C2 (ESS), C3 (NUTS) and C4 (DR) jobs of this run; the
    oracle runs here, in the CPU leg, on bounded samples."""
    import numpy as np

    from oracle import oracle as O
    from paper_2503_17405_amd import diagnostics as Dx
    out = {}
    if ess_sample is not None and R_ess is not None:
        k = min(ess_sample.shape[0], R_ess.shape[0])
        n = min(ess_sample.shape[1], R_ess.shape[1])
        out["C2_ess"] = parted_fraction(ess_sample[:k, :n], R_ess[:k, :n])
    if nuts_check is not None:
        c = nuts_check
        t0 = time.perf_counter()
        tg = O.logreg_target(c["X"].astype(np.float64), c["y"])
        m, n = c["sample"].shape[0], c["sample"].shape[1]
        R, _, _ = O.run_chains(tg, O.nuts_sampler(c["eps"], c["depth"]), c["seed"], range(m), n, x0=c["x0"],
                               threads=threads)
        z = Dx.z_scores(c["moments"], Dx.moments(R[:, :, :4]))
        out["C3_nuts"] = dict(flip=parted_fraction(c["sample"], R), **z,
                              oracle_sample="%d chains x %d draws, %.1f s" % (m, n, time.perf_counter() - t0),
                              note="moments of the first 100 draws (the oracle sample's window): GPU every "
                                   "chain, oracle the sample; first four coordinates")
    if batch_check is not None:
        c = batch_check
        t0 = time.perf_counter()
        tg, sp = O.funnel_target(c["dim"]), O.dr_sampler((1.0, 0.3, 0.1))
        Rm, _, _ = O.run_chains(tg, sp, c["seed"], range(1024), c["sample"].shape[1], threads=threads)
        m = c["sample"].shape[0]
        z = Dx.z_scores(c["moments"], Dx.moments(Rm[:, :, :4]))
        out["C4_dr"] = dict(flip=parted_fraction(c["sample"], Rm[:m]), **z,
                            oracle_sample="1024 chains x %d draws, %.1f s" % (c["sample"].shape[1],
                                                                             time.perf_counter() - t0),
                            note="funnel D=10: coordinate 0 is v; moments of the first 200 draws (the oracle "
                                 "sample's window): GPU every chain of the 65536-chain job, oracle the sample; "
                                 "the x coordinates are heavy-tailed, so their variance MCSE is rough")
    return out


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
    ap.add_argument("--nuts-c3-chains", type=int, default=4096,
                    help="also run the logistic-regression NUTS job at this chain count (0: skip)")
    ap.add_argument("--no-mog", action="store_true")
    ap.add_argument("--mog-chains", type=int, nargs="+", default=[100, 500, 4096])
    ap.add_argument("--mog-draws", type=int, default=1000)
    ap.add_argument("--mog-eps", type=float, default=MOG_EPS)
    ap.add_argument("--tune-mog-eps", action="store_true",
                    help="run dual averaging for the mixture's step size and exit")
    ap.add_argument("--no-drsym", action="store_true")
    ap.add_argument("--drsym-chains", type=int, nargs="+", default=[1024, 65536])
    ap.add_argument("--drsym-draws", type=int, default=10000)
    ap.add_argument("--no-slice", action="store_true")
    ap.add_argument("--slice-chains", type=int, nargs="+", default=[1024, 65536])
    ap.add_argument("--slice-draws", type=int, default=1000)
    ap.add_argument("--no-gph", action="store_true")
    ap.add_argument("--gph-obs", type=int, nargs="+", default=[25, 100, 414])
    ap.add_argument("--gph-big-draws", type=int, default=100)
    ap.add_argument("--gph-chains", type=int, default=1024)
    ap.add_argument("--gph-draws", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sync", action="store_true")
    ap.add_argument("--cpu-draws", type=int, default=2000)
    ap.add_argument("--cpu-chains-per-thread", type=int, default=16)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--funnel-chains", type=int, default=65536)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-jobs", type=int, default=40)
    ap.add_argument("--serve-budget-gib", type=int, default=64)
    ap.add_argument("--no-ceilings", action="store_true")
    ap.add_argument("--calib-copy-gib", type=int, default=0,
                    help="also run a plain device copy of this many GiB (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU: the chains are independent and this build runs on a "
              "single MI355X (--gpus %d is not supported)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2503_17405_amd import fsmmc as F

    if args.calib_copy_gib > 0:
        a = torch.empty(args.calib_copy_gib << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log("calibration copy: %d GiB read, %d GiB written" % (args.calib_copy_gib, args.calib_copy_gib))
        del a, b
        torch.cuda.empty_cache()

    ceilings = None
    if not args.no_ceilings and not args.tune_mog_eps:
        # the units' measured rates beside the spec peaks the rooflines use
        meas = F.measure_ceilings(0)
        ceilings = dict(measured=meas, spec=dict(
            hbm_gbps=8000.0, mfma_bf16_tflops=PEAK_MFMA_BF16, mfma_f32_tflops=PEAK_MFMA_F32,
            valu_f32_tflops=157.3, valu_f64_tflops=78.6,
            note="spec FP32 vector 157.3 counts packed FP32 (two lanes' worth per instruction); this "
                 "library never emits packed FP32, so its vector FP32 ceiling is half of that"))
        log("ceilings: copy %.0f GB/s, bf16 MFMA %.0f TFLOP/s, FP32 MFMA %.1f, FP32 FMA %.1f, FP64 FMA %.1f, "
            "exp2 %.0f G/s" % (meas["hbm_copy_gbps"], meas["mfma_bf16_tflops"], meas["mfma_f32_tflops"],
                               meas["valu_f32_tflops"], meas["valu_f64_tflops"], meas["exp_f32_gops"]))
    ctx = F.Context(0)
    if args.tune_mog_eps:
        eps = tune_mog_step_size(F, ctx)
        print(json.dumps({"mog_step_size": eps}))
        ctx.close()
        return
    ess, w, seed = bench_ess(F, ctx, args)
    log("ESS: FSM %.3g draws/s" % ess["draws_per_s"])
    nuts = nuts_c3 = None
    if not args.no_nuts:
        nuts = bench_nuts(F, ctx, args)
        log("NUTS: FSM %.3g draws/s" % nuts["draws_per_s"])
        if args.nuts_c3_chains > 0:
            nuts_c3 = bench_nuts(F, ctx, args, m=args.nuts_c3_chains, light=True)
            log("NUTS (%d chains): FSM %.3g draws/s" % (args.nuts_c3_chains, nuts_c3["draws_per_s"]))
    mog = None
    if not args.no_mog:
        mog = bench_mog(F, ctx, args)
    drsym = None if args.no_drsym else bench_drsym(F, ctx, args)
    slc = None if args.no_slice else bench_slice(F, ctx, args)
    gph = None if args.no_gph else bench_gphyper(F, ctx, args)
    batch = None
    if not args.no_batch:
        batch = bench_batch(F, ctx, args)
        log("C4: batch %.3f s vs one at a time %.3f s (%.2fx), bit-exact %s"
            % (batch["batch_s"], batch["alone_s"], batch["speedup"], batch["bit_exact_vs_alone"]))
    ctx.close()
    serve = None
    if not args.no_serve:
        serve = bench_serve(F, args)
        log("C5: server %.3g draws/s p50 %.2f s p99 %.2f s; one at a time %.3g draws/s p50 %.2f s p99 %.2f s"
            % (serve["server"]["draws_per_s"], serve["server"]["p50_s"], serve["server"]["p99_s"],
               serve["one_at_a_time"]["draws_per_s"], serve["one_at_a_time"]["p50_s"],
               serve["one_at_a_time"]["p99_s"]))
    cpu = None
    if not args.no_cpu_baseline:
        threads = min(os.cpu_count() or 1, 16)
        cpu, R_ess = cpu_baseline(w, seed, args.cpu_chains_per_thread * threads, args.cpu_draws, threads,
                                  ess.get("_moments"))
        log("cpu oracle: %.3g draws/s (%s)" % (cpu["value"], cpu["sample"]))
        cpu["checks"] = oracle_checks(ess.get("_sample"), R_ess, nuts.get("_check") if nuts else None,
                                      batch.get("_check") if batch else None, threads)
        log("oracle checks: %s" % json.dumps(cpu["checks"]))

    if ceilings and nuts:
        gr = nuts["gradient"]["roofline"]
        gr["frac_of_measured_peak"] = gr["achieved"] / (ceilings["measured"]["mfma_bf16_tflops"] / PIECE_PRODUCTS)
    ess.pop("_moments", None)
    ess.pop("_sample", None)
    if nuts:
        nuts.pop("_check", None)
    if batch:
        batch.pop("_check", None)
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
        "arithmetic": "FP32 throughout; the direction GEMM (Dp > 512) multiplies exact three-piece bf16 "
                      "splits of its FP32 operands on the bf16 matrix cores (six piece products per FP32 "
                      "product, FP32 accumulation) and matches the FP32 product to ~1e-6",
        "data": "synthetic",
        "config": {"workload": "ESS GP-logistic D=1024 (SE lengthscale 0.05, jitter 1e-5), "
                               "%d chains x %d draws, FP32; one step = one whole sampling job"
                               % (args.chains, args.draws),
                   "chains": args.chains, "draws": args.draws, "dim": 1024},
        "roofline": {"bound": "mfma", "kernel": g["kernel"], "achieved": g["tflops"],
                     "peak": PEAK_GEMM, "unit": "TFLOP/s", "frac": g["tflops"] / PEAK_GEMM,
                     "traffic": stored_traffic(), "avg_launch_us": g["avg_us"], "launches": g["launches"],
                     "flop_per_launch": g["flop_per_launch"],
                     "note": "achieved = the FP32 product's D(D+1) flop per column; the kernel runs them as "
                             "six bf16 piece products on the bf16 matrix cores, so peak = 2500 / 6 TFLOP/s "
                             "(executed bf16 rate = 6 x achieved; for scale, the FP32 MFMA peak is 157.3). "
                             "In the job, each window's GEMM overlaps the previous window's FSM kernel.",
                     "executed_bf16_tflops": PIECE_PRODUCTS * g["tflops"],
                     "isolated": {"achieved": ess["gemm_isolated"]["tflops"],
                                  "frac": ess["gemm_isolated"]["tflops"] / PEAK_GEMM,
                                  "avg_launch_us": ess["gemm_isolated"]["avg_us"]},
                     "frac_of_measured_peak": (g["tflops"] / (ceilings["measured"]["mfma_bf16_tflops"]
                                                             / PIECE_PRODUCTS)) if ceilings else None},
        "ceilings": ceilings,
        "ess": ess,
        "speedup_vs_sync_vmap": ess["sync"].get("vmap", {}).get("speedup_fsm"),
        "speedup_vs_sync_compact": ess["sync"].get("compact", {}).get("speedup_fsm"),
        "nuts": nuts,
        "nuts_c3": nuts_c3,
        "nuts_mog": mog,
        "drsym": drsym,
        "slice": slc,
        "ess_gp_hyper": gph,
        "batch": batch,
        "serve": serve,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()

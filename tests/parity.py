"""Helpers of the GPU-vs-oracle parity tests (test code; calls the oracle).

Per-draw error: ||x_gpu - x_orc||_2 / max(||x_orc||_2, 1).

A chain *parts* from the oracle at the first draw whose loop count differs
(a different number of shrinks, stages or leapfrogs) or whose error exceeds
the tolerance; draws from there on are not compared.  A parting is accepted
only as a near-tie flip: the oracle replays that draw from its own previous
state once for every decision whose margin is below
64 eps32 (1 + sum |terms|), with that one decision inverted, and one of these
replays must reproduce the GPU's draw (same loop count, error within the
tolerance).  So the margin that is tested is the margin of the decision at
which the two runs part, not the smallest margin anywhere in the draw, and a
draw that no single near-tie decision explains is a failure.
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as O

EPS32 = np.finfo(np.float32).eps


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b, axis=-1) / np.maximum(np.linalg.norm(b, axis=-1), 1.0))


def explain_parting(target, sampler, seed, chain, draw, x_prev, gpu_x, gpu_count, tol=1e-4,
                    eps=EPS32):
    """Is the GPU's draw `draw` (from a state equal to the oracle's x_prev up
    to rounding) the oracle's draw with one near-tie decision inverted?
    Returns (explained, decision index or -1, relative margin of that
    decision or of the closest decision when unexplained, number of
    near-tie decisions in the draw)."""
    x, cnt, mar, sca = O.draw_traced(target, sampler, seed, chain, draw, x_prev)
    rel = mar / (1.0 + sca)
    near = np.nonzero(rel < 64 * eps)[0]
    for k in near:
        xf, cf, _, _ = O.draw_traced(target, sampler, seed, chain, draw, x_prev, flip_at=int(k))
        if cf == int(gpu_count) and rel_err(gpu_x, xf) <= tol:
            return True, int(k), float(rel[k]), int(near.size)
    return False, -1, float(rel.min()) if rel.size else np.inf, int(near.size)


def check_chains(gpu, gpu_counts, orc, orc_counts, target, sampler, seed, chains, x_init,
                 first=100, tol=1e-4):
    """Compares GPU chains with oracle chains draw by draw.

    gpu, orc: (m, n, D) draws of the chains `chains` (stream ids); counts
    (m, n); x_init: (m, D) the oracle's initial states.  Returns a dict:
    worst (max error over compared draws), parted (chains that parted),
    bad (partings not explained by one near-tie decision), margins (relative
    margins of the explained flips), flip_frac."""
    m = gpu.shape[0]
    n = min(first, gpu.shape[1], orc.shape[1])
    worst, parted, bad, margins = 0.0, 0, [], []
    for j in range(m):
        a = gpu[j, :n].astype(np.float64)
        b = orc[j, :n]
        err = np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1.0)
        off = np.nonzero((gpu_counts[j, :n] != orc_counts[j, :n]) | (err > tol))[0]
        upto = n if off.size == 0 else int(off[0])
        if upto > 0:
            worst = max(worst, float(err[:upto].max()))
        if off.size == 0:
            continue
        parted += 1
        t = upto
        xp = orc[j, t - 1] if t > 0 else x_init[j]
        ok, k, rel, _ = explain_parting(target, sampler, seed, int(chains[j]), t, xp, a[t],
                                        gpu_counts[j, t], tol=tol)
        if ok:
            margins.append(rel)
        else:
            bad.append((int(chains[j]), t, rel))
    return dict(worst=worst, parted=parted, bad=bad, margins=margins,
                flip_frac=parted / max(m, 1), compared=n)


def summary(name, r):
    return ("%s: max rel err %.3g over %d draws; chains parted %d (%.2f%%), all near-tie flips: %s%s"
            % (name, r["worst"], r["compared"], r["parted"], 100 * r["flip_frac"], not r["bad"],
               "" if not r["bad"] else " unexplained %s" % r["bad"][:4]))


# ------------------------------------------------ jobs of a batch or server mix
def oracle_job(spec):
    """The oracle's (target, sampler, chain seed, initial state of chain j) for
    a tagged job spec of the batch / serving tests:
      ("ess", dim, chains, draws, data seed, chain seed)       GP-logistic ESS
      ("dr", "funnel"|"gauss", dim, chains, draws, seed)       3-stage DR
      ("nuts", rows, dim, chains, draws, data seed, chain seed, step)
    The inputs are regenerated from the seeded generators; the Gaussian
    target's precisions are torch's linspace (what the GPU job was given)."""
    from paper_2503_17405_amd import inputs
    kind = spec[0]
    if kind == "ess":
        _, D, m, n, ds, cs = spec
        w = inputs.gp_logistic(dim=D, lengthscale=0.05, jitter=1e-5, seed=ds)
        return O.gp_target(w["y"]), O.ess_sampler(w["L"]), cs, lambda j: O.ess_init(w["L"], cs, j)
    if kind == "dr":
        _, tk, D, m, n, seed = spec
        if tk == "funnel":
            return O.funnel_target(D), O.dr_sampler(), seed, lambda j: O.funnel_init(D, seed, j)
        import torch
        prec = torch.linspace(0.5, 2.0, D, device="cuda").cpu().numpy().astype(np.float64)
        return O.gauss_target(prec), O.dr_sampler(), seed, lambda j: O.normal_init(D, seed, j)
    _, N, D, m, n, ds, cs, eps = spec
    w = inputs.logreg(n_data=N, dim=D, seed=ds)
    x0 = inputs.logreg_laplace(w["X"], w["y"], m, seed=ds + 7)["x0"]
    x0 = x0.astype(np.float32).astype(np.float64)  # the GPU job starts from the FP32 values
    return (O.logreg_target(w["X"].astype(np.float64), w["y"]), O.nuts_sampler(eps), cs,
            lambda j: x0[j])


def check_job(spec, S, C, chains, first=100, tol=1e-4):
    """Oracle parity of chains `chains` of one job of a mix; S, C are the
    job's full (m, n, D) draws and (m, n) loop counts from the GPU."""
    tg, sp, seed, init = oracle_job(spec)
    chains = list(chains)
    x_init = np.array([init(j) for j in chains])
    n = min(first, S.shape[1])
    R, RC, _ = O.run_chains(tg, sp, seed, chains, n, x0=x_init)
    return check_chains(S[chains, :n], C[chains, :n], R, RC, tg, sp, seed, chains, x_init,
                        first=n, tol=tol)


def sample_chains(m, k, seed):
    """First, last and k-2 random chain indices of an m-chain job."""
    rest = np.random.default_rng(seed).choice(np.arange(1, max(m - 1, 1)), size=max(0, min(k - 2, m - 2)),
                                              replace=False) if m > 2 else []
    return sorted(set([0, m - 1] + [int(i) for i in rest]))

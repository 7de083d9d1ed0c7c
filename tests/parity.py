"""Helpers of the GPU-vs-oracle parity tests (test code; calls the oracle).

Per-draw error: ||x_gpu - x_orc||_2 / max(||x_orc||_2, 1).  A chain "flips"
at the first draw whose loop count differs from the oracle's (a different
number of shrinks, stages or leapfrogs); draws from the flip on are not
compared.  A flip is a near-tie when the oracle's decision margin at the
evaluation where the two runs part is below 64 eps32 (1 + sum |terms|).
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as O

EPS32 = np.finfo(np.float32).eps


def compare_draws(gpu, orc, gpu_counts, orc_counts, first=100, jump=1e-3):
    """Returns (max error before flips, flip draw per chain or -1).

    A chain flips at the first draw whose loop count differs from the
    oracle's, or whose error jumps above `jump` -- a branch taken differently
    without changing the loop count (a NUTS leaf or merge pick) moves the draw
    by O(1), far above rounding drift (which the 1e-4 bound checks)."""
    m = gpu.shape[0]
    n = min(first, gpu.shape[1])
    flips = np.full(m, -1)
    worst = 0.0
    for j in range(m):
        a = gpu[j, :n].astype(np.float64)
        b = orc[j, :n]
        err = np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1.0)
        bad = np.nonzero((gpu_counts[j, :n] != orc_counts[j, :n]) | (err > jump))[0]
        upto = n if bad.size == 0 else bad[0]
        if bad.size:
            flips[j] = bad[0]
        if upto > 0:
            worst = max(worst, float(err[:upto].max()))
    return worst, flips


def ess_flip_margin(target, L, seed, chain, draw, x_prev, gpu_count, orc_count, noise_sd=None):
    """Decision margin of the oracle at the evaluation where a GPU ESS chain
    with a different loop count parted from it, and the magnitude scale."""
    D = L.shape[0]
    lx = O.gp_loglik(target, x_prev)
    nu = L @ O.normals(seed, chain, draw, O.ROLE_NU, 0, D)
    logy = lx + np.log(O.uniform(seed, chain, draw, O.ROLE_THRESH, 0))
    theta = 2 * np.pi * O.uniform(seed, chain, draw, O.ROLE_ANGLE, 0)
    tmin, tmax = theta - 2 * np.pi, theta
    k_at = min(gpu_count, orc_count)  # the evaluation where the decisions differ
    for ev in range(1, k_at + 1):
        xp = x_prev * np.cos(theta) + nu * np.sin(theta)
        lp = O.gp_loglik(target, xp)
        if ev == k_at:
            y = target.y
            if noise_sd is None:
                terms = np.sum(np.abs(y * xp)) + np.sum(np.logaddexp(0, xp))
            else:
                terms = np.sum((y - xp) ** 2) / (2 * noise_sd ** 2)
            return abs(lp - logy), terms + abs(logy)
        if theta < 0:
            tmin = theta
        else:
            tmax = theta
        theta = tmin + (tmax - tmin) * O.uniform(seed, chain, draw, O.ROLE_ANGLE, ev)
    return np.inf, 0.0


def is_near_tie(margin, terms, eps=EPS32):
    return margin < 64 * eps * (1.0 + terms)


def _lq(a, b, sc):
    r = b - a
    return -float(r @ r) / (2.0 * sc * sc)


def dr_flip_near_tie(target, scales, n_stages, seed, chain, draw, x_prev, eps=EPS32):
    """Smallest relative margin of the oracle's DR acceptance decisions in one
    draw from x_prev (stages walked as the oracle walks them)."""
    D = target.dim
    lx = O.logpdf(target, x_prev)
    ys, ls, rel = [], [], []
    for s in range(n_stages):
        y = x_prev + scales[s] * O.normals(seed, chain, draw, O.ROLE_PROP, s, D)
        ly = O.logpdf(target, y)
        ys.append(y)
        ls.append(ly)
        if s == 0:
            la, qs = O.dr_log_alpha1(lx, ly), []
        elif s == 1:
            qs = [_lq(x_prev, ys[0], scales[0]), _lq(y, ys[0], scales[0])]
            la = O.dr_log_alpha2(lx, ls[0], ly, *qs)
        else:
            qs = [_lq(x_prev, ys[0], scales[0]), _lq(ys[1], ys[0], scales[0]), _lq(x_prev, ys[1], scales[1]),
                  _lq(y, ys[1], scales[0]), _lq(y, ys[0], scales[1]), _lq(ys[0], ys[1], scales[0])]
            la = O.dr_log_alpha3(lx, ls[0], ls[1], ly, qs)
        lu = np.log(O.uniform(seed, chain, draw, O.ROLE_ACC, s))
        scale = abs(lx) + sum(abs(v) for v in ls) + sum(abs(q) for q in qs)
        if np.isfinite(la):
            rel.append(abs(lu - la) / (1.0 + scale))
        if lu < la:
            break
    r = min(rel) if rel else np.inf
    return r < 64 * eps, r


def nuts_flip_near_tie(target, eps_step, max_depth, seed, chain, draw, x_prev, eps=EPS32):
    """Smallest relative decision margin of the oracle's NUTS draw from x_prev,
    and whether it is a near-tie."""
    mar, sca = O.nuts_decisions(target, eps_step, max_depth, seed, chain, draw, x_prev)
    rel = mar / (1.0 + sca)
    r = float(rel.min()) if rel.size else np.inf
    return r < 64 * eps, r

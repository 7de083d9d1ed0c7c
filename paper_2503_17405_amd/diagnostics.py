"""Host-side statistics for the benchmark report (not on the sampling path).

* ``r_of_m``: the paper's efficiency bound R(m) = E[max_{j<=m} N_j] / E[N]
  (Sec. 4.2) for i.i.d. loop counts N with the empirical distribution of a
  job's per-draw counts.  E[max] is taken as the sum over the distinct count
  values x_i (ascending) of x_i (F(x_i)^m - F(x_{i-1})^m).
* ``ess``: multi-chain effective sample size of each coordinate, Geyer's
  initial monotone sequence estimator (Geyer 1992, Statist. Sci. 7) on the
  autocorrelation pooled over chains with the between/within-chain variance
  of Gelman et al. (BDA3, Sec. 11.5); chains x draws x coordinates at once.
* ``moments``: per-coordinate mean and variance with their Monte Carlo
  standard errors (sd / sqrt(ESS), the variance's from the ESS of the
  squared deviations), and ``z_scores``: the difference of two such
  estimates in units of their combined standard error.
"""
from __future__ import annotations

import numpy as np


def r_of_m(counts, m):
    """R(m) from the empirical distribution of loop counts (any shape)."""
    c = np.asarray(counts, dtype=np.float64).ravel()
    if c.size == 0 or c.max() <= 0:
        return 1.0
    vals, cnt = np.unique(c, return_counts=True)
    cdf = np.cumsum(cnt) / c.size
    pm = cdf ** m
    prev = np.concatenate(([0.0], pm[:-1]))
    e_max = float(np.sum(vals * (pm - prev)))
    return e_max / float(c.mean())


def ess(draws):
    """ESS per coordinate; draws: (chains, n) or (chains, n, k).  Returns (k,)."""
    x = np.asarray(draws, dtype=np.float64)
    if x.ndim == 2:
        x = x[:, :, None]
    m, n, k = x.shape
    if n < 4:
        return np.full(k, float(m * n))
    dev = x - x.mean(axis=1, keepdims=True)
    spec = np.fft.rfft(dev, n=2 * n, axis=1)
    acov = np.fft.irfft(spec * np.conj(spec), n=2 * n, axis=1)[:, :n, :] / n  # (m, n, k), biased
    within = (acov[:, 0, :] * n / (n - 1.0)).mean(axis=0)  # W
    between = n * x.mean(axis=1).var(axis=0, ddof=1) if m > 1 else np.zeros(k)  # B
    var_plus = (n - 1.0) / n * within + between / n
    out = np.full(k, float(m * n))
    for j in range(k):
        if var_plus[j] <= 0:
            continue
        rho = 1.0 - (within[j] - acov[:, :, j].mean(axis=0)) / var_plus[j]
        rho[0] = 1.0
        half = n // 2
        pairs = rho[0:2 * half:2] + rho[1:2 * half:2]
        nonpos = np.nonzero(pairs <= 0.0)[0]
        pairs = pairs[: nonpos[0]] if nonpos.size else pairs
        if pairs.size == 0:
            continue
        tau = 2.0 * np.minimum.accumulate(pairs).sum() - 1.0
        tau = max(tau, 1.0 / np.log10(m * n + 10.0))
        out[j] = m * n / tau
    return out


def moments(draws, mcse_chains=1024):
    """Mean, variance and their MCSEs per coordinate of draws (chains, n, k);
    the ESS is estimated on the first mcse_chains chains and scaled to all."""
    x = np.asarray(draws, dtype=np.float64)
    if x.ndim == 2:
        x = x[:, :, None]
    m = x.shape[0]
    c = min(m, mcse_chains)
    mean = x.mean(axis=(0, 1))
    var = x.var(axis=(0, 1))
    sq = (x - mean) ** 2
    e1 = ess(x[:c]) * (m / c)
    e2 = ess(sq[:c]) * (m / c)
    return dict(mean=mean, var=var, mean_mcse=np.sqrt(var / e1), var_mcse=sq.std(axis=(0, 1)) / np.sqrt(e2))


def z_scores(a, b):
    """Differences of two moments() results in units of their combined MCSE."""
    zm = (a["mean"] - b["mean"]) / np.sqrt(a["mean_mcse"] ** 2 + b["mean_mcse"] ** 2)
    zv = (a["var"] - b["var"]) / np.sqrt(a["var_mcse"] ** 2 + b["var_mcse"] ** 2)
    return dict(mean_z=[float(v) for v in zm], var_z=[float(v) for v in zv])

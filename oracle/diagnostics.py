"""Sampler diagnostics used by the tests and the benchmark report.

TEST INFRASTRUCTURE (same status as the rest of ``oracle/``).

* ``ess``: multi-chain effective sample size with Geyer's initial monotone
  sequence estimator (Geyer 1992), between/within-chain variance as in
  Gelman et al., BDA3 Sec. 11.5.
* ``mcse_mean``: Monte Carlo standard error of a posterior mean.
* ``r_hat_m``: the efficiency bound R(m) = E max_{j<=m} N_j / E N_1 of the
  paper (Sec. 4.2), estimated from an empirical loop-count distribution
  assuming i.i.d. chains: E max = sum_{k>=1} (1 - F(k-1)^m).
"""
from __future__ import annotations

import numpy as np


def _autocov(x):
    """Biased autocovariance of a 1-D series via FFT."""
    n = x.size
    x = x - x.mean()
    f = np.fft.rfft(x, 2 * n)
    ac = np.fft.irfft(f * np.conj(f))[:n] / n
    return ac


def ess(chains):
    """Effective sample size of a scalar quantity; chains: (m, n)."""
    chains = np.asarray(chains, dtype=np.float64)
    if chains.ndim == 1:
        chains = chains[None]
    m, n = chains.shape
    if n < 4:
        return float(m * n)
    acov = np.stack([_autocov(c) for c in chains])  # (m, n)
    chain_mean = chains.mean(axis=1)
    chain_var = acov[:, 0] * n / (n - 1.0)
    W = chain_var.mean()
    B = n * chain_mean.var(ddof=1) if m > 1 else 0.0
    var_plus = (n - 1.0) / n * W + B / n
    if var_plus <= 0:
        return float(m * n)
    rho = 1.0 - (W - acov.mean(axis=0)) / var_plus
    rho[0] = 1.0
    # Geyer: sums of adjacent pairs, truncated at the first non-positive
    # pair, then made monotone non-increasing.
    npairs = n // 2
    P = rho[0:2 * npairs:2] + rho[1:2 * npairs:2]
    keep = []
    for k in range(npairs):
        if P[k] <= 0:
            break
        keep.append(P[k])
    if not keep:
        return float(m * n)
    P = np.minimum.accumulate(np.array(keep))
    tau = -1.0 + 2.0 * P.sum()
    tau = max(tau, 1.0 / np.log10(m * n + 10))
    return float(m * n / tau)


def mcse_mean(chains):
    chains = np.asarray(chains, dtype=np.float64)
    return float(chains.std(ddof=1) / np.sqrt(ess(chains)))


def mcse_var(chains):
    """MCSE of the variance estimate, from the ESS of (x - mean)^2."""
    chains = np.asarray(chains, dtype=np.float64)
    sq = (chains - chains.mean()) ** 2
    return float(sq.std(ddof=1) / np.sqrt(ess(sq)))


def r_hat_m(counts, m):
    """R(m) from an empirical distribution of per-draw loop counts N >= 0."""
    counts = np.asarray(counts).ravel()
    mean = counts.mean()
    if mean <= 0:
        return 1.0
    kmax = int(counts.max())
    hist = np.bincount(counts.astype(np.int64), minlength=kmax + 1).astype(np.float64)
    F = np.cumsum(hist) / counts.size  # F[k] = P(N <= k)
    emax = np.sum(1.0 - F[:kmax] ** m)  # sum_{k=1}^{kmax} (1 - F(k-1)^m)
    return float(emax / mean)


def e_max(counts, m):
    counts = np.asarray(counts).ravel()
    kmax = int(counts.max())
    hist = np.bincount(counts.astype(np.int64), minlength=kmax + 1).astype(np.float64)
    F = np.cumsum(hist) / counts.size
    return float(np.sum(1.0 - F[:kmax] ** m))

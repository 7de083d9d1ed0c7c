"""Seeded synthetic workloads shared by the HIP path's tests/benchmark and the oracle.

This module draws problem data only (GP inputs, prior covariance and its
Cholesky factor, labels, design matrices, initial states); it contains none
of the samplers' arithmetic.  Every generator is a pure function of its seed
(numpy PCG64), so both sides read identical arrays.

Workload recipes (the sizes the benchmark and tests use):
  * ``gp_gauss``: D inputs uniform on [0, 1], squared-exponential prior
    covariance var * exp(-(a-b)^2 / (2 l^2)) + jitter * I, latent f drawn from
    the prior, observations y = f + noise_sd * eps.
  * ``gp_logistic``: as above with Bernoulli labels y_i ~ Bern(sigmoid(f_i)),
    f from a seeded prior draw.
  * ``logreg``: X (N x D) i.i.d. N(0, 1) in FP32, beta_true ~ N(0, I),
    y ~ Bern(sigmoid(X beta_true)); optional Laplace-approximation starting
    points beta0 ~ N(beta_MAP, H^-1), H = X^T W X + I.
  * ``mog``: the correlated mixture of Gaussians of the NUTS experiment:
    D-dimensional, one covariance Sigma = (1 - rho) I + rho 1 1^T shared by K
    equally weighted components whose means sit at c 1 for c in ``modes``
    (along the principal direction 1 / sqrt(D)); the precision matrix
    Sigma^-1, the means and the log weights are rounded to FP32 so that every
    side reads the same numbers; starting points are exact draws from the
    mixture.
  * ``gp_hyper``: GP regression data standing in for the paper's 6-feature
    real-estate regression: n inputs uniform on [0, 1]^6, outputs
    f(x) + 0.3 eps with f drawn from a GP with tau = 1, lambda = 1.5, then
    standardised; starting hyperparameters drawn from the N(0, I) prior.
"""
from __future__ import annotations

import numpy as np


def _rng(seed):
    return np.random.Generator(np.random.PCG64(int(seed)))


def se_cov(points, lengthscale, variance=1.0, jitter=0.0):
    d = points[:, None] - points[None, :]
    K = variance * np.exp(-(d * d) / (2.0 * lengthscale * lengthscale))
    K[np.diag_indices_from(K)] += jitter
    return K


def _sigmoid(a):
    return 0.5 * (1.0 + np.tanh(0.5 * a))


def gp_gauss(dim=16, lengthscale=0.2, variance=1.0, jitter=1e-6, noise_sd=0.1, seed=1001):
    """GP prior + Gaussian likelihood (the closed-form-posterior workload)."""
    g = _rng(seed)
    pts = g.uniform(0.0, 1.0, size=dim)
    K = se_cov(pts, lengthscale, variance, jitter)
    L = np.linalg.cholesky(K)
    f = L @ g.standard_normal(dim)
    y = f + noise_sd * g.standard_normal(dim)
    return dict(points=pts, K=K, L=L, f=f, y=y, noise_sd=noise_sd)


def gp_logistic(dim=1024, lengthscale=0.05, variance=1.0, jitter=1e-5, seed=2001):
    """GP prior + Bernoulli-logistic likelihood, labels from a seeded prior draw."""
    g = _rng(seed)
    pts = g.uniform(0.0, 1.0, size=dim)
    K = se_cov(pts, lengthscale, variance, jitter)
    L = np.linalg.cholesky(K)
    f = L @ g.standard_normal(dim)
    y = (g.uniform(size=dim) < _sigmoid(f)).astype(np.float64)
    return dict(points=pts, K=K, L=L, f=f, y=y)


def logreg(n_data=10000, dim=100, seed=3001):
    """Bayesian logistic regression data: X FP32 N(0,1), prior N(0, I)."""
    g = _rng(seed)
    X = g.standard_normal((n_data, dim)).astype(np.float32)
    beta = g.standard_normal(dim)
    y = (g.uniform(size=n_data) < _sigmoid(X.astype(np.float64) @ beta)).astype(np.float64)
    return dict(X=X, y=y, beta_true=beta)


def logreg_laplace(X, y, n_chains, seed, iters=50):
    """Starting points beta0 ~ N(beta_MAP, H^-1) from an FP64 Newton fit."""
    X = np.asarray(X, dtype=np.float64)
    D = X.shape[1]
    b = np.zeros(D)
    for _ in range(iters):
        p = _sigmoid(X @ b)
        grad = X.T @ (y - p) - b
        H = (X * (p * (1 - p))[:, None]).T @ X + np.eye(D)
        step = np.linalg.solve(H, grad)
        b = b + step
        if np.max(np.abs(step)) < 1e-12:
            break
    p = _sigmoid(X @ b)
    H = (X * (p * (1 - p))[:, None]).T @ X + np.eye(D)
    Lh = np.linalg.cholesky(H)
    g = _rng(seed)
    Z = g.standard_normal((n_chains, D))
    # beta0 = b + H^{-1/2} z with H = Lh Lh^T  ->  solve Lh^T w = z
    W = np.linalg.solve(Lh.T, Z.T).T
    return dict(map=b, hessian=H, x0=np.ascontiguousarray(b[None, :] + W))


def ess_uneven_targets(n_targets=32, dmin=64, dmax=1024, mmin=256, mmax=2048, nmin=200,
                       nmax=2000, seed=4003):
    """A mix of GP-logistic ESS targets of uneven dimension, chain count and budget."""
    g = _rng(seed)
    out = []
    for i in range(n_targets):
        D = int(g.integers(dmin, dmax + 1))
        m = int(g.integers(mmin, mmax + 1))
        n = int(g.integers(nmin, nmax + 1))
        out.append(dict(dim=D, n_chains=m, n_draws=n, data_seed=int(g.integers(1 << 31)),
                        chain_seed=int(g.integers(1 << 62))))
    return out


def mog(dim=100, rho=0.99, modes=(-10.0, 0.0, 10.0), n_chains=0, seed=6001):
    """Correlated mixture of Gaussians; x0: n_chains exact draws (or None)."""
    D, K = int(dim), len(modes)
    cov = (1.0 - rho) * np.eye(D) + rho * np.ones((D, D))
    prec = np.linalg.inv(cov)
    prec = 0.5 * (prec + prec.T)
    prec32 = prec.astype(np.float32)
    means = np.array([[c] * D for c in modes], dtype=np.float32)
    logw = np.full(K, np.log(1.0 / K), dtype=np.float32)
    # the covariance the rounded precision defines (both sides sample that target)
    cov_r = np.linalg.inv(prec32.astype(np.float64))
    cov_r = 0.5 * (cov_r + cov_r.T)
    x0 = None
    if n_chains > 0:
        g = _rng(seed)
        comp = g.integers(0, K, size=n_chains)
        Lc = np.linalg.cholesky(cov_r)
        Z = g.standard_normal((n_chains, D))
        x0 = np.ascontiguousarray(means.astype(np.float64)[comp] + Z @ Lc.T)
    return dict(prec=prec32, means=means, log_weights=logw, cov=cov_r, x0=x0, rho=rho, modes=tuple(modes))


def gp_hyper(n=100, p=6, n_chains=0, seed=9001):
    """GP-regression data for the hyperparameter posterior; x0: prior draws."""
    g = _rng(seed)
    X = g.uniform(0.0, 1.0, size=(n, p))
    d2 = ((X[:, None, :] - X[None, :, :]) ** 2).sum(axis=2)
    K = np.exp(-(1.5 ** 2) * d2) + 1e-8 * np.eye(n)
    f = np.linalg.cholesky(K) @ g.standard_normal(n)
    y = f + 0.3 * g.standard_normal(n)
    if n > 1:
        y = (y - y.mean()) / y.std()
    x0 = g.standard_normal((n_chains, 3)) if n_chains > 0 else None
    return dict(X=X, y=y, x0=x0, jitter=1e-6)

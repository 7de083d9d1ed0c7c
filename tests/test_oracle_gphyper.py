"""Pins of the oracle's GP-hyperparameter target (Sec. 7.2): the marginal
likelihood of theta = (tau, lambda, sigma) under y ~ N(0, tau^2 K_lambda +
(sigma^2 + jitter) I), sampled by elliptical slice sampling with the N(0, I)
prior.

* log-likelihood against scipy's multivariate normal log-density (plus the
  dropped n/2 log 2 pi), at random hyperparameters and data sizes;
* a singular covariance gives -inf (the Cholesky factor does not exist);
* one observation: the likelihood does not involve lambda, so lambda's
  posterior is the N(0, 1) prior, and tau^2 + sigma^2 has a posterior mean
  computed here by quadrature on a grid; ESS matches both within 3 MCSE.
"""
import numpy as np
import pytest
from scipy.stats import multivariate_normal

from oracle import diagnostics as OD
from oracle import oracle as O
from paper_2503_17405_amd import inputs


def _cov(X, th, jitter):
    d2 = ((X[:, None, :] - X[None, :, :]) ** 2).sum(axis=2)
    return th[0] ** 2 * np.exp(-th[1] ** 2 * d2) + (th[2] ** 2 + jitter) * np.eye(X.shape[0])


@pytest.mark.parametrize("n,seed", [(1, 1), (5, 2), (25, 3), (100, 4)])
def test_loglik_matches_scipy(n, seed):
    w = inputs.gp_hyper(n=n, seed=seed)
    tg = O.gp_hyper_target(w["X"], w["y"], w["jitter"])
    g = np.random.default_rng(seed)
    for _ in range(10):
        th = g.standard_normal(3)
        want = multivariate_normal.logpdf(w["y"], np.zeros(n), _cov(w["X"], th, w["jitter"])) \
            + 0.5 * n * np.log(2 * np.pi)
        got = O.gp_hyper_loglik(tg, th)
        assert abs(got - want) <= 1e-8 * (1 + abs(want)), (th, got, want)


def test_singular_covariance_is_minus_infinity():
    X = np.zeros((4, 6))  # four identical inputs: K = 1 1^T
    tg = O.gp_hyper_target(X, np.arange(4.0), jitter=0.0)
    assert O.gp_hyper_loglik(tg, [1.3, 0.7, 0.0]) == -np.inf
    assert np.isfinite(O.gp_hyper_loglik(tg, [1.3, 0.7, 0.2]))


def test_ess_one_observation_posterior():
    y = 1.7
    tg = O.gp_hyper_target(np.zeros((1, 6)), [y], jitter=1e-6)
    draws, counts, guards = O.run_chains(tg, O.ess_sampler(np.eye(3)), 21, range(32), 3000)
    b = draws[:, 300:, :]
    lam = b[:, :, 1]
    assert abs(lam.mean()) < 3 * OD.mcse_mean(lam)
    assert abs(lam.var() - 1.0) < 3 * OD.mcse_var(lam)
    # E[tau^2 + sigma^2] by quadrature over (tau, sigma) with the N(0, 1) priors
    t = np.linspace(-7, 7, 1401)
    T, S = np.meshgrid(t, t, indexing="ij")
    v = T ** 2 + S ** 2 + 1e-6
    w = np.exp(-0.5 * (T ** 2 + S ** 2)) * np.exp(-0.5 * y * y / v) / np.sqrt(v)
    want = (v * w).sum() / w.sum()
    s = b[:, :, 0] ** 2 + b[:, :, 2] ** 2
    assert abs(s.mean() - want) < 3 * OD.mcse_mean(s), (s.mean(), want)
    assert np.sum(guards) == 0

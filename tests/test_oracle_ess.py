"""Pins of the oracle's elliptical slice sampler (Appendix, Alg. "Transition
kernel for elliptical slice sampler"; FSM of Fig. "Finite state machines ...")."""
import numpy as np
import pytest

from oracle import diagnostics as Dg
from oracle import oracle as O
from paper_2503_17405_amd import inputs

ESS_EDGES = {(1, 2), (1, 3), (2, 2), (2, 3), (3, 1)}


def _closed_form(w):
    K, y, s2 = w["K"], w["y"], w["noise_sd"] ** 2
    A = np.linalg.solve(K + s2 * np.eye(len(y)), np.eye(len(y)))
    mu = K @ A @ y
    S = K - K @ A @ K
    return mu, S


@pytest.fixture(scope="module")
def c1_run():
    # The 16-dimensional Gaussian-Gaussian workload, 64 chains, fixed seed.
    # 4000 draws per chain: at 1000 draws the multi-chain ESS of a coordinate
    # is only ~400 and the MCSE of a variance estimate is itself too noisy
    # for a 3-MCSE bound over 32 statistics.
    w = inputs.gp_gauss(dim=16, lengthscale=0.2, jitter=1e-6, noise_sd=0.1, seed=1001)
    tg = O.gp_target(w["y"], noise_sd=w["noise_sd"])
    sp = O.ess_sampler(w["L"])
    draws, counts, guards = O.run_chains(tg, sp, seed=1002, chains=range(64), n=4000)
    return w, draws, counts, guards


def test_ess_gaussian_posterior_closed_form(c1_run):
    w, draws, counts, guards = c1_run
    assert guards == 0
    mu, S = _closed_form(w)
    burn = draws[:, 400:, :]
    for d in range(16):
        x = burn[:, :, d]
        assert abs(x.mean() - mu[d]) < 3 * Dg.mcse_mean(x), d
        assert abs(x.var() - S[d, d]) < 3 * Dg.mcse_var(x), d


def test_ess_mahalanobis_chi2(c1_run):
    # sum of squared whitened posterior residuals ~ chi^2_16 on average
    w, draws, _, _ = c1_run
    mu, S = _closed_form(w)
    Ls = np.linalg.cholesky(S)
    r = np.linalg.solve(Ls, (draws[:, 400:, :] - mu).reshape(-1, 16).T)
    q = (r * r).sum(axis=0).reshape(64, -1)
    assert abs(q.mean() - 16) < 3 * Dg.mcse_mean(q)


def test_ess_flat_likelihood_zero_shrinks():
    # noise_sd = inf gives log L = 0: every first proposal beats log y = log u < 0,
    # so each draw uses one evaluation and the chain targets the prior itself.
    w = inputs.gp_gauss(dim=8, lengthscale=0.3, seed=77)
    tg = O.gp_target(np.zeros(8), noise_sd=np.inf)
    sp = O.ess_sampler(w["L"])
    draws, counts, _ = O.run_chains(tg, sp, seed=5, chains=range(32), n=400)
    assert np.all(counts == 1)
    K = w["K"]
    for d in range(8):
        x = draws[:, :, d]
        assert abs(x.mean()) < 3 * Dg.mcse_mean(x)
        assert abs(x.var() - K[d, d]) < 3 * Dg.mcse_var(x)


@pytest.mark.parametrize("kind", ["gauss", "logistic"])
def test_ess_fsm_equals_sample(kind):
    if kind == "gauss":
        w = inputs.gp_gauss(dim=16, seed=1001)
        tg = O.gp_target(w["y"], noise_sd=0.1)
    else:
        w = inputs.gp_logistic(dim=64, lengthscale=0.1, seed=9)
        tg = O.gp_target(w["y"])
    sp = O.ess_sampler(w["L"])
    for chain in range(4):
        a = O.run_chain(tg, sp, 42, chain, 200)
        b = O.run_chain(tg, sp, 42, chain, 200, use_fsm=True, want_edges=True)
        assert np.array_equal(a["draws"], b["draws"])
        assert np.array_equal(a["counts"], b["counts"])
        E = b["edges"]
        seen = {(i, j) for i in range(4) for j in range(4) if E[i, j] > 0}
        assert seen <= ESS_EDGES
        assert (1, 2) in seen and (2, 2) in seen and (2, 3) in seen and (3, 1) in seen
        # every FSM step evaluates once in INIT/SHRINK, plus one DONE step per draw
        assert b["steps"] == a["counts"].sum() + 200


def test_ess_sample_respects_threshold():
    # every accepted state beats the slice threshold computed from its predecessor
    w = inputs.gp_logistic(dim=32, lengthscale=0.1, seed=3)
    tg = O.gp_target(w["y"])
    x = O.ess_init(w["L"], 8, 0)
    lx = O.gp_loglik(tg, x)
    for t in range(50):
        u = O.uniform(8, 0, t, O.ROLE_THRESH)
        r = O.run_chain(tg, O.ess_sampler(w["L"]), 8, 0, t + 1)
        xn = r["draws"][t]
        assert O.gp_loglik(tg, xn) > lx + np.log(u)
        x, lx = xn, O.gp_loglik(tg, xn)


def test_ess_default_init_is_prior_draw():
    w = inputs.gp_gauss(dim=6, seed=4)
    z = O.normals(3, 7, 0, O.ROLE_INIT, 0, 6)
    assert np.allclose(O.ess_init(w["L"], 3, 7), w["L"] @ z, rtol=1e-14, atol=1e-14)

"""Pins of the oracle's NUTS (Sec. 7.3, iterative two-nested-loop form; FSM
of Fig. "Finite state machines ...", HMC-NUTS panel)."""
import numpy as np
import pytest

from oracle import diagnostics as Dg
from oracle import oracle as O
from paper_2503_17405_amd import inputs

NUTS_EDGES = {(1, 2), (2, 3), (3, 3), (3, 4), (4, 2), (4, 5), (1, 5), (5, 1)}


def _seq_dot(a, b):
    s = 0.0
    for u, v in zip(a, b):
        s += u * v
    return s


@pytest.fixture(scope="module")
def small_logreg():
    d = inputs.logreg(n_data=500, dim=5, seed=17)
    return O.logreg_target(d["X"].astype(np.float64), d["y"]), d


def test_potential_gradient_matches_finite_differences(small_logreg):
    tg, _ = small_logreg
    for tgt in [tg, O.funnel_target(10), O.gauss_target(np.array([1.0, 3.0, 0.1]))]:
        th = np.random.default_rng(1).standard_normal(tgt.dim) * 0.5
        U, g = O.potential(tgt, th, grad=True)
        for d in range(tgt.dim):
            h = 1e-6
            e = np.zeros(tgt.dim)
            e[d] = h
            fd = (O.potential(tgt, th + e) - O.potential(tgt, th - e)) / (2 * h)
            assert fd == pytest.approx(g[d], rel=1e-6, abs=1e-6)


@pytest.mark.parametrize("L", [1, 8, 64])
def test_leapfrog_reversibility(small_logreg, L):
    tg, _ = small_logreg
    g0 = np.random.default_rng(L)
    th0 = g0.standard_normal(5) * 0.1
    p0 = g0.standard_normal(5)
    _, grad0 = O.potential(tg, th0, grad=True)
    th, p, g = th0, p0, grad0
    for _ in range(L):
        th, p, g, _ = O.leapfrog(tg, 0.01, th, p, g)
    p = -p
    for _ in range(L):
        th, p, g, _ = O.leapfrog(tg, 0.01, th, p, g)
    assert np.max(np.abs(th - th0)) <= 1e-12 * L
    assert np.max(np.abs(-p - p0)) <= 1e-12 * L * 10


def test_leapfrog_energy_closed_form():
    # Gaussian of precision w^2 per direction: leapfrog conserves
    # p^2 + w^2 (1 - eps^2 w^2 / 4) q^2, so H_t - H_0 = (eps^2 w^4 / 8)(q_t^2 - q_0^2).
    prec = np.array([0.5, 2.0, 9.0])
    tg = O.gauss_target(prec)
    eps = 0.3
    th = np.array([1.0, -0.5, 0.2])
    p = np.array([0.3, 1.0, -2.0])
    U0, g = O.potential(tg, th, grad=True)
    H0 = U0 + 0.5 * p @ p
    q0 = th.copy()
    for _ in range(50):
        th, p, g, U = O.leapfrog(tg, eps, th, p, g)
        H = U + 0.5 * p @ p
        pred = np.sum(eps ** 2 * prec ** 2 / 8 * (th ** 2 - q0 ** 2))
        assert H - H0 == pytest.approx(pred, rel=1e-11, abs=1e-13)


def test_nuts_depth_one_is_one_step_hmc():
    tg = O.gauss_target(np.array([1.0, 2.0, 0.5, 3.0]))
    seed, chain, eps = 9, 2, 0.7
    th = O.normal_init(4, seed, chain)
    U, g = O.potential(tg, th, grad=True)
    r = O.run_chain(tg, O.nuts_sampler(eps, max_depth=1), seed, chain, 200)
    acc = 0
    for t in range(200):
        p = O.normals(seed, chain, t, O.ROLE_MOM, 0, 4)
        v = 1 if O.uniform(seed, chain, t, O.ROLE_DIR, 0) < 0.5 else -1
        H0 = U + 0.5 * _seq_dot(p, p)
        th1, p1, g1, U1 = O.leapfrog(tg, v * eps, th, p, g)
        H1 = U1 + 0.5 * _seq_dot(p1, p1)
        if np.log(O.uniform(seed, chain, t, O.ROLE_MERGE, 0)) < H0 - H1:
            th, U, g = th1, U1, g1
            acc += 1
        assert np.array_equal(r["draws"][t], th)
    assert np.all(r["counts"] == 1)
    assert 20 < acc < 200


def _brute_first_turn(moms):
    n, D = moms.shape
    for leaf in range(n):
        k = 1
        while (leaf + 1) % (1 << k) == 0 and (1 << k) <= n:
            s = leaf + 1 - (1 << k)
            rho = moms[s:leaf + 1].sum(axis=0)
            if moms[s] @ rho <= 0 or moms[leaf] @ rho <= 0:
                return leaf
            k += 1
    return n


def test_nuts_uturn_checkpoints_brute_force():
    g = np.random.default_rng(3)
    hits = 0
    for trial in range(300):
        j = int(g.integers(1, 7))
        n = 1 << j
        w = g.uniform(0.05, 1.2)
        ang = w * np.arange(n) + g.uniform(0, 6.3)
        moms = np.stack([np.cos(ang), np.sin(ang), 0.3 * g.standard_normal(n)], axis=1)
        got = O.nuts_subtree_first_turn(moms)
        assert got == _brute_first_turn(moms), (trial, j)
        hits += got < n
    assert 30 < hits < 290


def test_nuts_standard_gaussian_moments():
    D = 10
    tg = O.gauss_target(np.ones(D))
    sp = O.nuts_sampler(0.4, max_depth=10)
    draws, counts, _ = O.run_chains(tg, sp, seed=21, chains=range(16), n=1500)
    burn = draws[:, 200:, :]
    for d in range(D):
        x = burn[:, :, d]
        assert abs(x.mean()) < 3 * Dg.mcse_mean(x)
        assert abs(x.var() - 1.0) < 3 * Dg.mcse_var(x)
    U = 0.5 * (burn ** 2).sum(axis=2)  # Gamma(D/2, 1): mean = var = D/2
    assert abs(U.mean() - D / 2) < 3 * Dg.mcse_mean(U)
    assert abs(U.var() - D / 2) < 3 * Dg.mcse_var(U)


@pytest.mark.parametrize("target", ["logreg", "funnel"])
def test_nuts_fsm_equals_sample(small_logreg, target):
    if target == "logreg":
        tg, d = small_logreg
        sp = O.nuts_sampler(0.1, max_depth=6)
    else:
        tg = O.funnel_target(10)
        sp = O.nuts_sampler(0.2, max_depth=8)
    for chain in range(3):
        a = O.run_chain(tg, sp, 5, chain, 150)
        b = O.run_chain(tg, sp, 5, chain, 150, use_fsm=True, want_edges=True)
        assert np.array_equal(a["draws"], b["draws"])
        assert np.array_equal(a["counts"], b["counts"])
        E = b["edges"]
        seen = {(i, k) for i in range(6) for k in range(6) if E[i, k] > 0}
        assert seen <= NUTS_EDGES
        assert {(1, 2), (2, 3), (3, 4), (4, 5), (5, 1)} <= seen


def test_nuts_logreg_near_laplace():
    # a well-conditioned logistic posterior: NUTS means sit near the MAP
    d = inputs.logreg(n_data=2000, dim=4, seed=5)
    tg = O.logreg_target(d["X"].astype(np.float64), d["y"])
    lap = inputs.logreg_laplace(d["X"], d["y"], 8, seed=6)
    draws, counts, _ = O.run_chains(tg, O.nuts_sampler(0.05, 10), 7, range(8), 400, x0=lap["x0"])
    sd = np.sqrt(np.diag(np.linalg.inv(lap["hessian"])))
    mean = draws[:, 50:, :].reshape(-1, 4).mean(axis=0)
    assert np.all(np.abs(mean - lap["map"]) < 0.2 * sd + 4 * sd / np.sqrt(8 * 350 / 4))
    assert counts.min() >= 1 and counts.max() <= 1023

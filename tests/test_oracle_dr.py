"""Pins of the oracle's delayed-rejection MH (Sec. 7.1; FSM of Fig. "Finite
state machines ...", delayed-rejection panel).  Reading: Tierney-Mira
acceptance with every stage centred at the current state."""
import itertools

import numpy as np
import pytest

from oracle import diagnostics as Dg
from oracle import oracle as O

DR_EDGES = {(1, 2), (1, 3), (2, 2), (2, 3), (3, 1)}


def _lattice_kernel(P_off, K):
    k = np.zeros(K)
    for off, w in P_off.items():
        k[off % K] += w
        k[(-off) % K] += w
    return k / k.sum()


def _log(v):
    return np.log(v) if v > 0 else -np.inf


def _dr_matrix(lp, ks):
    """Transition matrix of 3-stage DR on a ring with symmetric kernels ks,
    accumulated path by path from the oracle's acceptance functions."""
    K = lp.size
    q = [lambda a, b, s=s: ks[s][(b - a) % K] for s in range(3)]
    lq = [lambda a, b, s=s: _log(ks[s][(b - a) % K]) for s in range(3)]
    a1 = lambda a, b: np.exp(O.dr_log_alpha1(lp[a], lp[b]))
    a2 = lambda a, b, c: np.exp(O.dr_log_alpha2(lp[a], lp[b], lp[c], lq[0](a, b), lq[0](c, b)))

    def a3(x, y1, y2, y3):
        qq = [lq[0](x, y1), lq[0](y2, y1), lq[1](x, y2), lq[0](y3, y2), lq[1](y3, y1), lq[0](y1, y2)]
        return np.exp(O.dr_log_alpha3(lp[x], lp[y1], lp[y2], lp[y3], qq))

    P = np.zeros((K, K))
    for x in range(K):
        for y1 in range(K):
            p1 = q[0](x, y1)
            if p1 == 0:
                continue
            A1 = a1(x, y1)
            P[x, y1] += p1 * A1
            r1 = p1 * (1 - A1)
            if r1 == 0:
                continue
            for y2 in range(K):
                p2 = q[1](x, y2)
                if p2 == 0:
                    continue
                A2 = a2(x, y1, y2)
                P[x, y2] += r1 * p2 * A2
                r2 = r1 * p2 * (1 - A2)
                if r2 == 0:
                    continue
                for y3 in range(K):
                    p3 = q[2](x, y3)
                    if p3 == 0:
                        continue
                    P[x, y3] += r2 * p3 * a3(x, y1, y2, y3)
        P[x, x] += 1.0 - P[x].sum()
    return P


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_dr_detailed_balance_brute_force(seed):
    g = np.random.default_rng(seed)
    K = 9
    pi = g.uniform(0.05, 1.0, size=K) ** 3
    pi /= pi.sum()
    ks = [_lattice_kernel({1: 0.5, 2: 0.3, 4: 0.2}, K),
          _lattice_kernel({1: 0.7, 3: 0.3}, K),
          _lattice_kernel({0: 0.2, 1: 0.5, 2: 0.3}, K)]
    P = _dr_matrix(np.log(pi), ks)
    assert np.all(P >= -1e-15)
    assert np.allclose(P.sum(axis=1), 1.0, atol=1e-14)
    F = pi[:, None] * P
    assert np.max(np.abs(F - F.T)) <= 1e-13
    assert np.max(np.abs(pi @ P - pi)) <= 1e-13
    # the later stages carry mass: the brute force exercises alpha_2 and alpha_3
    P1 = np.zeros_like(P)
    for x in range(K):
        for y in range(K):
            P1[x, y] = ks[0][(y - x) % K] * np.exp(O.dr_log_alpha1(np.log(pi[x]), np.log(pi[y])))
    assert np.max(np.abs(P - P1) - np.eye(K) * 10) > 1e-3


def test_log1mexp():
    assert O.log1mexp(0.0) == -np.inf
    assert O.log1mexp(-np.inf) == 0.0
    for a in [-1e-12, -1e-3, -0.5, -0.7, -1.0, -5.0, -40.0]:
        assert O.log1mexp(a) == pytest.approx(np.log(-np.expm1(a)), rel=1e-12)


def test_dr_one_stage_is_random_walk_metropolis():
    tg = O.gauss_target(np.array([1.0, 4.0, 0.25]))
    sp = O.dr_sampler(scales=(0.8,), n_stages=1)
    seed, chain, n = 31, 5, 300
    x = O.normal_init(3, seed, chain)
    lx = O.logpdf(tg, x)
    r = O.run_chain(tg, sp, seed, chain, n)
    for t in range(n):
        z = O.normals(seed, chain, t, O.ROLE_PROP, 0, 3)
        y = x + 0.8 * z
        ly = O.logpdf(tg, y)
        if np.log(O.uniform(seed, chain, t, O.ROLE_ACC, 0)) < min(0.0, ly - lx):
            x, lx = y, ly
        assert np.array_equal(r["draws"][t], x)
    assert np.all(r["counts"] == 1)


def test_dr_gaussian_moments():
    tg = O.gauss_target(np.ones(10))
    sp = O.dr_sampler(scales=(1.0, 0.3, 0.1))
    draws, counts, _ = O.run_chains(tg, sp, seed=12, chains=range(32), n=3000)
    burn = draws[:, 300:, :]
    for d in range(10):
        x = burn[:, :, d]
        assert abs(x.mean()) < 3 * Dg.mcse_mean(x)
        assert abs(x.var() - 1.0) < 3 * Dg.mcse_var(x)
    assert set(np.unique(counts)) <= {1, 2, 3}
    assert (counts == 3).any() and (counts == 1).any()


@pytest.mark.parametrize("target", ["funnel", "gauss"])
def test_dr_fsm_equals_sample(target):
    tg = O.funnel_target(10) if target == "funnel" else O.gauss_target(np.linspace(0.5, 2, 10))
    sp = O.dr_sampler(scales=(1.0, 0.3, 0.1))
    for chain in range(4):
        a = O.run_chain(tg, sp, 77, chain, 500)
        b = O.run_chain(tg, sp, 77, chain, 500, use_fsm=True, want_edges=True)
        assert np.array_equal(a["draws"], b["draws"])
        assert np.array_equal(a["counts"], b["counts"])
        E = b["edges"]
        seen = {(i, j) for i in range(4) for j in range(4) if E[i, j] > 0}
        assert seen <= DR_EDGES
        assert b["steps"] == a["counts"].sum() + 2 * 500


def test_funnel_exact_init_and_density():
    x = O.funnel_init(10, 3, 9)
    z = O.normals(3, 9, 0, O.ROLE_INIT, 0, 10)
    assert x[0] == 3 * z[0]
    assert np.allclose(x[1:], np.exp(x[0] / 2) * z[1:], rtol=1e-15)
    tg = O.funnel_target(10)
    v, xs = x[0], x[1:]
    ref = -v * v / 18 - 4.5 * v - 0.5 * np.exp(-v) * np.sum(xs * xs)
    assert O.logpdf(tg, x) == pytest.approx(ref, rel=1e-13)

"""Pins of the oracle's symmetric delayed rejection (Mira 2001; Sec. 7.1).

* the acceptance function satisfies detailed balance along re-centred paths:
  for random points x, y_1 .. y_k and symmetric proposals (which cancel),
    pi(x) prod_{j<k} (1 - a_j(x; y_1..y_j)) a_k(x; y_1..y_k)
      = pi(y_k) prod_{j<k} (1 - a_j(y_k; y_{k-1}..y_{k-j})) a_k(y_k; y_{k-1}..y_1, x),
  with a_j(start; path) = alpha from pi(start), pi(last), max pi(earlier);
* the same on a finite state space by brute force: a ring with a symmetric
  proposal kernel, every re-centred path of up to M tries enumerated, pi P = pi
  and pi_i P_ij = pi_j P_ji;
* one try is random-walk Metropolis (textbook reduction), bit for bit;
* N(0, 1) moments within 3 MCSE; the FSM-step form equals sample().
"""
import numpy as np
import pytest

from oracle import diagnostics as OD
from oracle import oracle as O


def _a(l_start, l_path):
    """alpha of the last point of l_path for a path that starts at l_start."""
    lstar = max(l_path[:-1]) if len(l_path) > 1 else -np.inf
    return O.drsym_alpha(l_start, l_path[-1], lstar)


def _path_weight(l):
    """pi(l[0]) * prob. of rejecting l[1..k-1] and accepting l[k], starting at l[0]."""
    w = np.exp(l[0])
    for j in range(1, len(l) - 1):
        w *= 1.0 - _a(l[0], l[1:j + 1])
    return w * _a(l[0], l[1:])


@pytest.mark.parametrize("k", [1, 2, 3, 4, 6])
def test_alpha_detailed_balance_along_paths(k):
    g = np.random.default_rng(k)
    checked = 0
    for _ in range(4000):
        l = list(g.normal(0.0, 1.5, size=k + 1))
        fwd = _path_weight(l)
        rev = _path_weight(l[::-1])
        assert abs(fwd - rev) <= 1e-12 * max(1.0, abs(fwd)), (l, fwd, rev)
        checked += fwd > 0
    assert checked > 100


def test_brute_force_invariance_on_a_ring():
    K = 7
    pi = np.array([0.05, 0.2, 0.1, 0.3, 0.05, 0.15, 0.15])
    lpi = np.log(pi)
    steps = {-2: 0.15, -1: 0.35, 1: 0.35, 2: 0.15}  # symmetric proposal kernel
    def walk(P, x, c, lstar, prob, s, M):
        # try s from centre c: every move, accept or go on re-centred at y
        for mv, q in steps.items():
            y = (c + mv) % K
            a = O.drsym_alpha(lpi[x], lpi[y], lstar)
            P[x, y] += prob * q * a
            rej = prob * q * (1.0 - a)
            if s + 1 < M:
                walk(P, x, y, max(lstar, lpi[y]), rej, s + 1, M)
            else:
                P[x, x] += rej  # all M tries rejected

    for M in (1, 2, 3, 4, 5):
        P = np.zeros((K, K))
        for x in range(K):
            walk(P, x, x, -np.inf, 1.0, 0, M)
        assert np.allclose(P.sum(axis=1), 1.0, atol=1e-13)
        assert np.allclose(pi @ P, pi, atol=1e-13), M
        F = pi[:, None] * P
        assert np.allclose(F, F.T, atol=1e-13), M


def test_one_try_is_random_walk_metropolis():
    tg = O.gauss_target(np.array([1.0, 4.0]))
    seed, chain, sigma = 3, 5, 0.7
    x = O.normal_init(2, seed, chain)
    r = O.run_chain(tg, O.drsym_sampler(1, sigma), seed, chain, 300)
    for t in range(300):
        y = x + sigma * O.normals(seed, chain, t, O.ROLE_PROP, 0, 2)
        if O.uniform(seed, chain, t, O.ROLE_ACC, 0) < min(1.0, np.exp(O.logpdf(tg, y) - O.logpdf(tg, x))):
            x = y
        assert np.array_equal(r["draws"][t], x)
    assert np.all(r["counts"] == 1)


def test_standard_normal_moments():
    tg = O.gauss_target(np.array([1.0]))
    m, n = 32, 4000
    draws, counts, _ = O.run_chains(tg, O.drsym_sampler(20, 1.5), 17, range(m), n)
    b = draws[:, 400:, 0]
    assert abs(b.mean()) < 3 * OD.mcse_mean(b)
    assert abs(b.var() - 1.0) < 3 * OD.mcse_var(b)
    assert counts.max() > 1 and counts.max() <= 20


def test_fsm_step_equals_sample():
    tg = O.gauss_target(np.array([1.0]))
    for M, sigma in [(100, 0.1), (3, 2.0)]:
        a = O.run_chain(tg, O.drsym_sampler(M, sigma), 9, 2, 500)
        b = O.run_chain(tg, O.drsym_sampler(M, sigma), 9, 2, 500, use_fsm=True)
        assert np.array_equal(a["draws"], b["draws"]) and np.array_equal(a["counts"], b["counts"])
        assert b["steps"] == a["counts"].sum()

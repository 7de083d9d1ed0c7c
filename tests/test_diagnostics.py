"""Pins of the diagnostics: effective sample size and the efficiency bound R(m)."""
import numpy as np

from oracle import diagnostics as Dg


def test_ess_ar1_closed_form():
    # AR(1) with coefficient phi: integrated autocorrelation time (1+phi)/(1-phi)
    g = np.random.default_rng(0)
    for phi in [0.0, 0.5, 0.9]:
        m, n = 8, 20000
        x = np.zeros((m, n))
        e = g.standard_normal((m, n)) * np.sqrt(1 - phi * phi)
        x[:, 0] = g.standard_normal(m)
        for t in range(1, n):
            x[:, t] = phi * x[:, t - 1] + e[:, t]
        want = m * n * (1 - phi) / (1 + phi)
        assert abs(Dg.ess(x) / want - 1) < 0.12, phi


def test_r_of_m_bernoulli_closed_form():
    # N = B * Bern(p) gives R(m) = (1 - (1-p)^m) / p (Sec. 4.2)
    g = np.random.default_rng(1)
    B = 50
    for p in [0.02, 0.1, 0.5]:
        N = B * (g.uniform(size=200000) < p)
        ph = (N > 0).mean()
        for m in [1, 4, 32, 1024]:
            want_hat = (1 - (1 - ph) ** m) / ph
            assert Dg.r_hat_m(N, m) == np.float64(want_hat) or abs(Dg.r_hat_m(N, m) - want_hat) < 1e-9
            want = (1 - (1 - p) ** m) / p
            assert abs(Dg.r_hat_m(N, m) - want) < 0.05 * want + 1e-9


def test_r_of_m_constant_and_geometric():
    assert Dg.r_hat_m(np.full(100, 7), 1000) == 1.0
    # geometric loop counts: E max over m grows like log m
    g = np.random.default_rng(2)
    N = g.geometric(0.2, size=400000)
    r4, r64, r1024 = (Dg.r_hat_m(N, m) for m in (4, 64, 1024))
    assert 1 < r4 < r64 < r1024 < 10

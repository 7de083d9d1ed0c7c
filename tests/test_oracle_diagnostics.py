"""Pins for the oracle's sampler diagnostics (used by the MCSE-based tests and,
through tests/test_diagnostics.py, to check the benchmark's own statistics).

* ESS: for a stationary AR(1) series with coefficient phi the integrated
  autocorrelation time is (1 + phi) / (1 - phi), so long chains give
  ESS ~ m n (1 - phi) / (1 + phi).
* R(m): E[max of m i.i.d. draws] for a two-point law in closed form, and by
  enumeration of every m-tuple for a small support.
"""
import itertools

import numpy as np
import pytest

from oracle import diagnostics as Dg


def _ar1(g, m, n, phi):
    x = np.empty((m, n))
    x[:, 0] = g.standard_normal(m) / np.sqrt(1 - phi * phi)
    for t in range(1, n):
        x[:, t] = phi * x[:, t - 1] + g.standard_normal(m)
    return x


@pytest.mark.parametrize("phi", [0.0, 0.5, 0.9, -0.5])
def test_ess_ar1_closed_form(phi):
    m, n = 8, 20000
    x = _ar1(np.random.default_rng(int(100 * abs(phi)) + (7 if phi >= 0 else 8)), m, n, phi)
    want = m * n * (1 - phi) / (1 + phi)
    got = Dg.ess(x)
    if phi < 0:  # antithetic: Geyer's pairs cap tau near its floor, ESS >= m n
        assert got >= 0.95 * m * n
    else:
        assert got == pytest.approx(want, rel=0.1)


def test_mcse_mean_iid():
    x = np.random.default_rng(3).standard_normal((16, 4000))
    assert Dg.mcse_mean(x) == pytest.approx(1.0 / np.sqrt(x.size), rel=0.1)


@pytest.mark.parametrize("m", [1, 2, 7, 64, 8192])
def test_r_of_m_two_point_closed_form(m):
    counts = np.array([1] * 750 + [2] * 250)  # P(N = 2) = 1/4 exactly
    want = (2.0 - 0.75 ** m) / 1.25
    assert Dg.r_hat_m(counts, m) == pytest.approx(want, rel=1e-12)


@pytest.mark.parametrize("m", [1, 2, 3])
def test_r_of_m_enumeration(m):
    counts = np.array([0, 1, 1, 2, 5, 5, 3])
    e_max = np.mean([max(t) for t in itertools.product(counts, repeat=m)])
    assert Dg.r_hat_m(counts, m) == pytest.approx(e_max / counts.mean(), rel=1e-12)

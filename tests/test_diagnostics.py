"""The benchmark's report statistics (package, host side) against the
oracle's diagnostics, which are pinned on AR(1) series and closed forms in
test_oracle_pins.py.  Two independent implementations of the same
definitions must agree to rounding."""
import numpy as np
import pytest

from oracle import diagnostics as Dg
from paper_2503_17405_amd import diagnostics as P


@pytest.mark.parametrize("m", [1, 16, 1000, 8192])
def test_r_of_m_matches_oracle(m):
    g = np.random.default_rng(m)
    for p in (0.9, 0.5, 0.15):
        counts = g.geometric(p, size=(64, 50))
        assert P.r_of_m(counts, m) == pytest.approx(Dg.r_hat_m(counts, m), rel=1e-12)
    assert P.r_of_m(np.full(10, 3), m) == pytest.approx(1.0)


def _ar1(g, m, n, phi):
    x = np.empty((m, n))
    x[:, 0] = g.standard_normal(m) / np.sqrt(1 - phi * phi)
    for t in range(1, n):
        x[:, t] = phi * x[:, t - 1] + g.standard_normal(m)
    return x


@pytest.mark.parametrize("m,n", [(1, 500), (4, 300), (16, 1000)])
def test_ess_matches_oracle(m, n):
    g = np.random.default_rng(m * 1000 + n)
    cols = [_ar1(g, m, n, phi) for phi in (0.0, 0.5, 0.9, -0.3)]
    cols.append(np.cumsum(g.standard_normal((m, n)), axis=1))  # random walk: ESS near the floor
    x = np.stack(cols, axis=2)
    got = P.ess(x)
    for j in range(x.shape[2]):
        assert got[j] == pytest.approx(Dg.ess(x[:, :, j]), rel=1e-9), j


def test_ess_shapes_and_short_chains():
    x = np.random.default_rng(0).standard_normal((3, 3, 2))
    assert np.all(P.ess(x) == 9.0)
    assert P.ess(np.random.default_rng(1).standard_normal((5, 40))).shape == (1,)

"""Pins of the oracle's target densities and delayed-rejection acceptance
against their textbook definitions, evaluated with scipy (independent code).

* GP-logistic likelihood factor (Appendix, Alg. "Transition kernel for
  elliptical slice sampler", with the log-likelihood-factor reading of
  Sec. 2.2): sum_i log Bernoulli(y_i | sigmoid(f_i)).
* GP-Gaussian likelihood factor: sum_i log N(y_i | f_i, sd^2) up to a constant.
* Logistic-regression potential: -sum_i log Bernoulli(y_i | sigmoid(x_i.b))
  - log N(b | 0, I), up to a constant.
* Neal's funnel: log N(v | 0, 3^2) + sum_i log N(x_i | 0, e^v), up to a
  constant.
* Delayed rejection (Sec. 7.1; Tierney and Mira 1999): the stage-2 and
  stage-3 acceptance probabilities assembled in this file from Gaussian
  proposal densities N(b | a, scale_s^2 I) written with scipy, including the
  stage-2/3 proposal factors that cancel for proposals centred at the
  current state, compared with the acceptance the oracle's draw uses.

Constants of the densities are removed by comparing differences between
points, so a misread normalisation cannot hide a misread shape.
"""
import numpy as np
import pytest
from scipy import stats
from scipy.special import expit

from oracle import oracle as O
from paper_2503_17405_amd import inputs


def _pairs(rng, D, n, scale):
    return [(rng.standard_normal(D) * scale, rng.standard_normal(D) * scale) for _ in range(n)]


def test_gp_logistic_loglik_is_bernoulli_logpmf():
    rng = np.random.default_rng(0)
    for D in [1, 7, 64, 300]:
        y = (rng.uniform(size=D) < 0.5).astype(np.float64)
        tg = O.gp_target(y)
        for scale in [0.1, 1.0, 3.0]:
            # |f| <= 8 keeps scipy's log(1 - sigmoid(f)) accurate (1 - p >= 3e-4)
            f = np.clip(rng.standard_normal(D) * scale, -8.0, 8.0)
            ref = stats.bernoulli.logpmf(y, expit(f)).sum()
            assert O.gp_loglik(tg, f) == pytest.approx(ref, rel=1e-10, abs=1e-10), (D, scale)


def test_gp_gauss_loglik_is_normal_logpdf_up_to_a_constant():
    rng = np.random.default_rng(1)
    for D, sd in [(16, 0.1), (5, 1.3)]:
        y = rng.standard_normal(D)
        tg = O.gp_target(y, noise_sd=sd)
        for a, b in _pairs(rng, D, 5, 1.0):
            ref = stats.norm.logpdf(y, a, sd).sum() - stats.norm.logpdf(y, b, sd).sum()
            got = O.gp_loglik(tg, a) - O.gp_loglik(tg, b)
            assert got == pytest.approx(ref, rel=1e-10, abs=1e-9)


def test_logreg_potential_is_bernoulli_plus_gaussian_prior():
    d = inputs.logreg(n_data=300, dim=6, seed=5)
    X, y = d["X"].astype(np.float64), d["y"]
    tg = O.logreg_target(X, y)
    prior = stats.multivariate_normal(np.zeros(6), np.eye(6))

    def logpost(b):
        return stats.bernoulli.logpmf(y, expit(X @ b)).sum() + prior.logpdf(b)

    rng = np.random.default_rng(2)
    for a, b in _pairs(rng, 6, 6, 0.7):
        ref = -(logpost(a) - logpost(b))
        got = O.potential(tg, a) - O.potential(tg, b)
        assert got == pytest.approx(ref, rel=1e-9, abs=1e-9)


@pytest.mark.parametrize("D", [2, 10])
def test_funnel_density_is_neal_funnel(D):
    tg = O.funnel_target(D)

    def ref(x):
        v = x[0]
        return stats.norm.logpdf(v, 0.0, 3.0) + stats.norm.logpdf(x[1:], 0.0, np.exp(v / 2)).sum()

    rng = np.random.default_rng(D)
    for a, b in _pairs(rng, D, 8, 1.5):
        got = O.logpdf(tg, a) - O.logpdf(tg, b)
        assert got == pytest.approx(ref(a) - ref(b), rel=1e-10, abs=1e-10)


# --------------------------------------------------------------- DR
def _lq(a, b, sc):
    """log q(a -> b) for a proposal N(b | a, sc^2 I), from scipy."""
    return stats.multivariate_normal(a, sc * sc * np.eye(a.size)).logpdf(b)


def _log1m(la):
    """log(1 - e^la) for la <= 0."""
    return np.log(-np.expm1(la)) if la < 0 else -np.inf


def _tm_alphas(lpi, x, ys, scales):
    """Tierney-Mira log acceptance of stages 1..len(ys) from x, every stage's
    proposal centred at the current state: q_s(a, ..., b) = N(b | a, sc_s^2)."""
    s1, s2 = scales[0], scales[1] if len(scales) > 1 else None
    s3 = scales[2] if len(scales) > 2 else None
    la1 = lambda a, b: min(0.0, lpi(b) - lpi(a))  # noqa: E731

    def la2(a, b, c):
        # from a, b rejected at stage 1, c proposed at stage 2
        num = lpi(c) + _lq(c, b, s1) + _lq(c, a, s2) + _log1m(la1(c, b))
        den = lpi(a) + _lq(a, b, s1) + _lq(a, c, s2) + _log1m(la1(a, b))
        return -np.inf if num == -np.inf else min(0.0, num - den)

    out = [la1(x, ys[0])]
    if len(ys) > 1:
        out.append(la2(x, ys[0], ys[1]))
    if len(ys) > 2:
        y1, y2, y3 = ys
        num = (lpi(y3) + _lq(y3, y2, s1) + _lq(y3, y1, s2) + _lq(y3, x, s3)
               + _log1m(la1(y3, y2)) + _log1m(la2(y3, y2, y1)))
        den = (lpi(x) + _lq(x, y1, s1) + _lq(x, y2, s2) + _lq(x, y3, s3)
               + _log1m(la1(x, y1)) + _log1m(la2(x, y1, y2)))
        out.append(min(0.0, num - den))
    return out


@pytest.mark.parametrize("scales", [(1.0, 0.3, 0.1), (2.5, 0.7, 0.25)])
def test_dr_stage_acceptance_matches_tierney_mira(scales):
    prec = np.array([0.5, 1.0, 2.0, 4.0])
    tg = O.gauss_target(prec)
    sp = O.dr_sampler(scales)
    mvn = stats.multivariate_normal(np.zeros(4), np.diag(1.0 / prec))
    lpi = mvn.logpdf
    rng = np.random.default_rng(7)
    seed, reached = 123, {0: 0, 1: 0, 2: 0}
    for trial in range(400):
        x = rng.standard_normal(4) * 1.5
        draw, chain = trial, trial % 5
        xo, cnt, mar, _ = O.draw_traced(tg, sp, seed, chain, draw, x)
        ys = [x + scales[s] * O.normals(seed, chain, draw, O.ROLE_PROP, s, 4) for s in range(cnt)]
        la = _tm_alphas(lpi, x, ys, scales)
        for s in range(cnt):
            lu = np.log(O.uniform(seed, chain, draw, O.ROLE_ACC, s))
            reached[s] += 1
            if np.isfinite(la[s]):
                assert mar[s] == pytest.approx(abs(lu - la[s]), rel=1e-8, abs=1e-9), (trial, s)
            else:
                assert mar[s] == np.inf
            acc = lu < la[s]
            assert acc == (s == cnt - 1 and not np.array_equal(xo, x)), (trial, s)
        if not np.array_equal(xo, x):
            assert np.array_equal(xo, ys[cnt - 1])
    # every stage was exercised many times
    assert reached[1] > 100 and reached[2] > 50, reached


# ----------------------------------------------------- the decision record
def _targets():
    w = inputs.gp_logistic(dim=48, lengthscale=0.1, seed=3)
    d = inputs.logreg(n_data=200, dim=5, seed=4)
    return [
        ("ess", O.gp_target(w["y"]), O.ess_sampler(w["L"]), lambda s, j: O.ess_init(w["L"], s, j)),
        ("nuts", O.logreg_target(d["X"].astype(np.float64), d["y"]), O.nuts_sampler(0.15, 6),
         lambda s, j: O.normal_init(5, s, j) * 0.3),
        ("dr", O.funnel_target(10), O.dr_sampler(), lambda s, j: O.funnel_init(10, s, j)),
    ]


@pytest.mark.parametrize("name,tg,sp,init", _targets())
def test_traced_draw_is_the_chain_draw(name, tg, sp, init):
    seed, chain, n = 11, 3, 25
    x0 = init(seed, chain)
    r = O.run_chain(tg, sp, seed, chain, n, x0=x0)
    x = x0
    for t in range(n):
        xn, cnt, mar, sca = O.draw_traced(tg, sp, seed, chain, t, x)
        assert np.array_equal(xn, r["draws"][t]), (name, t)
        assert cnt == r["counts"][t]
        assert mar.size >= 1 and np.all(sca >= 0)
        x = xn


@pytest.mark.parametrize("name,tg,sp,init", _targets())
def test_parting_check_accepts_only_a_near_tie_flip(name, tg, sp, init):
    """A draw that differs from the oracle by one inverted decision is
    explained when that decision is a near-tie (eps large enough to make it
    one) and is not when it is not; an arbitrary perturbation of the draw is
    never explained."""
    import parity
    seed, chain = 5, 1
    x = init(seed, chain)
    for t in range(40):
        xn, cnt, mar, sca = O.draw_traced(tg, sp, seed, chain, t, x)
        rel = mar / (1 + sca)
        order = [k for k in np.argsort(rel, kind="stable") if np.isfinite(rel[k])]
        for i, k in enumerate(order[:3]):
            xf, cf, _, _ = O.draw_traced(tg, sp, seed, chain, t, x, flip_at=int(k))
            if cf == cnt and parity.rel_err(xf, xn) <= 1e-4:
                continue  # an inversion that changes nothing cannot be seen
            ok, kk, _, _ = parity.explain_parting(tg, sp, seed, chain, t, x, xf, cf, eps=rel[k] / 32)
            assert ok, (name, t, k)
            if i == 0:
                # with the threshold below every margin of the draw nothing explains it
                ok, _, _, _ = parity.explain_parting(tg, sp, seed, chain, t, x, xf, cf, eps=rel[k] / 128)
                assert not ok, (name, t, k)
        bad = xn + 1e-2 * (1.0 + np.abs(xn))
        ok, _, _, _ = parity.explain_parting(tg, sp, seed, chain, t, x, bad, cnt, eps=1.0)
        assert not ok
        x = xn

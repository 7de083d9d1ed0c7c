"""Pins of the oracle's slice sampler along random directions (Neal 2003;
Sec. 3.1's five-state slice FSM).

* the FSM-step form equals sample() bit for bit, and every transition it
  takes is an edge of the FSM that fsmgen builds from the slice program
  (which matches the paper's figure);
* invariance, checked on closed forms: N(0, diag(1/prec)) moments, and the
  funnel's v marginal N(0, 9), within 3 MCSE;
* one draw written out from the definition (stepping out, shrinkage) with
  the oracle's random streams reproduces the oracle's draw.
"""
import numpy as np
import pytest

from oracle import diagnostics as OD
from oracle import oracle as O
from paper_2503_17405_amd import fsm_programs as P
from paper_2503_17405_amd import fsmgen as G


@pytest.mark.parametrize("target", ["gauss", "funnel"])
def test_fsm_step_equals_sample_and_follows_the_fsm(target):
    tg = O.gauss_target(np.array([1.0, 4.0, 0.25])) if target == "gauss" else O.funnel_target(10)
    sp = O.slice_sampler(1.0)
    a = O.run_chain(tg, sp, 5, 3, 300)
    b = O.run_chain(tg, sp, 5, 3, 300, use_fsm=True, want_edges=True)
    assert np.array_equal(a["draws"], b["draws"]) and np.array_equal(a["counts"], b["counts"])
    fsm = G.make_fsm(P.SLICE)
    allowed = set(fsm.edges) | {(5, 1)}  # DONE -> INIT E: the next draw
    taken = {(i, j) for i in range(6) for j in range(6) if b["edges"][i, j] > 0}
    assert taken <= allowed, taken - allowed
    assert (2, 2) in taken and (4, 4) in taken  # both loops ran
    assert a["guards"] == 0 and a["counts"].min() >= 3


def test_gaussian_moments():
    prec = np.array([1.0, 4.0, 0.25])
    tg = O.gauss_target(prec)
    draws, counts, _ = O.run_chains(tg, O.slice_sampler(1.0), 7, range(24), 3000)
    b = draws[:, 300:, :]
    for d in range(3):
        assert abs(b[:, :, d].mean()) < 3 * OD.mcse_mean(b[:, :, d]), d
        assert abs(b[:, :, d].var() - 1.0 / prec[d]) < 3 * OD.mcse_var(b[:, :, d]), d


def test_funnel_v_marginal():
    tg = O.funnel_target(10)
    draws, counts, guards = O.run_chains(tg, O.slice_sampler(1.0), 11, range(32), 3000)
    v = draws[:, 300:, 0]
    assert abs(v.mean()) < 3 * OD.mcse_mean(v)
    assert abs(v.var() - 9.0) < 3 * OD.mcse_var(v)
    assert np.sum(guards) == 0
    print("funnel slice: mean evaluations %.1f, max %d" % (counts.mean(), counts.max()))


def test_one_draw_from_the_definition():
    tg = O.gauss_target(np.array([1.0, 2.0]))
    seed, chain, w = 13, 4, 0.5
    x = np.array([0.3, -1.2])
    for t in range(50):
        lx = O.logpdf(tg, x)
        logy = lx + np.log(O.uniform(seed, chain, t, O.ROLE_THRESH, 0))
        z = O.normals(seed, chain, t, O.ROLE_NU, 0, 2)
        d = z / np.sqrt(z @ z)
        L = -w * O.uniform(seed, chain, t, O.ROLE_ANGLE, 0)
        R = L + w
        inside = lambda s: O.logpdf(tg, x + s * d) > logy
        n = 2
        inL, inR = inside(L), inside(R)
        while inL or inR:
            if inL:
                L -= w
                inL = inside(L)
            else:
                R += w
                inR = inside(R)
            n += 1
        s = 0
        while True:
            tt = L + (R - L) * O.uniform(seed, chain, t, O.ROLE_ANGLE, 1 + s)
            n += 1
            if inside(tt):
                break
            if tt < 0:
                L = tt
            else:
                R = tt
            s += 1
        want = x + tt * d
        got, cnt, _, _ = O.draw_traced(tg, O.slice_sampler(w), seed, chain, t, x)
        assert cnt == n, t
        assert np.allclose(got, want, rtol=0, atol=1e-14), t
        x = got

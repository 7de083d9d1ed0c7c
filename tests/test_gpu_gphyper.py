"""GPU parity of elliptical slice sampling on GP-regression hyperparameters
(Sec. 7.2): an O(n^3) Cholesky of the n x n kernel matrix inside every loop
iteration, computed in FP64 by the chain's wavefront (n <= 96) or by a
block with a blocked factorisation (n > 96).  FSM runtime ==
synchronized runtime (vmap and compact) bit for bit; draws match the FP64
oracle per draw (1e-9 relative: both sides FP64, the factorisations add up
in different orders)."""
import numpy as np
import pytest
import torch

import parity
from oracle import oracle as O
from paper_2503_17405_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    from paper_2503_17405_amd import fsmmc
    return fsmmc


@pytest.fixture(scope="module")
def ctx(F):
    c = F.Context(0)
    yield c
    c.close()


def target(F, w):
    return F.gp_hyper_target(torch.tensor(w["X"], device="cuda"), torch.tensor(w["y"], device="cuda"),
                             w["jitter"])


def run(F, ctx, w, m, n, seed, runtime="fsm", max_steps=0, x0=None):
    x0t = None if x0 is None else torch.tensor(x0, device="cuda")
    job = F.Job(ctx, target(F, w), F.ess_sampler(F.F64), m, n, seed, x0=x0t)
    try:
        if runtime == "fsm":
            for _ in range(100000):
                if job.step_fsm(max_steps):
                    break
        else:
            assert job.step_synchronized(n, F.SYNC_VMAP if runtime == "vmap" else F.SYNC_COMPACT)
        return job.samples(), job.counts(), job.stats()
    finally:
        job.free()


@pytest.mark.parametrize("nobs,m,n", [(40, 96, 30), (300, 24, 6)])
def test_gphyper_runtimes_bit_exact(F, ctx, nobs, m, n):
    w = inputs.gp_hyper(n=nobs, seed=11)
    seed = 12
    S0, C0, st0 = run(F, ctx, w, m, n, seed, runtime="vmap")
    for runtime, steps in [("fsm", 0), ("fsm", 3), ("compact", 0)]:
        S, C, st = run(F, ctx, w, m, n, seed, runtime, steps)
        assert np.array_equal(S, S0) and np.array_equal(C, C0), (runtime, steps)
        assert st["steps"] == C.sum()
    assert st0["steps"] + st0["padded_steps"] == m * C0.max(axis=0).sum()
    assert st0["guard_trips"] == 0 and np.isfinite(S0).all()
    print("GP hyper n=%d: mean evaluations %.2f, mean max over %d chains %.1f, R %.2f"
          % (nobs, C0.mean(), m, C0.max(axis=0).mean(), st0["r_hat"]))


@pytest.mark.parametrize("nobs", [1, 25, 64, 65, 96, 97, 100, 128, 129, 250, 414])
def test_gphyper_oracle_parity(F, ctx, nobs):
    # up to 96: the chain's wave (one row per lane up to 64, two above);
    # 97 .. 414: the block factorisation (a ragged last panel at 97, 100, 129,
    # 250 and 414; 414 is the paper's data size)
    m = 32 if nobs <= 128 else 8
    w = inputs.gp_hyper(n=nobs, n_chains=m, seed=20 + nobs)
    n, seed = (100 if nobs < 96 else 40 if nobs <= 128 else 12), 21 + nobs
    x0 = w["x0"]
    S, C, _ = run(F, ctx, w, m, n, seed, x0=x0)
    tg = O.gp_hyper_target(w["X"], w["y"], w["jitter"])
    sp = O.ess_sampler(np.eye(3))
    R, RC, _ = O.run_chains(tg, sp, seed, range(m), n, x0=x0)
    r = parity.check_chains(S, C, R, RC, tg, sp, seed, range(m), x0, first=n, tol=1e-9)
    print(parity.summary("GP hyper n=%d" % nobs, r))
    assert r["worst"] <= 1e-9 and not r["bad"]
    assert r["flip_frac"] <= 0.05


def test_gphyper_default_start(F, ctx):
    # no x0: theta0 from the prior on the INIT stream, as the oracle's ESS start
    w = inputs.gp_hyper(n=10, seed=3)
    m, n, seed = 16, 50, 4
    S, C, _ = run(F, ctx, w, m, n, seed)
    tg = O.gp_hyper_target(w["X"], w["y"], w["jitter"])
    sp = O.ess_sampler(np.eye(3))
    R, RC, _ = O.run_chains(tg, sp, seed, range(m), n)
    x_init = np.array([O.ess_init(np.eye(3), seed, j) for j in range(m)])
    r = parity.check_chains(S, C, R, RC, tg, sp, seed, range(m), x_init, first=n, tol=1e-9)
    assert r["worst"] <= 1e-9 and not r["bad"]


def test_gphyper_argument_errors(F, ctx):
    w = inputs.gp_hyper(n=513, seed=1)
    with pytest.raises(F.FsmmcError) as e:
        F.Job(ctx, target(F, w), F.ess_sampler(F.F64), 4, 4, 1)
    assert e.value.status == F.ENOTSUP
    w = inputs.gp_hyper(n=10, seed=1)
    with pytest.raises(F.FsmmcError) as e:
        F.Job(ctx, target(F, w), F.ess_sampler(F.F32), 4, 4, 1)
    assert e.value.status == F.ENOTSUP

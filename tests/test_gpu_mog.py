"""GPU parity of NUTS on the correlated mixture of Gaussians (Sec. 7.3)
through the C ABI: the persistent kernel with the gradient computed by each
chain's wavefront.

* U and grad U against the FP64 oracle at exact mixture draws;
* FSM runtime == synchronized runtime (vmap and compact), bit for bit, for
  several step budgets; the vmap padding makes every draw cost m * max_j N_j;
* GPU vs the FP64 oracle per draw over the first 100 draws (1e-4 relative;
  a parting must be the oracle's draw with one near-tie decision inverted),
  and the acceptance statistic against the oracle's;
* the loop-count statistics of fsmmc_job_stats (histogram, R(m)) against
  the counts themselves.
"""
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


def mog_job(F, ctx, w, m, n, seed, eps, J, x0=None, out=None):
    means = torch.tensor(w["means"], device="cuda")
    logw = torch.tensor(w["log_weights"], device="cuda")
    prec = torch.tensor(w["prec"], device="cuda")
    x0t = None if x0 is None else torch.tensor(np.asarray(x0), dtype=torch.float32, device="cuda")
    return F.Job(ctx, F.mog_target(means, logw, prec), F.nuts_sampler(eps, J), m, n, seed, x0=x0t, out=out)


def run(F, ctx, w, m, n, seed, eps, J, x0=None, runtime="fsm", max_steps=0):
    job = mog_job(F, ctx, w, m, n, seed, eps, J, x0=x0)
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


def oracle_target(w):
    return O.mog_target(w["means"].astype(np.float64), w["log_weights"].astype(np.float64),
                        w["prec"].astype(np.float64))


@pytest.mark.parametrize("D,K", [(100, 3), (37, 2), (64, 1)])
def test_mog_potential_and_gradient_vs_oracle(F, ctx, D, K):
    modes = (-10.0, 0.0, 10.0)[:K] if K > 1 else (2.0,)
    w = inputs.mog(dim=D, modes=modes, n_chains=50, seed=D + K)
    job = mog_job(F, ctx, w, 50, 1, 1, 0.05, 4)
    try:
        pts = w["x0"].astype(np.float32)
        U, g = job.potential(torch.tensor(pts, device="cuda"))
        U, g = U.cpu().numpy().astype(np.float64), g.cpu().numpy().astype(np.float64)
    finally:
        job.free()
    tg = oracle_target(w)
    for i in range(50):
        Ur, gr = O.potential(tg, pts[i].astype(np.float64), grad=True)
        # FP32 results of sums carried in FP64: a few FP32 roundings of the result
        assert abs(U[i] - Ur) <= 1e-6 * (1.0 + abs(Ur)), (i, U[i], Ur)
        assert np.max(np.abs(g[i] - gr)) <= 1e-6 * (1.0 + np.abs(gr).max()), (i, np.max(np.abs(g[i] - gr)))


def test_mog_fsm_equals_synchronized(F, ctx):
    w = inputs.mog(dim=100, n_chains=64, seed=61)
    m, n, seed, eps, J = 64, 40, 62, 0.0473, 10
    ref = run(F, ctx, w, m, n, seed, eps, J, x0=w["x0"], runtime="vmap")
    for runtime, steps in [("fsm", 0), ("fsm", 7), ("fsm", 333), ("compact", 0)]:
        S, C, st = run(F, ctx, w, m, n, seed, eps, J, x0=w["x0"], runtime=runtime, max_steps=steps)
        assert np.array_equal(S, ref[0]), (runtime, steps)
        assert np.array_equal(C, ref[1]), (runtime, steps)
        assert st["steps"] == C.sum(), (runtime, steps)
        assert st["padded_steps"] == 0
    C, st = ref[1], ref[2]
    assert st["steps"] + st["padded_steps"] == m * C.max(axis=0).sum()
    assert C.min() >= 1 and C.max() <= 2 ** J - 1 and np.isfinite(ref[0]).all()
    # loop-count statistics of the job against the counts
    hist = np.bincount(np.minimum(C.ravel(), F.HIST_BINS - 1), minlength=F.HIST_BINS)
    assert np.array_equal(st["hist"], hist)
    assert st["mean_loops"] == pytest.approx(C.mean(), rel=1e-12)
    assert st["mean_max_loops"] == pytest.approx(C.max(axis=0).mean(), rel=1e-12)
    assert st["r_hat"] == pytest.approx(C.max(axis=0).mean() / C.mean(), rel=1e-12)
    assert st["active_lanes"] == st["steps"] * 100
    assert 0.0 < st["accept_sum"] <= st["steps"]
    print("MoG D=100 m=64: mean leapfrogs %.2f, mean max %.1f, R(64) %.2f, acceptance %.3f"
          % (C.mean(), C.max(axis=0).mean(), st["r_hat"], st["accept_sum"] / st["steps"]))


def test_mog_oracle_parity_first_100_draws(F, ctx):
    # a step where a few trajectories run to hundreds of leapfrogs
    w = inputs.mog(dim=100, n_chains=16, seed=71)
    m, n, seed, eps, J = 16, 100, 72, 0.0445, 10
    S, C, st = run(F, ctx, w, m, n, seed, eps, J, x0=w["x0"])
    tg = oracle_target(w)
    x0 = w["x0"].astype(np.float32).astype(np.float64)  # the GPU chains start from the FP32 values
    R, RC, _ = O.run_chains(tg, O.nuts_sampler(eps, J), seed, range(m), n, x0=x0)
    r = parity.check_chains(S, C, R, RC, tg, O.nuts_sampler(eps, J), seed, range(m), x0, first=n)
    print(parity.summary("NUTS MoG D=100, first 100 draws", r))
    assert r["worst"] <= 1e-4 and not r["bad"]
    assert r["flip_frac"] <= 0.25
    print("leapfrogs per draw: mean %.1f, max %d" % (C.mean(), C.max()))
    # the acceptance statistic, summed over every leapfrog, against the
    # oracle's (when no chain parted from it)
    if r["parted"] == 0:
        acc = 0.0
        for j in range(m):
            th = x0[j].copy()
            U, g = O.potential(tg, th, grad=True)
            for t in range(n):
                th, U, g, info = O.nuts_sample(tg, eps, J, seed, j, t, th, U, g)
                acc += info["accept"]
        assert st["accept_sum"] == pytest.approx(acc, rel=1e-4)


def test_mog_default_init_and_small_dims(F, ctx):
    # N(0, I) starts, D = 5 (one register per lane), depth 6, two components
    w = inputs.mog(dim=5, rho=0.5, modes=(-2.0, 2.0), n_chains=0, seed=3)
    m, n, seed, eps, J = 24, 60, 5, 0.3, 6
    S, C, _ = run(F, ctx, w, m, n, seed, eps, J)
    tg = oracle_target(w)
    R, RC, _ = O.run_chains(tg, O.nuts_sampler(eps, J), seed, range(m), n)
    x_init = np.array([O.normal_init(5, seed, j) for j in range(m)])
    r = parity.check_chains(S, C, R, RC, tg, O.nuts_sampler(eps, J), seed, range(m), x_init, first=n)
    print(parity.summary("NUTS MoG D=5", r))
    assert r["worst"] <= 1e-4 and not r["bad"] and r["flip_frac"] <= 0.25
    # the synchronized runtime from the default start gives the same bits
    S2, C2, _ = run(F, ctx, w, m, n, seed, eps, J, runtime="compact")
    assert np.array_equal(S, S2) and np.array_equal(C, C2)


def test_mog_argument_errors(F, ctx):
    w = inputs.mog(dim=8, n_chains=0, seed=1)
    means = torch.tensor(w["means"], device="cuda")
    logw = torch.tensor(w["log_weights"], device="cuda")
    prec = torch.tensor(w["prec"], device="cuda")
    spec, keep = F.mog_target(means, logw, prec)
    bad = F.TargetSpec(spec.kind, spec.dim, 9, 0, spec.X, spec.y, None, spec.prec, 0.0)
    with pytest.raises(F.FsmmcError) as e:
        F.Job(ctx, (bad, keep), F.nuts_sampler(0.1, 5), 4, 4, 1)
    assert e.value.status == F.EINVAL
    noprec = F.TargetSpec(spec.kind, spec.dim, 3, 0, spec.X, spec.y, None, None, 0.0)
    with pytest.raises(F.FsmmcError) as e:
        F.Job(ctx, (noprec, keep), F.nuts_sampler(0.1, 5), 4, 4, 1)
    assert e.value.status == F.EINVAL
    # not batched or served
    job = F.Job(ctx, (spec, keep), F.nuts_sampler(0.1, 5), 4, 4, 1)
    try:
        with pytest.raises(F.FsmmcError) as e:
            F.Batch(ctx, [job])
        assert e.value.status == F.ENOTSUP
    finally:
        job.free()

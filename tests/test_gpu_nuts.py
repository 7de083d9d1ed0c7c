"""GPU parity of NUTS on Bayesian logistic regression through the C ABI.

* FSM runtime == synchronized runtime (vmap and compact), bit for bit.
* GPU vs the FP64 oracle per draw: 1e-4 relative over the first draws up to
  the draw where a chain parts from the oracle; that draw must be the
  oracle's draw with one near-tie decision inverted.
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


def gpu_nuts(F, ctx, d, m, n, seed, eps, J, x0=None, runtime="fsm", max_steps=0, out=None):
    X = torch.tensor(d["X"], dtype=torch.float32, device="cuda")
    y = torch.tensor(d["y"], dtype=torch.float32, device="cuda")
    x0t = None if x0 is None else torch.tensor(np.asarray(x0), dtype=torch.float32, device="cuda")
    job = F.Job(ctx, F.logreg_target(X, y), F.nuts_sampler(eps, J), m, n, seed, x0=x0t, out=out)
    try:
        if runtime == "fsm":
            for _ in range(100000):
                if job.step_fsm(max_steps):
                    break
        else:
            mode = F.SYNC_VMAP if runtime == "vmap" else F.SYNC_COMPACT
            assert job.step_synchronized(n, mode)
        if out is not None:
            return None, job.counts(), job.stats()
        return job.samples(), job.counts(), job.stats()
    finally:
        job.free()


def oracle_nuts(d, m, n, seed, eps, J, x0=None):
    tg = O.logreg_target(d["X"].astype(np.float64), d["y"])
    draws, counts, _ = O.run_chains(tg, O.nuts_sampler(eps, J), seed, range(m), n, x0=x0)
    return draws, counts, tg


def check_parity(S, C, R, RC, tg, seed, eps, J, x0, first, chains=None):
    """Per-draw comparison with the oracle; a parting must be the oracle's
    draw with one near-tie decision inverted."""
    m = S.shape[0]
    chains = list(range(m)) if chains is None else list(chains)
    x_init = x0 if x0 is not None else np.array([O.normal_init(tg.dim, seed, j) for j in chains])
    return parity.check_chains(S, C, R, RC, tg, O.nuts_sampler(eps, J), seed, chains, x_init,
                               first=first)


@pytest.mark.parametrize("N,D", [(2000, 20), (10000, 100), (777, 3), (1, 1), (513, 64), (1001, 65), (3000, 128)])
def test_logreg_potential_and_gradient_vs_oracle(F, ctx, N, D):
    # the fused MFMA gradient kernel against the oracle's plain sums
    d = inputs.logreg(n_data=N, dim=D, seed=N * 7 + D)
    X = torch.tensor(d["X"], dtype=torch.float32, device="cuda")
    y = torch.tensor(d["y"], dtype=torch.float32, device="cuda")
    m = 70
    job = F.Job(ctx, F.logreg_target(X, y), F.nuts_sampler(0.1, 5), m, 2, 1)
    try:
        th = np.random.default_rng(D).standard_normal((m, D)) * 0.3
        U, g = job.potential(torch.tensor(th, dtype=torch.float32, device="cuda"))
        U, g = U.cpu().numpy().astype(np.float64), g.cpu().numpy().astype(np.float64)
    finally:
        job.free()
    tg = O.logreg_target(d["X"].astype(np.float64), d["y"])
    for i in range(m):
        th32 = th[i].astype(np.float32).astype(np.float64)
        Ur, gr = O.potential(tg, th32, grad=True)
        scale = 1.0 + np.abs(d["X"]).sum(axis=0).max()  # bound on |sum_i x_id r_i|
        assert abs(U[i] - Ur) <= 1e-5 * (1.0 + N), (i, U[i], Ur)
        assert np.max(np.abs(g[i] - gr)) <= 1e-5 * scale, (i, np.max(np.abs(g[i] - gr)))


def test_nuts_fsm_equals_synchronized(F, ctx):
    d = inputs.logreg(n_data=700, dim=7, seed=41)
    lap = inputs.logreg_laplace(d["X"], d["y"], 70, seed=42)
    m, n, seed, eps, J = 70, 60, 43, 0.08, 6
    ref = gpu_nuts(F, ctx, d, m, n, seed, eps, J, x0=lap["x0"], runtime="vmap")
    for runtime, steps in [("fsm", 0), ("fsm", 3), ("fsm", 17), ("compact", 0)]:
        S, C, st = gpu_nuts(F, ctx, d, m, n, seed, eps, J, x0=lap["x0"], runtime=runtime, max_steps=steps)
        assert np.array_equal(S, ref[0]), (runtime, steps)
        assert np.array_equal(C, ref[1]), (runtime, steps)
        assert st["steps"] == C.sum()
    C = ref[1]
    assert ref[2]["steps"] + ref[2]["padded_steps"] == m * C.max(axis=0).sum()
    assert C.min() >= 1 and C.max() <= 2 ** J - 1


@pytest.mark.parametrize("N,D,eps,J", [(2000, 20, 0.05, 10), (777, 3, 0.1, 8), (1000, 64, 0.05, 10),
                                       (1001, 65, 0.05, 8), (3000, 128, 0.03, 8)])
def test_nuts_oracle_parity(F, ctx, N, D, eps, J):
    # 32 chains: the rows go out in 32-row slices (a ragged last one at N = 1001);
    # D = 65 and 128: the first and the last dimension of the wide tile
    d = inputs.logreg(n_data=N, dim=D, seed=N + D)
    m, n, seed = 32, 60, 7
    lap = inputs.logreg_laplace(d["X"], d["y"], m, seed=8)
    S, C, st = gpu_nuts(F, ctx, d, m, n, seed, eps, J, x0=lap["x0"])
    R, RC, tg = oracle_nuts(d, m, n, seed, eps, J, x0=lap["x0"])
    r = check_parity(S, C, R, RC, tg, seed, eps, J, lap["x0"], first=n)
    print(parity.summary("NUTS N=%d D=%d" % (N, D), r))
    assert r["worst"] <= 1e-4
    assert not r["bad"]
    assert r["flip_frac"] <= 0.25


def test_nuts_logreg_c3_shape_parity(F, ctx):
    # the benchmark's logistic-regression shape (N=10000, D=100, eps=0.05, depth 10)
    d = inputs.logreg(n_data=10000, dim=100, seed=3001)
    m, n, seed, eps, J = 16, 100, 3003, 0.05, 10
    lap = inputs.logreg_laplace(d["X"], d["y"], m, seed=3002)
    S, C, _ = gpu_nuts(F, ctx, d, m, n, seed, eps, J, x0=lap["x0"])
    R, RC, tg = oracle_nuts(d, m, n, seed, eps, J, x0=lap["x0"])
    r = check_parity(S, C, R, RC, tg, seed, eps, J, lap["x0"], first=n)
    print(parity.summary("NUTS C3 shape, first 100 draws", r))
    assert r["worst"] <= 1e-4 and not r["bad"]
    assert r["flip_frac"] <= 0.25


def test_nuts_c3_full_size_sampled_chains_oracle_parity(F, ctx):
    """The benchmark's NUTS job itself (8192 chains x 1000 draws, N = 10000,
    D = 100): sampled chains against the oracle run for those chains alone,
    over their first 100 draws; partings must be near-tie flips."""
    d = inputs.logreg(n_data=10000, dim=100, seed=3001)
    m, n, seed, eps, J, first = 8192, 1000, 3003, 0.05, 10, 100
    lap = inputs.logreg_laplace(d["X"], d["y"], m, seed=3002)
    out = torch.empty((m, n, 100), dtype=torch.float32, device="cuda")
    _, C, st = gpu_nuts(F, ctx, d, m, n, seed, eps, J, x0=lap["x0"], out=out)
    idx = [0, 1, 4095, 8191] + sorted(int(i) for i in np.random.default_rng(13).choice(m, 4, replace=False))
    S = out[idx, :first].cpu().numpy()
    del out
    torch.cuda.empty_cache()
    assert st["chains_done"] == m and st["draws"] == m * n
    tg = O.logreg_target(d["X"].astype(np.float64), d["y"])
    x0 = lap["x0"][idx]
    R, RC, _ = O.run_chains(tg, O.nuts_sampler(eps, J), seed, idx, first, x0=x0)
    r = check_parity(S, C[idx], R, RC, tg, seed, eps, J, x0, first=first, chains=idx)
    print(parity.summary("C3 full size, chains %s" % idx, r))
    assert r["worst"] <= 1e-4 and not r["bad"]
    assert r["parted"] <= 2


def test_nuts_depth_one_and_default_init(F, ctx):
    d = inputs.logreg(n_data=300, dim=4, seed=5)
    m, n, seed = 9, 40, 6
    for J, eps in [(1, 0.1), (10, 0.02)]:
        S, C, _ = gpu_nuts(F, ctx, d, m, n, seed, eps, J)  # default start: N(0, I)
        R, RC, tg = oracle_nuts(d, m, n, seed, eps, J)
        r = check_parity(S, C, R, RC, tg, seed, eps, J, None, first=n)
        assert r["worst"] <= 1e-4 and not r["bad"], J
        assert r["parted"] <= 1, J
        if J == 1:
            assert np.all(C == 1)


def test_nuts_argument_errors(F, ctx):
    d = inputs.logreg(n_data=100, dim=3, seed=1)
    X = torch.tensor(d["X"], dtype=torch.float32, device="cuda")
    y = torch.tensor(d["y"], dtype=torch.float32, device="cuda")
    for sampler, status in [(F.nuts_sampler(0.1, 0), F.EINVAL), (F.nuts_sampler(0.1, 16), F.EINVAL),
                            (F.nuts_sampler(-1.0, 5), F.EINVAL), (F.nuts_sampler(0.1, 5, F.F64), F.ENOTSUP)]:
        with pytest.raises(F.FsmmcError) as e:
            F.Job(ctx, F.logreg_target(X, y), sampler, 4, 4, 1)
        assert e.value.status == status
    Xw = torch.zeros((100, 200), device="cuda")
    with pytest.raises(F.FsmmcError) as e:
        F.Job(ctx, F.logreg_target(Xw, y), F.nuts_sampler(0.1, 5), 4, 4, 1)
    assert e.value.status == F.ENOTSUP


def test_nuts_full_size_fsm_equals_synchronized(F, ctx):
    # 4096 chains x 1000 draws of the N=10000, D=100 workload: the two
    # runtimes write identical bits (compared on the device)
    d = inputs.logreg(n_data=10000, dim=100, seed=3001)
    m, n, seed = 4096, 1000, 3003
    lap = inputs.logreg_laplace(d["X"], d["y"], m, seed=3002)
    a = torch.empty((m, n, 100), dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    _, Ca, sa = gpu_nuts(F, ctx, d, m, n, seed, 0.05, 10, x0=lap["x0"], out=a)
    _, Cb, sb = gpu_nuts(F, ctx, d, m, n, seed, 0.05, 10, x0=lap["x0"], runtime="compact", out=b)
    assert torch.equal(a, b)
    assert np.array_equal(Ca, Cb)
    assert torch.isfinite(a).all()
    print("full size: mean leapfrogs %.2f, max %d, steps %d" % (Ca.mean(), Ca.max(), sa["steps"]))

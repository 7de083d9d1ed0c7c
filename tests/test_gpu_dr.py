"""GPU parity of 3-stage delayed-rejection MH (funnel, Gaussian) through the C ABI."""
import numpy as np
import pytest
import torch

import parity
from oracle import diagnostics as Dg
from oracle import oracle as O

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


def gpu_dr(F, ctx, target, m, n, seed, scales=(1.0, 0.3, 0.1), runtime="fsm", max_steps=0, x0=None,
           out=None):
    x0t = None if x0 is None else torch.tensor(np.asarray(x0), dtype=torch.float32, device="cuda")
    job = F.Job(ctx, target, F.dr_sampler(scales), m, n, seed, x0=x0t, out=out)
    try:
        if runtime == "fsm":
            for _ in range(100000):
                if job.step_fsm(max_steps):
                    break
        else:
            assert job.step_synchronized(n, F.SYNC_VMAP if runtime == "vmap" else F.SYNC_COMPACT)
        if out is not None:
            return None, job.counts(), job.stats()
        return job.samples(), job.counts(), job.stats()
    finally:
        job.free()


def test_dr_fsm_equals_synchronized(F, ctx):
    m, n, seed = 1000, 200, 5
    tgt = F.funnel_target(10)
    ref = gpu_dr(F, ctx, tgt, m, n, seed, runtime="vmap")
    for runtime, steps in [("fsm", 0), ("fsm", 7), ("fsm", 100), ("compact", 0)]:
        S, C, st = gpu_dr(F, ctx, tgt, m, n, seed, runtime=runtime, max_steps=steps)
        assert np.array_equal(S, ref[0]), (runtime, steps)
        assert np.array_equal(C, ref[1]), (runtime, steps)
        assert st["steps"] == C.sum()
    C = ref[1]
    assert set(np.unique(C)) <= {1, 2, 3}
    assert ref[2]["steps"] + ref[2]["padded_steps"] == m * C.max(axis=0).sum()


@pytest.mark.parametrize("kind", ["funnel", "gauss"])
def test_dr_oracle_parity(F, ctx, kind):
    m, n, seed, scales = 64, 100, 9, (1.0, 0.3, 0.1)
    if kind == "funnel":
        tg_gpu, tg = F.funnel_target(10), O.funnel_target(10)
    else:
        prec = np.linspace(0.5, 3.0, 7)
        tg_gpu = F.gauss_target(torch.tensor(prec, dtype=torch.float32, device="cuda"))
        tg = O.gauss_target(prec.astype(np.float32).astype(np.float64))
    S, C, _ = gpu_dr(F, ctx, tg_gpu, m, n, seed, scales)
    R, RC, _ = O.run_chains(tg, O.dr_sampler(scales), seed, range(m), n)
    init = (lambda j: O.funnel_init(10, seed, j)) if kind == "funnel" else (lambda j: O.normal_init(tg.dim, seed, j))
    x_init = np.array([init(j) for j in range(m)])
    r = parity.check_chains(S, C, R, RC, tg, O.dr_sampler(scales), seed, range(m), x_init, first=n)
    print(parity.summary("DR %s" % kind, r))
    assert r["worst"] <= 1e-4
    assert not r["bad"]
    assert r["flip_frac"] <= 0.1


def test_dr_one_stage_and_explicit_start(F, ctx):
    prec = np.array([1.0, 2.0, 0.5])
    tg_gpu = F.gauss_target(torch.tensor(prec, dtype=torch.float32, device="cuda"))
    tg = O.gauss_target(prec)
    x0 = np.random.default_rng(1).standard_normal((33, 3))
    x0 = x0.astype(np.float32).astype(np.float64)
    S, C, _ = gpu_dr(F, ctx, tg_gpu, 33, 80, 4, scales=(0.8,), x0=x0)
    R, RC, _ = O.run_chains(tg, O.dr_sampler((0.8,)), 4, range(33), 80, x0=x0)
    r = parity.check_chains(S, C, R, RC, tg, O.dr_sampler((0.8,)), 4, range(33), x0, first=80)
    assert np.all(C == 1)
    assert r["worst"] <= 1e-4 and not r["bad"] and r["parted"] <= 1


def test_dr_gaussian_moments(F, ctx):
    tg_gpu = F.gauss_target(torch.ones(10, device="cuda"))
    S, C, _ = gpu_dr(F, ctx, tg_gpu, 512, 600, 21)
    b = S[:, 100:, :].astype(np.float64)
    for d in range(10):
        assert abs(b[:, :, d].mean()) < 3 * Dg.mcse_mean(b[:, :, d])
        assert abs(b[:, :, d].var() - 1.0) < 3 * Dg.mcse_var(b[:, :, d])


def test_dr_argument_errors(F, ctx):
    tgt = F.funnel_target(10)
    for scales, status in [((), F.EINVAL), ((1.0, 0.5, 0.2, 0.1), F.EINVAL), ((1.0, -0.3), F.EINVAL)]:
        with pytest.raises(F.FsmmcError) as e:
            F.Job(ctx, tgt, F.dr_sampler(scales), 4, 4, 1)
        assert e.value.status == status
    with pytest.raises(F.FsmmcError) as e:
        F.Job(ctx, F.funnel_target(20), F.dr_sampler(), 4, 4, 1)
    assert e.value.status == F.ENOTSUP
    with pytest.raises(F.FsmmcError) as e:
        F.Job(ctx, tgt, F.dr_sampler(dtype=F.F64), 4, 4, 1)
    assert e.value.status == F.ENOTSUP


def test_dr_funnel_full_size_fsm_equals_synchronized(F, ctx):
    # 65536 chains x 1000 draws of the D = 10 funnel: identical bits on device
    m, n = 65536, 1000
    a = torch.empty((m, n, 10), dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    _, Ca, sa = gpu_dr(F, ctx, F.funnel_target(10), m, n, 4002, out=a)
    _, Cb, sb = gpu_dr(F, ctx, F.funnel_target(10), m, n, 4002, runtime="vmap", out=b)
    assert torch.equal(a, b) and np.array_equal(Ca, Cb)
    assert torch.isfinite(a).all()

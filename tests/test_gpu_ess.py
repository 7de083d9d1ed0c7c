"""GPU parity of elliptical slice sampling through the C ABI.

* FSM runtime == synchronized runtime, bit for bit, per chain (the FSM
  changes the schedule, not the draws: Sec. 1, Sec. 3.2).
* GPU vs the FP64 oracle per draw: 1e-4 relative in FP32 over the first
  100 draws (1e-10 in FP64) up to the first flip; every flip a near-tie.
* Schedule independence: window sizes, step budgets and chunking give the
  same bits.
"""
import numpy as np
import pytest
import torch

import parity
from oracle import diagnostics as Dg
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


def _dev(a, dtype):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda")


def gpu_ess(F, ctx, w, m, n, seed, fp64=False, noise_sd=None, runtime="fsm", window=0,
            max_steps=0, x0=None):
    dt = torch.float64 if fp64 else torch.float32
    L, y = _dev(w["L"], dt), _dev(w["y"], dt)
    x0t = None if x0 is None else _dev(x0, dt)
    job = F.Job(ctx, F.gp_target(L, y, noise_sd), F.ess_sampler(F.F64 if fp64 else F.F32), m, n,
                seed, x0=x0t, window=window)
    try:
        if runtime == "fsm":
            for _ in range(100000):
                if job.step_fsm(max_steps):
                    break
        else:
            mode = F.SYNC_VMAP if runtime == "vmap" else F.SYNC_COMPACT
            assert job.step_synchronized(n, mode)
        return job.samples(), job.counts(), job.stats()
    finally:
        job.free()


def oracle_ess(w, m, n, seed, noise_sd=None, x0=None):
    tg = O.gp_target(w["y"], noise_sd=noise_sd)
    draws, counts, guards = O.run_chains(tg, O.ess_sampler(w["L"]), seed, range(m), n, x0=x0)
    assert guards == 0
    return draws, counts, tg


def ess_parity(w, S, C, R, RC, seed, chains, noise_sd=None, x0=None, first=100, tol=1e-4):
    """Per-draw comparison with the oracle; partings must be near-tie flips
    at the decision where the two runs part."""
    tg = O.gp_target(w["y"], noise_sd=noise_sd)
    chains = list(chains)
    x_init = x0 if x0 is not None else np.array([O.ess_init(w["L"], seed, int(j)) for j in chains])
    return parity.check_chains(S, C, R, RC, tg, O.ess_sampler(w["L"]), seed, chains, x_init,
                               first=first, tol=tol)


def test_ess_fp64_d16_oracle_parity(F, ctx):
    w = inputs.gp_gauss(dim=16, lengthscale=0.2, jitter=1e-6, noise_sd=0.1, seed=1001)
    S, C, st = gpu_ess(F, ctx, w, 64, 100, 1002, fp64=True, noise_sd=0.1)
    R, RC, _ = oracle_ess(w, 64, 100, 1002, noise_sd=0.1)
    r = ess_parity(w, S, C, R, RC, 1002, range(64), noise_sd=0.1, tol=1e-10)
    print(parity.summary("fp64 d16", r))
    assert r["parted"] == 0
    assert r["worst"] <= 1e-10
    assert st["guard_trips"] == 0 and st["chains_done"] == 64


def test_ess_fp64_d16_closed_form(F, ctx):
    # the GPU chains of the pinned oracle run reproduce the closed-form posterior
    w = inputs.gp_gauss(dim=16, lengthscale=0.2, jitter=1e-6, noise_sd=0.1, seed=1001)
    S, C, _ = gpu_ess(F, ctx, w, 64, 4000, 1002, fp64=True, noise_sd=0.1)
    K, y = w["K"], w["y"]
    A = np.linalg.solve(K + 0.01 * np.eye(16), np.eye(16))
    mu, Sig = K @ A @ y, K - K @ A @ K
    b = S[:, 400:, :]
    for d in range(16):
        assert abs(b[:, :, d].mean() - mu[d]) < 3 * Dg.mcse_mean(b[:, :, d])
        assert abs(b[:, :, d].var() - Sig[d, d]) < 3 * Dg.mcse_var(b[:, :, d])


@pytest.mark.parametrize("fp64", [True, False])
def test_ess_fsm_equals_synchronized(F, ctx, fp64):
    if fp64:
        w = inputs.gp_gauss(dim=16, seed=1001)
        kw = dict(noise_sd=0.1, fp64=True)
    else:
        w = inputs.gp_logistic(dim=300, lengthscale=0.05, jitter=1e-5, seed=77)
        kw = {}
    m, n = 258, 150
    ref = gpu_ess(F, ctx, w, m, n, 5, runtime="vmap", **kw)
    for runtime, window, steps in [("fsm", 0, 0), ("fsm", 1, 0), ("fsm", 7, 5), ("fsm", 64, 13),
                                   ("compact", 0, 0)]:
        S, C, st = gpu_ess(F, ctx, w, m, n, 5, runtime=runtime, window=window, max_steps=steps, **kw)
        assert np.array_equal(S, ref[0]), (runtime, window, steps)
        assert np.array_equal(C, ref[1]), (runtime, window, steps)
        assert st["steps"] == C.sum()
    # the vmap baseline ran max_j N_ij bodies for every chain and draw
    C = ref[1]
    assert ref[2]["steps"] + ref[2]["padded_steps"] == m * C.max(axis=0).sum()


def test_ess_fp32_d1024_oracle_parity(F, ctx):
    w = inputs.gp_logistic(dim=1024, lengthscale=0.05, jitter=1e-5, seed=2001)
    m, n, seed = 64, 100, 2002
    S, C, st = gpu_ess(F, ctx, w, m, n, seed)
    R, RC, tg = oracle_ess(w, m, n, seed)
    r = ess_parity(w, S, C, R, RC, seed, range(m))
    print(parity.summary("fp32 d1024", r))
    assert r["worst"] <= 1e-4
    assert not r["bad"]
    assert r["flip_frac"] <= 0.1


@pytest.mark.parametrize("D", [300, 700, 1024])
def test_ess_first_draw_has_fp32_accuracy(F, ctx, D):
    """At Dp > 256 the prior and direction products run on the bf16 matrix
    cores from exact three-piece splits (six piece products per FP32
    product).  The first draw, x0 cos(theta) + nu sin(theta) with x0 and nu
    both from that product, must match the FP64 oracle to FP32 rounding:
    2^-24 per operation, grown by sqrt(D) <= 32 over the D-term sums and by
    the FP32 normals, gives about 1e-6; the bound is 1e-5, while a product
    from single bf16 operands (8-bit significands) would be off by ~1e-3."""
    w = inputs.gp_logistic(dim=D, lengthscale=0.05, jitter=1e-5, seed=2001)
    m, n, seed = 64, 1, 2003
    S, C, _ = gpu_ess(F, ctx, w, m, n, seed)
    R, RC, _ = oracle_ess(w, m, n, seed)
    same = C[:, 0] == RC[:, 0]
    assert same.sum() >= m // 2
    a = S[same, 0].astype(np.float64)
    b = R[same, 0]
    err = np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)
    print("D=%d first draw: max rel err %.3g, mean %.3g over %d chains" % (D, err.max(), err.mean(), int(same.sum())))
    assert err.max() <= 1e-5


def test_ess_c2_full_size_sampled_chains_oracle_parity(F, ctx):
    """The benchmark's job itself (8192 chains x 2000 draws, D = 1024, default
    window, pipelined GEMM): sampled chains against the oracle run for those
    chain indices alone, over their first 100 draws; flips must be near-ties."""
    w = inputs.gp_logistic(dim=1024, lengthscale=0.05, jitter=1e-5, seed=2001)
    m, n, D, seed, first = 8192, 2000, 1024, 2002, 100
    out = torch.empty((m, n, D), dtype=torch.float32, device="cuda")
    job = F.Job(ctx, F.gp_target(_dev(w["L"], torch.float32), _dev(w["y"], torch.float32)),
                F.ess_sampler(F.F32), m, n, seed, out=out)
    try:
        assert job.step_fsm(0)
        C = job.counts()
        st = job.stats()
    finally:
        job.free()
    idx = [0, 1, 4095, 4096, 8191] + sorted(int(i) for i in np.random.default_rng(11).choice(m, 5, replace=False))
    S = out[idx, :first].cpu().numpy()
    del out
    torch.cuda.empty_cache()
    assert st["chains_done"] == m and st["guard_trips"] == 0 and st["draws"] == m * n
    tg = O.gp_target(w["y"])
    R, RC, guards = O.run_chains(tg, O.ess_sampler(w["L"]), seed, idx, first)
    assert guards == 0
    r = ess_parity(w, S, C[idx], R, RC, seed, idx, first=first)
    print(parity.summary("C2 full size, chains %s" % idx, r))
    assert r["worst"] <= 1e-4 and not r["bad"]
    assert r["parted"] <= 2


@pytest.mark.parametrize("D", [1, 17, 64, 100, 128, 333, 700, 769, 1000])
def test_ess_ragged_dims_oracle_parity(F, ctx, D):
    # 64 and 128 fill the lanes (the mask-free kernels at one and two
    # elements per lane); the others leave a ragged last element
    w = inputs.gp_logistic(dim=D, lengthscale=0.1, jitter=1e-5, seed=D)
    m, n = 37, 40
    S, C, _ = gpu_ess(F, ctx, w, m, n, 9)
    R, RC, _ = oracle_ess(w, m, n, 9)
    r = ess_parity(w, S, C, R, RC, 9, range(m), first=n)
    print(parity.summary("D=%d" % D, r))
    assert r["worst"] <= 1e-4, D
    assert not r["bad"] and r["parted"] <= 2


def test_ess_explicit_x0(F, ctx):
    w = inputs.gp_logistic(dim=64, lengthscale=0.1, seed=3)
    x0 = np.random.default_rng(0).standard_normal((12, 64)) * 0.5
    S, C, _ = gpu_ess(F, ctx, w, 12, 30, 4, x0=x0)
    R, RC, _ = oracle_ess(w, 12, 30, 4, x0=x0)
    r = ess_parity(w, S, C, R, RC, 4, range(12), x0=x0, first=30)
    assert r["worst"] <= 1e-4 and r["parted"] == 0


@pytest.mark.parametrize("fp64", [True, False])
def test_ess_pipelined_windows_equal_sequential(F, ctx, fp64):
    # step_fsm(0) overlaps the next window's ellipse GEMM with the current
    # window; a finite budget takes the sequential path.  Many small windows.
    w = inputs.gp_gauss(dim=40, lengthscale=0.2, jitter=1e-6, noise_sd=0.1, seed=77) if fp64 else \
        inputs.gp_logistic(dim=200, lengthscale=0.05, jitter=1e-5, seed=78)
    noise = 0.1 if fp64 else None
    a = gpu_ess(F, ctx, w, 33, 61, 9, fp64=fp64, noise_sd=noise, window=4)
    b = gpu_ess(F, ctx, w, 33, 61, 9, fp64=fp64, noise_sd=noise, window=4, max_steps=10 ** 9)
    c = gpu_ess(F, ctx, w, 33, 61, 9, fp64=fp64, noise_sd=noise, window=4, runtime="compact")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert np.array_equal(a[0], c[0]) and np.array_equal(a[1], c[1])
    # draws use distinct ellipse directions: no two draws of a chain repeat a proposal step
    R, RC, _ = oracle_ess(w, 4, 61, 9, noise_sd=noise)
    r = ess_parity(w, a[0][:4], a[1][:4], R, RC, 9, range(4), noise_sd=noise, first=61,
                   tol=1e-10 if fp64 else 1e-4)
    assert r["worst"] <= (1e-10 if fp64 else 1e-4) and not r["bad"]


def test_ess_step_budget_semantics(F, ctx):
    w = inputs.gp_logistic(dim=128, lengthscale=0.1, seed=5)
    L, y = _dev(w["L"], torch.float32), _dev(w["y"], torch.float32)
    job = F.Job(ctx, F.gp_target(L, y), F.ess_sampler(F.F32), 40, 500, 11)
    try:
        assert not job.step_fsm(3)
        assert job.stats()["steps"] == 3 * 40
        assert not job.step_fsm(4)
        assert job.stats()["steps"] == 7 * 40
        prog = job.progress()
        assert prog.max() <= 7
        with pytest.raises(F.FsmmcError):
            job.samples(0, 400)  # not produced yet
        while not job.step_fsm(0):
            pass
        assert job.stats()["chains_done"] == 40
    finally:
        job.free()


def test_ess_argument_errors(F, ctx):
    w = inputs.gp_logistic(dim=8, seed=1)
    L, y = _dev(w["L"], torch.float32), _dev(w["y"], torch.float32)
    tgt = F.gp_target(L, y)
    with pytest.raises(F.FsmmcError) as e:
        F.Job(ctx, tgt, F.ess_sampler(F.F32), 0, 10, 1)
    assert e.value.status == F.EINVAL
    big = torch.zeros((2000, 2000), device="cuda")
    with pytest.raises(F.FsmmcError) as e:
        F.Job(ctx, F.gp_target(big, torch.zeros(2000, device="cuda")), F.ess_sampler(F.F32), 4, 4, 1)
    assert e.value.status == F.ENOTSUP
    small = F.Context(0, hbm_budget_bytes=1 << 20)
    try:
        with pytest.raises(F.FsmmcError) as e:
            F.Job(small, tgt, F.ess_sampler(F.F32), 4096, 1000, 1)
        assert e.value.status == F.EBUDGET
        assert small.bytes_in_use() == 0
    finally:
        small.close()

"""GPU parity of symmetric delayed rejection (Mira 2001; Sec. 7.1) through the
C ABI: the condensed FSM (one state per try), the split FSM (the loop body as
four states) and the synchronized runtime give the same bits, and the draws
match the FP64 oracle per draw (1e-4 relative; a parting must be the
oracle's draw with one near-tie decision inverted)."""
import numpy as np
import pytest
import torch

import parity
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


def gauss(F, prec):
    return F.gauss_target(torch.tensor(np.asarray(prec, dtype=np.float32), device="cuda"))


def run(F, ctx, target, m, n, seed, M, sigma, runtime="fsm", max_steps=0, states=1):
    job = F.Job(ctx, target, F.drsym_sampler(M, sigma), m, n, seed, fsm_states=states)
    try:
        if runtime == "fsm":
            for _ in range(1000000):
                if job.step_fsm(max_steps):
                    break
        else:
            assert job.step_synchronized(n, F.SYNC_VMAP if runtime == "vmap" else F.SYNC_COMPACT)
        return job.samples(), job.counts(), job.stats()
    finally:
        job.free()


def test_drsym_runtimes_bit_exact(F, ctx):
    tg = gauss(F, [1.0])
    m, n, seed, M, sigma = 300, 200, 31, 100, 0.1
    ref = run(F, ctx, tg, m, n, seed, M, sigma, runtime="vmap")
    S0, C0, st0 = ref
    for runtime, steps, states in [("fsm", 0, 1), ("fsm", 0, 4), ("fsm", 7, 4), ("fsm", 333, 1),
                                   ("compact", 0, 1)]:
        S, C, st = run(F, ctx, tg, m, n, seed, M, sigma, runtime, steps, states)
        assert np.array_equal(S, S0), (runtime, steps, states)
        assert np.array_equal(C, C0), (runtime, steps, states)
        want = C.sum() * (4 if (runtime == "fsm" and states == 4) else 1)
        assert st["steps"] == want, (runtime, steps, states)
    assert st0["steps"] + st0["padded_steps"] == m * C0.max(axis=0).sum()
    assert C0.min() >= 1 and C0.max() <= M
    # lane occupancy: useful lane-iterations and 64 slots per wave iteration
    assert st0["active_lanes"] == C0.sum()
    assert st0["lane_slots"] >= st0["active_lanes"] and st0["lane_slots"] % 64 == 0
    print("DRSYM N(0,1) M=100 sigma=0.1: mean tries %.2f, mean max over %d chains %.1f, R %.2f"
          % (C0.mean(), m, C0.max(axis=0).mean(), st0["r_hat"]))


@pytest.mark.parametrize("kind,D,M,sigma", [("gauss", 1, 100, 0.1), ("gauss", 3, 6, 1.5), ("funnel", 10, 5, 0.5)])
def test_drsym_oracle_parity(F, ctx, kind, D, M, sigma):
    m, n, seed = 64, 100, 41 + D
    if kind == "gauss":
        prec = np.linspace(0.5, 2.0, D).astype(np.float32) if D > 1 else np.ones(1, np.float32)
        tg, otg = gauss(F, prec), O.gauss_target(prec.astype(np.float64))
        x_init = np.array([O.normal_init(D, seed, j) for j in range(m)])
    else:
        tg, otg = F.funnel_target(D), O.funnel_target(D)
        x_init = np.array([O.funnel_init(D, seed, j) for j in range(m)])
    S, C, _ = run(F, ctx, tg, m, n, seed, M, sigma, states=4)
    R, RC, _ = O.run_chains(otg, O.drsym_sampler(M, sigma), seed, range(m), n)
    r = parity.check_chains(S, C, R, RC, otg, O.drsym_sampler(M, sigma), seed, range(m), x_init, first=n)
    print(parity.summary("DRSYM %s D=%d M=%d" % (kind, D, M), r))
    assert r["worst"] <= 1e-4 and not r["bad"]
    assert r["flip_frac"] <= 0.1


def test_drsym_argument_errors(F, ctx):
    tg = gauss(F, [1.0])
    with pytest.raises(F.FsmmcError) as e:
        F.Job(ctx, tg, F.drsym_sampler(100, 0.1), 4, 4, 1, fsm_states=3)
    assert e.value.status == F.EINVAL
    for sampler in (F.drsym_sampler(0, 0.1), F.drsym_sampler(10, -1.0)):
        with pytest.raises(F.FsmmcError) as e:
            F.Job(ctx, tg, sampler, 4, 4, 1)
        assert e.value.status == F.EINVAL
    job = F.Job(ctx, tg, F.drsym_sampler(100, 0.1), 4, 4, 1, fsm_states=4)
    try:
        # mid-try (split sub-state pending): not at a draw boundary
        job.step_fsm(2)
        with pytest.raises(F.FsmmcError) as e:
            job.step_synchronized(1)
        assert e.value.status == F.EINVAL
    finally:
        job.free()

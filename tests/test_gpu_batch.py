"""GPU tests of the batch runtime (several jobs, one graph replay per round).

Every job's draws and loop counts in a batch must equal, bit for bit, the
same job run alone with step_fsm: chains are keyed by (seed, chain, draw),
so the mix, the queue order and the tuning never change a draw.
"""
import numpy as np
import pytest
import torch

import parity
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


# (dim, chains, draws, data seed, chain seed): one ESS job per elements-per-lane class
ESS_MIX = [(64, 40, 50, 11, 101), (100, 33, 70, 12, 102), (200, 20, 45, 13, 103), (300, 17, 60, 14, 104),
           (450, 9, 30, 15, 105), (700, 6, 25, 16, 106), (1000, 5, 20, 17, 107)]
# (target, dim, chains, draws, seed): DRMH jobs of the 4-, 8- and 12-wide lane classes
DR_MIX = [("funnel", 10, 300, 50, 201), ("gauss", 3, 70, 40, 202), ("gauss", 7, 65, 33, 203)]


def _dev(a):
    return torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda")


def make_jobs(F, ctx, ess_mix=ESS_MIX, dr_mix=DR_MIX, outs=None):
    jobs = []
    for i, (D, m, n, ds, cs) in enumerate(ess_mix):
        w = inputs.gp_logistic(dim=D, lengthscale=0.05, jitter=1e-5, seed=ds)
        out = None if outs is None else outs[i]
        jobs.append(F.Job(ctx, F.gp_target(_dev(w["L"]), _dev(w["y"])), F.ess_sampler(), m, n, cs, out=out))
    for i, (kind, D, m, n, seed) in enumerate(dr_mix):
        tgt = F.funnel_target(D) if kind == "funnel" else F.gauss_target(
            torch.linspace(0.5, 2.0, D, device="cuda"))
        out = None if outs is None else outs[len(ess_mix) + i]
        jobs.append(F.Job(ctx, tgt, F.dr_sampler(), m, n, seed, out=out))
    return jobs


def results(jobs):
    return [(j.samples(), j.counts()) for j in jobs]


def alone(F, ctx, ess_mix=ESS_MIX, dr_mix=DR_MIX):
    jobs = make_jobs(F, ctx, ess_mix, dr_mix)
    try:
        for j in jobs:
            while not j.step_fsm(0):
                pass
        return results(jobs)
    finally:
        for j in jobs:
            j.free()


def batched(F, ctx, ess_mix=ESS_MIX, dr_mix=DR_MIX, max_rounds=0, pre_steps=0, **tune):
    jobs = make_jobs(F, ctx, ess_mix, dr_mix)
    try:
        if pre_steps:
            for j in jobs:
                j.step_fsm(pre_steps)
        b = F.Batch(ctx, jobs, **tune)
        try:
            for _ in range(100000):
                if b.run(max_rounds):
                    break
            st = b.stats()
        finally:
            b.free()
        return results(jobs), st
    finally:
        for j in jobs:
            j.free()


def assert_same(got, ref):
    assert len(got) == len(ref)
    for k, ((S, C), (R, RC)) in enumerate(zip(got, ref)):
        assert np.array_equal(C, RC), "job %d counts" % k
        assert np.array_equal(S, R), "job %d draws" % k


@pytest.fixture(scope="module")
def reference(F, ctx):
    return alone(F, ctx)


def test_batch_equals_alone(F, ctx, reference):
    got, st = batched(F, ctx, window=8, dr_chunk=5, rounds_per_sync=2)
    assert_same(got, reference)
    assert st["draws"] == sum(m * n for _, m, n, _, _ in ESS_MIX) + sum(m * n for _, _, m, n, _ in DR_MIX)
    assert st["live_jobs"] == 0 and st["window"] == 8 and st["dr_chunk"] == 5
    assert st["captures"] >= 2  # recaptured as jobs finished


@pytest.mark.parametrize("tune", [dict(autotune=True), dict(window=64, dr_chunk=64, gemm_cols=128),
                                  dict(window=1, dr_chunk=1, rounds_per_sync=7)])
def test_batch_tuning_never_changes_draws(F, ctx, reference, tune):
    got, st = batched(F, ctx, **tune)
    assert_same(got, reference)
    if tune.get("autotune"):
        assert st["tune_trials"] >= 3
        print("autotuned: window %d, dr_chunk %d, gemm_cols %d after %d trials"
              % (st["window"], st["dr_chunk"], st["gemm_cols"], st["tune_trials"]))


def test_batch_round_by_round_and_mid_draw_start(F, ctx, reference):
    # one round per call, starting from chains left mid-draw by a step budget
    got, _ = batched(F, ctx, max_rounds=1, pre_steps=3, window=4, dr_chunk=3)
    assert_same(got, reference)


NUTS_MIX = [(700, 20, 30, 30, 31, 502, 0.05), (1500, 90, 20, 25, 32, 505, 0.03)]


def nuts_jobs(F, ctx, mix):
    jobs = []
    for N, D, m, n, ds, cs, eps in mix:
        w = inputs.logreg(n_data=N, dim=D, seed=ds)
        x0 = inputs.logreg_laplace(w["X"], w["y"], m, seed=ds + 7)["x0"]
        jobs.append(F.Job(ctx, F.logreg_target(_dev(w["X"]), _dev(w["y"])), F.nuts_sampler(eps), m, n, cs,
                          x0=_dev(x0)))
    return jobs


def test_batch_with_nuts_jobs(F, ctx, reference):
    ref_n = []
    for j in nuts_jobs(F, ctx, NUTS_MIX):
        while not j.step_fsm(0):
            pass
        ref_n.append((j.samples(), j.counts()))
        j.free()
    jobs = make_jobs(F, ctx) + nuts_jobs(F, ctx, NUTS_MIX)
    try:
        b = F.Batch(ctx, jobs, window=8, dr_chunk=8, nuts_steps=5, autotune=True)
        assert b.run(0)
        b.free()
        assert_same(results(jobs), reference + ref_n)
    finally:
        for j in jobs:
            j.free()


def test_batch_mix_oracle_parity(F, ctx):
    """ESS, DR and NUTS jobs batched together (autotuned): sampled chains of
    every job against the FP64 oracle over their first 40 draws (1e-4
    relative; a parting must be the oracle's draw with one near-tie decision
    inverted)."""
    specs = ([("ess",) + e for e in ESS_MIX] + [("dr",) + d for d in DR_MIX]
             + [("nuts",) + x for x in NUTS_MIX])
    jobs = make_jobs(F, ctx) + nuts_jobs(F, ctx, NUTS_MIX)
    try:
        b = F.Batch(ctx, jobs, window=8, dr_chunk=8, nuts_steps=5, autotune=True)
        assert b.run(0)
        b.free()
        res = results(jobs)
    finally:
        for j in jobs:
            j.free()
    parted = compared = 0
    for k, (spec, (S, C)) in enumerate(zip(specs, res)):
        chains = parity.sample_chains(S.shape[0], 4, 100 + k)
        r = parity.check_job(spec, S, C, chains, first=40)
        print(parity.summary("batched job %d %s" % (k, spec[:3]), r))
        assert r["worst"] <= 1e-4 and not r["bad"], (k, spec)
        parted += r["parted"]
        compared += len(chains)
    assert parted <= compared // 10


def test_batch_wide_drmh(F, ctx):
    mix = [("gauss", 16, 64, 20, 301), ("funnel", 13, 100, 30, 302)]
    ref = alone(F, ctx, ess_mix=ESS_MIX[:2], dr_mix=mix)
    got, _ = batched(F, ctx, ess_mix=ESS_MIX[:2], dr_mix=mix, window=16, dr_chunk=8)
    assert_same(got, ref)


def test_batch_ownership_and_errors(F, ctx):
    jobs = make_jobs(F, ctx, ESS_MIX[:1], DR_MIX[:1])
    w = inputs.gp_gauss(dim=16)
    f64 = F.Job(ctx, F.gp_target(torch.tensor(w["L"], device="cuda"), torch.tensor(w["y"], device="cuda"),
                                 noise_sd=0.1), F.ess_sampler(F.F64), 4, 4, 1)
    try:
        with pytest.raises(F.FsmmcError) as e:
            F.Batch(ctx, [jobs[0], f64])
        assert e.value.status == F.ENOTSUP
        with pytest.raises(F.FsmmcError) as e:
            F.Batch(ctx, [jobs[0], jobs[0]])
        assert e.value.status == F.EINVAL
        with pytest.raises(F.FsmmcError) as e:
            F.Batch(ctx, jobs, gemm_cols=96)
        assert e.value.status == F.EINVAL
        b = F.Batch(ctx, jobs)
        try:
            with pytest.raises(F.FsmmcError) as e:
                F.Batch(ctx, jobs[:1])
            assert e.value.status == F.EBUSY
            done = torch.zeros(1, dtype=torch.int32, device="cuda")
            for call in (lambda: jobs[0].step_fsm(0), lambda: jobs[1].step_synchronized(1),
                         lambda: jobs[0].step_fsm_async(0, done), lambda: F.fsmmc_job_free(jobs[0].handle)):
                with pytest.raises(F.FsmmcError) as e:
                    call()
                assert e.value.status == F.EBUSY
            assert not b.run(max_rounds=1)
        finally:
            b.free()
        # free-standing again: finish alone, same bits as a plain alone run
        for j in jobs:
            while not j.step_fsm(0):
                pass
        assert_same(results(jobs), alone(F, ctx, ESS_MIX[:1], DR_MIX[:1]))
    finally:
        f64.free()
        for j in jobs:
            j.free()


def _checksum(t):
    v = t.view(torch.int32)
    return int(v.sum(dtype=torch.int64)), int(v.view(-1)[::7].sum(dtype=torch.int64))


def test_batch_uneven_full_size(F, ctx):
    """32 GP-logistic ESS targets of uneven dim / chains / draws plus the 65536-chain
    D=10 funnel, autotuned: every job's draws equal its alone run (checksums of the
    bits) and its loop counts match exactly."""
    spec = inputs.ess_uneven_targets()
    ess_mix = [(s["dim"], s["n_chains"], s["n_draws"], s["data_seed"], s["chain_seed"]) for s in spec]
    dr_mix = [("funnel", 10, 65536, 1000, 4002)]
    sizes = [(m, n, D) for D, m, n, _, _ in ess_mix] + [(m, n, D) for _, D, m, n, _ in dr_mix]

    def run(batch):
        sums, counts = [], []
        if batch:
            outs = [torch.empty(s, dtype=torch.float32, device="cuda") for s in sizes]
            jobs = make_jobs(F, ctx, ess_mix, dr_mix, outs=outs)
            b = F.Batch(ctx, jobs, autotune=True)
            assert b.run(0)
            st = b.stats()
            b.free()
            for j, o in zip(jobs, outs):
                sums.append(_checksum(o))
                counts.append(j.counts())
                j.free()
            del outs
            return sums, counts, st
        for k in range(len(sizes)):
            o = torch.empty(sizes[k], dtype=torch.float32, device="cuda")
            e1, d1 = (ess_mix[k:k + 1], []) if k < len(ess_mix) else ([], dr_mix[k - len(ess_mix):][:1])
            (j,) = make_jobs(F, ctx, e1, d1, outs=[o])
            while not j.step_fsm(0):
                pass
            sums.append(_checksum(o))
            counts.append(j.counts())
            j.free()
            del o
        return sums, counts, None

    bs, bc, st = run(True)
    torch.cuda.empty_cache()
    as_, ac, _ = run(False)
    print("C4 batch: %d rounds, %.1f ms on device, window %d, dr_chunk %d, gemm_cols %d"
          % (st["rounds"], st["gpu_ms"], st["window"], st["dr_chunk"], st["gemm_cols"]))
    assert st["draws"] == sum(m * n for m, n, _ in sizes)
    for k in range(len(sizes)):
        assert bs[k] == as_[k], "job %d" % k
        assert np.array_equal(bc[k], ac[k]), "job %d counts" % k

"""fsmmc_step_fsm_async through the C ABI: the FSM runtime queued without
host reads, completion reported by the device into device or pinned host
memory.  Chains meet only at their n-th draw (Sec. 3.2), so the draws must
be the bits fsmmc_step_fsm gives, for every sampler, run to the end in one
call or in budgeted pieces."""
import numpy as np
import pytest
import torch

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


def _t(a, dtype=torch.float32):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda")


def make(F, ctx, kind):
    """A small job of each sampler: (job factory, budget for the pieces)."""
    if kind == "ess":
        w = inputs.gp_logistic(dim=100, seed=31)
        tg, smp, m, n, x0 = F.gp_target(_t(w["L"]), _t(w["y"])), F.ess_sampler(F.F32), 64, 70, None
        piece = 5
    elif kind == "ess64":
        w = inputs.gp_gauss(dim=16, seed=32)
        tg = F.gp_target(_t(w["L"], torch.float64), _t(w["y"], torch.float64), 0.1)
        smp, m, n, x0, piece = F.ess_sampler(F.F64), 40, 50, None, 0
    elif kind == "nuts":
        d = inputs.logreg(n_data=700, dim=12, seed=33)
        lap = inputs.logreg_laplace(d["X"], d["y"], 48, seed=34)
        tg, smp, m, n, x0 = F.logreg_target(_t(d["X"]), _t(d["y"])), F.nuts_sampler(0.05, 8), 48, 25, _t(lap["x0"])
        piece = 40
    elif kind == "mog":
        w = inputs.mog(dim=10, n_chains=32, seed=35)
        tg = F.mog_target(_t(w["means"]), _t(w["log_weights"]), _t(w["prec"]))
        smp, m, n, x0, piece = F.nuts_sampler(0.05, 6), 32, 30, _t(w["x0"]), 0
    elif kind == "gph":
        w = inputs.gp_hyper(n=40, n_chains=16, seed=36)
        tg = F.gp_hyper_target(_t(w["X"], torch.float64), _t(w["y"], torch.float64), w["jitter"])
        smp, m, n, x0, piece = F.ess_sampler(F.F64), 16, 20, _t(w["x0"], torch.float64), 0
    elif kind == "dr":
        tg, smp, m, n, x0, piece = F.funnel_target(10), F.dr_sampler(), 200, 60, None, 0
    elif kind == "drsym":
        tg, smp, m, n, x0, piece = F.gauss_target(torch.ones(10, device="cuda")), F.drsym_sampler(20, 0.1), 200, 40, None, 0
    else:
        tg, smp, m, n, x0, piece = F.funnel_target(10), F.slice_sampler(1.0), 200, 50, None, 0
    return (lambda: F.Job(ctx, tg, smp, m, n, 41, x0=x0)), piece


KINDS = ["ess", "ess64", "nuts", "mog", "gph", "dr", "drsym", "slice"]


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("where", ["device", "pinned"])
def test_async_equals_fsm(F, ctx, kind, where):
    new, piece = make(F, ctx, kind)
    ref = new()
    try:
        assert ref.step_fsm(0)
        S0, C0 = ref.samples(), ref.counts()
    finally:
        ref.free()
    done = torch.full((1,), -1, dtype=torch.int32, device="cuda") if where == "device" else \
        torch.full((1,), -1, dtype=torch.int32).pin_memory()
    job = new()
    try:
        calls = 0
        while True:
            job.step_fsm_async(piece, done)
            job.sync()
            calls += 1
            flag = int(done[0].item())
            assert flag in (0, 1)
            if flag == 1:
                break
            assert piece > 0 and calls < 10000
        S, C = job.samples(), job.counts()
        assert np.array_equal(S, S0) and np.array_equal(C, C0)
        assert (job.progress() >= job.n).all()
        # a further call finds nothing to do and reports done again
        done.fill_(-1)
        job.step_fsm_async(0 if kind != "nuts" else 1, done)
        job.sync()
        assert int(done[0].item()) == 1 and np.array_equal(job.samples(), S0)
    finally:
        job.free()
    if piece > 0:
        assert calls > 1  # the pieces really stopped short of the end


def test_async_budget_stops_where_fsm_does(F, ctx):
    # ESS with a budget: the state after the asynchronous call is the state
    # after the synchronous one (same draw counters)
    new, _ = make(F, ctx, "ess")
    a, b = new(), new()
    try:
        done = torch.zeros(1, dtype=torch.int32, device="cuda")
        assert not a.step_fsm(7)
        b.step_fsm_async(7, done)
        b.sync()
        assert int(done[0].item()) == 0
        assert np.array_equal(a.progress(), b.progress())
    finally:
        a.free()
        b.free()


def test_async_argument_errors(F, ctx):
    new, _ = make(F, ctx, "nuts")
    job = new()
    try:
        with pytest.raises(F.FsmmcError) as e:  # pageable host memory
            job.step_fsm_async(5, torch.zeros(1, dtype=torch.int32))
        assert e.value.status == F.EINVAL
        with pytest.raises(F.FsmmcError) as e:  # NUTS on logistic regression without a budget
            job.step_fsm_async(0, torch.zeros(1, dtype=torch.int32, device="cuda"))
        assert e.value.status == F.EINVAL
    finally:
        job.free()

"""The allocation-free potential evaluation against fsmmc_eval_potential.

Two calls in a row through the C ABI (the second with fewer points, so it
reads a workspace that still holds the first call's larger contents), each
compared bit for bit with the allocating entry point on the same job, and a
request beyond the workspace rejected with EINVAL and the outputs untouched.
"""
import numpy as np
import pytest
import torch

from paper_2503_17405_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    from paper_2503_17405_amd import fsmmc
    return fsmmc


def test_noalloc_potential_matches_allocating_entry_point(F):
    ctx = F.Context(0)
    try:
        d = inputs.logreg(n_data=2000, dim=100, seed=91)
        X = torch.tensor(d["X"], dtype=torch.float32, device="cuda")
        y = torch.tensor(d["y"], dtype=torch.float32, device="cuda")
        m = 300
        job = F.Job(ctx, F.logreg_target(X, y), F.nuts_sampler(0.05, 10), m, 2, 5)
        try:
            rng = np.random.default_rng(92)
            for npts in (m, 37):
                th = torch.tensor(rng.standard_normal((npts, 100)) * 0.3, dtype=torch.float32, device="cuda")
                U_ref, g_ref = job.potential(th)
                g = torch.full((npts, 100), float("nan"), device="cuda")
                U = torch.full((npts,), float("nan"), device="cuda")
                job.potential_noalloc(th, g, U)
                job.sync()
                print("noalloc points=%d max|dU|=%g" % (npts, (U - U_ref).abs().max().item()), flush=True)
                assert torch.equal(U, U_ref), npts
                assert torch.equal(g, g_ref), npts
                # gradient output is optional
                U2 = torch.full((npts,), float("nan"), device="cuda")
                F.fsmmc_eval_potential_noalloc(job.handle, th, None, U2)
                job.sync()
                assert torch.equal(U2, U_ref), npts
        finally:
            job.free()
        # beyond the workspace: n_points * (Dp + 1) * 4 > FSMMC_NOALLOC_SCRATCH_BYTES (Dp = 128 here)
        big = 16300
        job = F.Job(ctx, F.logreg_target(X, y), F.nuts_sampler(0.05, 10), big, 1, 5)
        try:
            th = torch.zeros((big, 100), device="cuda")
            g = torch.full((big, 100), 7.0, device="cuda")
            U = torch.full((big,), 7.0, device="cuda")
            with pytest.raises(F.FsmmcError) as ei:
                job.potential_noalloc(th, g, U)
            assert "workspace" in str(ei.value)
            job.sync()
            assert bool((g == 7.0).all()) and bool((U == 7.0).all())
            # the largest request that fits still runs
            ok = 16256
            U_ref, g_ref = job.potential(th[:ok])
            job.potential_noalloc(th[:ok], g[:ok], U[:ok])
            job.sync()
            assert torch.equal(U[:ok], U_ref) and torch.equal(g[:ok], g_ref)
        finally:
            job.free()
    finally:
        ctx.close()

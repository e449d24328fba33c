"""wmc_solve_noalloc (static device scratch, no allocation) against wmc_solve
on the same inputs and launch shape: bitwise equal, on two calls in a row,
the second with a smaller input, and its size limit rejected on the host."""
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wmc():
    import paper_1903_07189_amd as W
    W.lib()
    return W


def _rand(shape, seed):
    g = torch.Generator(device="cuda:0").manual_seed(seed)
    return torch.rand(shape, device="cuda:0", generator=g)


def test_noalloc_matches_solve(wmc):
    cases = [((2, 300, 517), 11, 0.0, 1), ((1, 64, 100), 7, 0.0, 2), ((3, 41, 70), 2, 0.3, 3)]
    for shape, iters, dt, seed in cases:
        f = _rand(shape, seed)
        lam = torch.linspace(0.5, 2.0, shape[0], device="cuda:0")
        ref = wmc.solve(f, lam, iters, dt=dt)
        out = torch.full_like(f, float("nan"))
        wmc.solve_noalloc(f, lam, iters, out, dt=dt)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (shape, iters)
        # the same with an explicit launch shape and a start state u0 != f
        u0 = _rand(shape, seed + 100)
        tn = {"cols": 1, "tsteps": 4, "seg_rows": 16}
        ref = wmc.solve(f, lam, iters, dt=dt, u0=u0, tuning=tn)
        out2 = torch.full_like(f, float("nan"))
        wmc.solve_noalloc(f, lam, iters, out2, dt=dt, u0=u0, tuning=tn)
        torch.cuda.synchronize()
        assert torch.equal(out2, ref), (shape, iters, "u0")


def test_noalloc_flow_mode_and_single_sweep(wmc):
    u0 = _rand((2, 90, 130), 7)
    ref = wmc.solve(None, iters=5, dt=0.5, u0=u0)
    out = torch.empty_like(u0)
    wmc.solve_noalloc(None, None, 5, out, dt=0.5, u0=u0)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    # one sweep needs no scratch; zero sweeps copy the start state
    f = _rand((1, 33, 47), 8)
    out = torch.empty_like(f)
    wmc.solve_noalloc(f, 1.0, 1, out)
    assert torch.equal(out, wmc.solve(f, 1.0, 1))
    wmc.solve_noalloc(f, 1.0, 0, out)
    assert torch.equal(out, f)


def test_noalloc_rejects_plane_sets_beyond_the_scratch(wmc):
    from paper_1903_07189_amd import wmc as M
    f = torch.zeros((1, 4097, 4096), device="cuda:0")   # 4097*4096*4 B > 64 MiB
    out = torch.empty_like(f)
    with pytest.raises(M.WMCError) as ei:
        wmc.solve_noalloc(f, 1.0, 2, out)
    assert ei.value.code == M.WMC_EINVAL and "scratch" in str(ei.value)
    # the largest plane set that fits runs
    g = _rand((1, 4096, 4096), 9)
    out = torch.empty_like(g)
    wmc.solve_noalloc(g, 1.0, 3, out, tuning={"cols": 2, "tsteps": 3, "seg_rows": 36})
    assert torch.equal(out, wmc.solve(g, 1.0, 3, tuning={"cols": 2, "tsteps": 3, "seg_rows": 36}))
    # checkpoints are not part of this entry point: ckpt is not an argument
    assert len(M.lib().wmc_solve_noalloc.argtypes) == 9

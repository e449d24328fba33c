"""The binding rejects arrays that do not cover the layout they are passed
with, with ValueError and before anything is enqueued: a plane set with fewer
planes than the state (the kernels would read past its end), a checkpoint
buffer from a solve with another period, and mismatched u0 / g_out."""
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wmc():
    import paper_1903_07189_amd as W
    W.lib()
    return W


def _gpu(*shape):
    return torch.rand(shape, device="cuda:0")


def test_step_rejects_f_with_fewer_planes(wmc):
    u, f = _gpu(2, 16, 20), _gpu(1, 16, 20)
    with pytest.raises(ValueError, match="f has shape"):
        wmc.step(u, f, 1.0)


def test_solve_rejects_mismatched_u0(wmc):
    f = _gpu(2, 16, 20)
    for bad in [(1, 16, 20), (2, 15, 20), (2, 16, 21)]:
        with pytest.raises(ValueError, match="u0 has shape"):
            wmc.solve(f, 1.0, 3, u0=_gpu(*bad))
    with pytest.raises(ValueError, match="u0 has shape"):
        wmc.solve_l1(f, 1.0, 0.05, 3, u0=_gpu(1, 16, 20))


def test_backward_rejects_foreign_checkpoints_and_shapes(wmc):
    f = _gpu(2, 16, 20)
    lam = torch.ones(2, device="cuda:0")
    out, ck = wmc.solve(f, lam, 10, ckpt_every=5)      # 2 checkpoint sets
    torch.cuda.synchronize()
    g = torch.ones_like(out)
    with pytest.raises(ValueError, match="ckpt has shape"):
        wmc.backward(g, f, lam, 10, ck, 2)             # period 2 would read 5 sets
    with pytest.raises(ValueError, match="ckpt has shape"):
        wmc.backward(g, f, lam, 10, ck[:, :1].contiguous(), 5)
    with pytest.raises(ValueError, match="g_out has shape"):
        wmc.backward(g[:1], f, lam, 10, ck, 5)
    with pytest.raises(ValueError, match="u0 has shape"):
        wmc.backward(g, f, lam, 10, ck, 5, u0=_gpu(1, 16, 20))
    with pytest.raises(ValueError, match="contiguous"):
        wmc.backward(g, f, lam, 10, ck.transpose(2, 3), 5)
    # the matching call still works
    g_f, _, g_lam = wmc.backward(g, f, lam, 10, ck, 5)
    torch.cuda.synchronize()
    assert torch.isfinite(g_f).all() and torch.isfinite(g_lam).all()

"""The learnable half-window layer of Sec. 4.3 (K learned 3x3 kernels and
the minimum-magnitude activation) on the GPU against the oracle.

Tolerances: each response is a 9-term FP32 dot product of weights |w| <~ 3
and values in [0, 1] (a few ulps of ~10: 1e-5 absolute).  Where two
responses of opposite magnitude order lie within TAU of each other FP32 and
FP64 may select differently; there the GPU's choice must be one of the
near-minimal responses and its value that response.  Gradients are compared
with the GPU's selection replayed by the oracle, norm-wise (FP32
accumulation over up to ~10^5 terms per weight: 2e-5)."""
import numpy as np
import pytest
import torch

import oracle
import wmc_synth

pytestmark = pytest.mark.gpu

TOL = 1e-5
TAU = 4e-5


@pytest.fixture(scope="module")
def wmc():
    import paper_1903_07189_amd as W
    W.lib()
    return W


def to_gpu(a, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).to("cuda:0")


def responses(U, w):
    return np.stack([oracle.layer_forward(U, w[k:k + 1]) for k in range(w.shape[0])])


def check_forward(U, w, out, sel):
    d = responses(U.astype(np.float64), w.astype(np.float64))
    ref_sel = np.argmin(np.abs(d), axis=0)
    mn = np.abs(d).min(axis=0)
    picked = np.take_along_axis(d, sel[None].astype(np.int64), axis=0)[0]
    # the chosen response is (near-)minimal and the output is that response
    assert np.all(np.abs(picked) <= mn + TAU)
    assert np.abs(out - picked).max() <= TOL
    agree = sel == ref_sel
    if not agree.all():  # only at near ties
        assert np.all(np.abs(np.abs(picked) - mn)[~agree] <= TAU)
    return agree.mean()


def test_printed_kernels_reproduce_the_operator(wmc):
    """With the printed kernels times 12 and integer images every value is
    exact: output = 12 H_d bitwise, selection identical (ties included), on
    the oracle and on the GPU operator."""
    from paper_1903_07189_amd.nn import PRINTED_KERNELS_X12
    K12 = np.array(PRINTED_KERNELS_X12, dtype=np.float32)
    rng = np.random.default_rng(41)
    for shape in [(1, 1), (2, 9), (9, 2), (63, 130), (200, 129)]:
        U = rng.integers(-30, 31, size=shape).astype(np.float32)
        out, sel = wmc.layer_forward(to_gpu(U), to_gpu(K12))
        hd, m = oracle.compute(U, return_argmin=True)
        assert np.array_equal(out.cpu().numpy(), (12 * hd).astype(np.float32))
        assert np.array_equal(sel.cpu().numpy(), m.astype(np.uint8))
        # the GPU operator scales by 1/12 in FP32: equal to rounding
        hd_gpu = wmc.compute(to_gpu(U)).cpu().numpy()
        assert np.allclose(12 * hd_gpu, out.cpu().numpy(), rtol=1e-6, atol=1e-5)


@pytest.mark.parametrize("K", [1, 3, 8, 16])
@pytest.mark.parametrize("shape", [(1, 1), (1, 5), (7, 1), (33, 65), (100, 130), (257, 300)])
def test_forward_parity_random_kernels(wmc, K, shape):
    rng = np.random.default_rng(K * 1000 + shape[0] + shape[1])
    U = rng.uniform(0, 1, size=shape).astype(np.float32)
    w = rng.uniform(-1, 1, size=(K, 3, 3)).astype(np.float32)
    out, sel = wmc.layer_forward(to_gpu(U), to_gpu(w))
    check_forward(U, w, out.cpu().numpy(), sel.cpu().numpy())


def test_forward_planes_and_natural_image(wmc):
    noisy, _ = wmc_synth.c3_image(3, 90, 200, 0.1)
    rng = np.random.default_rng(7)
    w = rng.standard_normal((8, 3, 3)).astype(np.float32)
    out, sel = wmc.layer_forward(to_gpu(noisy), to_gpu(w))
    for c in range(3):
        frac = check_forward(noisy[c], w, out[c].cpu().numpy(), sel[c].cpu().numpy())
        assert frac > 0.999


@pytest.mark.parametrize("K", [1, 4, 8, 16])
@pytest.mark.parametrize("shape", [(1, 1), (1, 6), (5, 1), (3, 61), (17, 62), (40, 121),
                                   (129, 250)])
def test_backward_parity(wmc, K, shape):
    rng = np.random.default_rng(K * 7 + shape[0] * 13 + shape[1])
    U = rng.uniform(0, 1, size=(2,) + shape).astype(np.float32)
    w = rng.uniform(-1, 1, size=(K, 3, 3)).astype(np.float32)
    g = rng.standard_normal((2,) + shape).astype(np.float32)
    Ug, wg = to_gpu(U), to_gpu(w)
    out, sel = wmc.layer_forward(Ug, wg)
    g_u, g_w = wmc.layer_backward(Ug, wg, sel, to_gpu(g))
    sel_np = sel.cpu().numpy()
    gw_ref = np.zeros((K, 3, 3))
    for p in range(2):
        gu_ref, gw_p = oracle.layer_backward(U[p], w, sel_np[p].astype(np.int8), g[p])
        gw_ref += gw_p
        err = np.linalg.norm(g_u[p].cpu().numpy() - gu_ref) / max(np.linalg.norm(gu_ref), 1e-30)
        assert err <= 1e-5
    err = np.linalg.norm(g_w.cpu().numpy() - gw_ref) / max(np.linalg.norm(gw_ref), 1e-30)
    assert err <= 2e-5
    # bitwise reproducible
    g_u2, g_w2 = wmc.layer_backward(Ug, wg, sel, to_gpu(g))
    assert torch.equal(g_u, g_u2) and torch.equal(g_w, g_w2)


def test_autograd_function(wmc):
    rng = np.random.default_rng(9)
    U = to_gpu(rng.uniform(0, 1, size=(3, 40, 70)))
    w = to_gpu(rng.uniform(-1, 1, size=(8, 3, 3)))
    u = U.clone().requires_grad_(True)
    wp = w.clone().requires_grad_(True)
    out = wmc.WMCKernelLayer.apply(u, wp)
    g = to_gpu(rng.standard_normal((3, 40, 70)))
    (out * g).sum().backward()
    ref_out, sel = wmc.layer_forward(U, w)
    gu, gw = wmc.layer_backward(U, w, sel, g)
    assert torch.equal(out.detach(), ref_out)
    assert torch.equal(u.grad, gu) and torch.equal(wp.grad, gw)


def test_layer_at_the_benchmark_size(wmc):
    """16 x 512 x 512, K = 8 printed-plus-learned-like kernels (the size the
    benchmark times): every output and the gradients against the oracle."""
    noisy, _ = wmc_synth.c4()
    U = noisy[:, 0]
    rng = np.random.default_rng(12)
    from paper_1903_07189_amd.nn import PRINTED_KERNELS_X12
    w = (np.array(PRINTED_KERNELS_X12, dtype=np.float32) / 12.0
         + 0.05 * rng.standard_normal((8, 3, 3))).astype(np.float32)
    Ug, wg = to_gpu(U), to_gpu(w)
    out, sel = wmc.layer_forward(Ug, wg)
    g = rng.standard_normal(U.shape).astype(np.float32)
    g_u, g_w = wmc.layer_backward(Ug, wg, sel, to_gpu(g))
    out, sel, g_u = out.cpu().numpy(), sel.cpu().numpy(), g_u.cpu().numpy()
    gw_ref = np.zeros((8, 3, 3))
    agree = []
    for p in range(U.shape[0]):
        agree.append(check_forward(U[p], w, out[p], sel[p]))
        gu_ref, gw_p = oracle.layer_backward(U[p], w, sel[p].astype(np.int8), g[p])
        gw_ref += gw_p
        assert np.linalg.norm(g_u[p] - gu_ref) <= 1e-5 * np.linalg.norm(gu_ref)
    assert min(agree) > 0.999
    assert np.linalg.norm(g_w.cpu().numpy() - gw_ref) <= 2e-5 * np.linalg.norm(gw_ref)

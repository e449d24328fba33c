"""Host-side tests of the C ABI: the library loads, exports every function the
header declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wmc.h")


def _declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(wmc[0-9]?_[a-z_0-9]+)\s*\(", txt, re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def wmc():
    from paper_1903_07189_amd import wmc as W
    if not os.path.exists(W.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return W


def test_header_declares_the_boundary():
    names = _declared_functions()
    for want in ["wmc_compute", "wmc_step", "wmc_solve", "wmc_solve_batched", "wmc_backward",
                 "wmc_autotune", "wmc_last_error", "wmc_release"]:
        assert want in names


def test_library_exports_every_declared_symbol(wmc):
    L = wmc.lib()
    for name in _declared_functions():
        assert hasattr(L, name), name
    assert set(_declared_functions()) == set(wmc.EXPORTS)


def test_workspace_queries(wmc):
    L = wmc.lib()
    S = wmc.Shape
    assert L.wmc_solve_workspace(S(1, 4096, 4096, 4096, 4096 * 4096)) == 4096 * 4096 * 4
    assert L.wmc_solve_workspace(S(3, 10, 10, 12, 130)) == 3 * 130 * 4
    assert L.wmc_solve_workspace(S(0, 10, 10, 10, 100)) == 0
    assert L.wmc_set_stride(S(1, 5, 7, 8, 0)) == 4 * 8 + 7
    assert L.wmc_num_checkpoints(20, 5) == 4
    assert L.wmc_num_checkpoints(21, 5) == 5
    assert L.wmc_num_checkpoints(0, 5) == 0
    assert L.wmc_backward_workspace(S(1, 32, 32, 32, 1024), 20, 5) > 0
    assert L.wmc_backward_workspace(S(1, 32, 32, 32, 1024), 20, 0) == 0


def test_workspace_bytes_dispatch(wmc):
    L = wmc.lib()
    S = wmc.Shape(2, 100, 130, 130, 100 * 130)
    assert L.wmc_workspace_bytes(wmc.WMC_OP_SOLVE, S, 0, 0) == L.wmc_solve_workspace(S)
    assert L.wmc_workspace_bytes(wmc.WMC_OP_FD_FLOW, S, 0, 0) == L.wmc_solve_workspace(S)
    assert L.wmc_workspace_bytes(wmc.WMC_OP_SOLVE_L1, S, 0, 0) == L.wmc_l1_workspace(S)
    assert L.wmc_workspace_bytes(wmc.WMC_OP_BACKWARD, S, 20, 5) == L.wmc_backward_workspace(S, 20, 5)
    assert L.wmc_workspace_bytes(wmc.WMC_OP_LAYER_BACKWARD, S, 8, 0) == L.wmc_layer_workspace(S, 8)
    assert L.wmc_layer_workspace(S, 8) > 0 and L.wmc_layer_workspace(S, 17) == 0
    assert L.wmc_workspace_bytes(99, S, 0, 0) == 0
    assert L.wmc_workspace_bytes(wmc.WMC_OP_SOLVE, wmc.Shape(0, 1, 1, 1, 1), 0, 0) == 0


P = ctypes.c_void_p


@pytest.mark.parametrize("shape,msg", [
    ((0, 4, 4, 4, 16), "n, h and w"),
    ((1, 0, 4, 4, 16), "n, h and w"),
    ((1, 4, 4, 3, 16), "ld must be"),
    ((2, 4, 4, 4, 10), "ps must be"),
    ((1, 1 << 30, 4, 4, 16), "2^30"),
])
def test_shape_validation(wmc, shape, msg):
    L = wmc.lib()
    rc = L.wmc_compute(P(4096), P(1 << 20), wmc.Shape(*shape), None)
    assert rc == wmc.WMC_EINVAL
    assert msg in L.wmc_last_error().decode()


def test_step_validation(wmc):
    L = wmc.lib()
    S = wmc.Shape(1, 4, 4, 4, 16)
    assert L.wmc_step(None, None, P(1 << 20), None, 0.0, None, S, None) == wmc.WMC_EINVAL
    # data term without lambda
    assert L.wmc_step(P(4096), P(8192), P(1 << 20), None, 0.0, None, S, None) == wmc.WMC_EINVAL
    assert "lam" in L.wmc_last_error().decode()
    # in-place update is rejected: Jacobi updates read every pixel of U^t
    assert L.wmc_step(P(4096), None, P(4096 + 16), None, 0.0, None, S, None) == wmc.WMC_EINVAL
    assert "overlap" in L.wmc_last_error().decode()
    assert L.wmc_step(P(4096), None, P(1 << 20), None, float("nan"), None, S, None) == wmc.WMC_EINVAL


def test_solve_validation(wmc):
    L = wmc.lib()
    S = wmc.Shape(1, 8, 8, 8, 64)
    # flow mode needs u0
    assert L.wmc_solve(None, None, P(1 << 20), None, 3, 0.0, None, 0, None, P(1 << 21), 1 << 12,
                       S, None) == wmc.WMC_EINVAL
    # negative iterations
    assert L.wmc_solve(P(4096), None, P(1 << 20), P(64), -1, 0.0, None, 0, None, P(1 << 21),
                       1 << 12, S, None) == wmc.WMC_EINVAL
    # workspace too small
    assert L.wmc_solve(P(4096), None, P(1 << 20), P(64), 5, 0.0, None, 0, None, P(1 << 21), 16, S,
                       None) == wmc.WMC_ENOMEM
    # checkpoints without a period
    assert L.wmc_solve(P(4096), None, P(1 << 20), P(64), 5, 0.0, P(1 << 22), 0, None, P(1 << 21),
                       1 << 12, S, None) == wmc.WMC_EINVAL
    # output aliasing the workspace
    assert L.wmc_solve(P(4096), None, P(1 << 20), P(64), 5, 0.0, None, 0, None, P(1 << 20),
                       1 << 12, S, None) == wmc.WMC_EINVAL
    # bad tuning
    t = wmc.Tuning(3, 4, 16, 1)
    assert L.wmc_solve(P(4096), None, P(1 << 20), P(64), 5, 0.0, None, 0, ctypes.byref(t),
                       P(1 << 21), 1 << 12, S, None) in (wmc.WMC_EINVAL, wmc.WMC_EHIP)


def test_solve_tuning_workspace_validation(wmc):
    """wmc_solve_tuning: a workspace of one plane set is accepted (the search
    reads U from f); with room for two sets (the second at the next 256-byte
    offset) the search ping-pongs inside it, so an input overlapping the
    second set is rejected -- and the same input beyond a one-set workspace
    is not."""
    import torch
    L = wmc.lib()
    S = wmc.Shape(1, 64, 64, 64, 4096)
    set_bytes = L.wmc_solve_workspace(S)
    assert set_bytes == 4096 * 4
    lam, ws = P(64), 1 << 24
    t = wmc.Tuning()
    f_in_second_set = ws + set_bytes + 4000
    # two sets: f lies inside the second one
    assert L.wmc_solve_tuning(P(f_in_second_set), None, lam, 0.0, P(ws), 2 * set_bytes + 256, S,
                              ctypes.byref(t), None) == wmc.WMC_EINVAL
    assert "overlaps" in L.wmc_last_error().decode()
    # too small for one set
    assert L.wmc_solve_tuning(P(1 << 20), None, lam, 0.0, P(ws), set_bytes - 4, S,
                              ctypes.byref(t), None) == wmc.WMC_ENOMEM
    if torch.cuda.is_available():
        return
    # one set: the same f is outside it, so validation passes and the call
    # stops at the missing device
    rc = L.wmc_solve_tuning(P(f_in_second_set), None, lam, 0.0, P(ws), set_bytes, S,
                            ctypes.byref(t), None)
    assert rc in (wmc.WMC_EHIP, wmc.WMC_EUNSUPPORTED)


def test_batched_validation(wmc):
    L = wmc.lib()
    imgs = (wmc.Image * 2)()
    imgs[0] = wmc.Image(None, P(4096), P(1 << 20), 8, 8, 8, 64, 1, 0)
    imgs[1] = wmc.Image(P(8192), None, P(1 << 21), 8, 8, 8, 64, 1, 0)  # mixed modes
    assert L.wmc_solve_batched(imgs, 2, P(64), 3, 0.0, None, P(1 << 22), 1 << 16, None) == wmc.WMC_EINVAL
    imgs[1] = wmc.Image(None, P(8192), P(1 << 20), 8, 8, 8, 64, 1, 0)  # outputs overlap
    assert L.wmc_solve_batched(imgs, 2, P(64), 3, 0.0, None, P(1 << 22), 1 << 16, None) == wmc.WMC_EINVAL
    assert L.wmc_batched_workspace(imgs, 2) == 2 * 64 * 4


def test_backward_validation(wmc):
    L = wmc.lib()
    S = wmc.Shape(1, 8, 8, 8, 64)
    assert L.wmc_backward(P(4096), None, P(64), 5, 0.0, None, 2, P(1 << 20), P(1 << 21), None,
                          None, P(1 << 22), 1 << 16, S, None) == wmc.WMC_EINVAL  # no ckpt
    assert L.wmc_backward(P(4096), None, P(64), 5, 0.0, P(1 << 23), 2, P(1 << 20), P(1 << 21),
                          None, None, P(1 << 22), 8, S, None) == wmc.WMC_ENOMEM
    need = L.wmc_backward_workspace(S, 5, 2)
    # g_f and g_u0 must be distinct buffers (the last step writes g_u0, then
    # dL/df adds it)
    assert L.wmc_backward(P(4096), None, P(64), 5, 0.0, P(1 << 23), 2, P(1 << 20), P(1 << 21),
                          P(1 << 21), None, P(1 << 24), need, S, None) == wmc.WMC_EINVAL
    assert "overlap" in L.wmc_last_error().decode()
    # the adjoint kernel takes the row stride as a 32-bit count
    S2 = wmc.Shape(1, 8, 8, 1 << 31, 1 << 34)
    assert L.wmc_backward(P(1 << 40), None, P(64), 5, 0.0, P(1 << 41), 2, P(1 << 42),
                          P(1 << 43), None, None, P(1 << 44), 1 << 30, S2, None) == wmc.WMC_EINVAL
    assert "ld" in L.wmc_last_error().decode()


def test_volume_solve_and_backward_validation(wmc):
    """The 3-D checkpointed solve and the 3-D backward reject bad arguments
    on the host; their workspace queries follow the volume layout."""
    L = wmc.lib()
    S3 = wmc.Shape3
    s = S3(2, 5, 6, 7, 8, 6 * 8, 5 * 6 * 8)
    set3 = 2 * 5 * 6 * 8
    assert L.wmc3_set_stride(s) == set3
    assert L.wmc3_set_stride(S3(1, 5, 6, 7, 8, 6 * 8, 0)) == 4 * 48 + 5 * 8 + 7
    assert L.wmc3_set_stride(S3(0, 5, 6, 7, 8, 48, 240)) == 0
    ws = L.wmc3_backward_workspace(s, 6, 3)
    # two recomputed states, two cotangents, a byte map, lambda partials
    assert ws >= (2 + 2) * set3 * 4 + set3
    assert L.wmc3_backward_workspace(s, 6, 0) == 0
    assert L.wmc3_backward_workspace(s, -1, 2) == 0
    # solve: ckpt_every < 1 with checkpoints, checkpoints overlapping u_out
    assert L.wmc3_solve(P(4096), None, P(1 << 20), P(64), 6, 0.0, P(1 << 22), 0, P(1 << 21),
                        1 << 16, s, None) == wmc.WMC_EINVAL
    assert L.wmc3_solve(P(4096), None, P(1 << 20), P(64), 6, 0.0, P(1 << 20), 3, P(1 << 21),
                        1 << 16, s, None) == wmc.WMC_EINVAL
    # step: the selection map must not overlap the output
    assert L.wmc3_step(P(4096), None, P(1 << 20), None, 0.5, P(1 << 20), s, None) == wmc.WMC_EINVAL
    # backward: no checkpoints, small workspace, overlapping outputs, flow without u0
    assert L.wmc3_backward(P(4096), None, P(64), 5, 0.0, None, 2, P(1 << 20), P(1 << 21), None,
                           None, P(1 << 22), 1 << 24, s, None) == wmc.WMC_EINVAL
    assert L.wmc3_backward(P(4096), None, P(64), 5, 0.0, P(1 << 23), 2, P(1 << 20), P(1 << 21),
                           None, None, P(1 << 22), 8, s, None) == wmc.WMC_ENOMEM
    need = L.wmc3_backward_workspace(s, 5, 2)
    assert L.wmc3_backward(P(4096), None, P(64), 5, 0.0, P(1 << 23), 2, P(1 << 20), P(1 << 21),
                           P(1 << 21), None, P(1 << 24), need, s, None) == wmc.WMC_EINVAL
    assert "overlap" in L.wmc_last_error().decode()
    assert L.wmc3_backward(None, None, None, 5, 0.0, P(1 << 23), 2, P(1 << 20), None, P(1 << 21),
                           None, P(1 << 24), need, s, None) == wmc.WMC_EINVAL
    assert L.wmc3_backward(P(4096), None, None, 5, 0.0, P(1 << 23), 2, P(1 << 20), P(1 << 21),
                           None, None, P(1 << 24), need, s, None) == wmc.WMC_EINVAL


def test_valid_call_without_device_reports_hip_error(wmc):
    """A valid call on a machine without a gfx950 device fails cleanly (no
    crash), with a HIP or unsupported-device status."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    L = wmc.lib()
    rc = L.wmc_compute(P(4096), P(1 << 20), wmc.Shape(1, 4, 4, 4, 16), None)
    assert rc in (wmc.WMC_EHIP, wmc.WMC_EUNSUPPORTED)
    assert L.wmc_last_error()


def test_tall_images_pass_validation(wmc):
    """Images taller than 65535 rows are valid for the solve and the backward
    (their plane copies stride over rows): without a device the calls get past
    validation and fail only at the HIP level."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    L = wmc.lib()
    S = wmc.Shape(1, 70000, 64, 64, 70000 * 64)
    nb = 70000 * 64 * 4
    ws = L.wmc_backward_workspace(S, 6, 3)
    assert ws > 0 and L.wmc_solve_workspace(S) == nb
    rc = L.wmc_solve(P(1 << 32), None, P(1 << 34), P(1 << 36), 6, 0.0, P(1 << 38), 3, None,
                     P(1 << 40), nb, S, None)
    assert rc in (wmc.WMC_EHIP, wmc.WMC_EUNSUPPORTED), L.wmc_last_error()
    rc = L.wmc_backward(P(1 << 32), None, P(1 << 36), 6, 0.0, P(1 << 38), 3, P(1 << 42),
                        P(1 << 44), None, P(1 << 46), P(1 << 48), ws, S, None)
    assert rc in (wmc.WMC_EHIP, wmc.WMC_EUNSUPPORTED), L.wmc_last_error()


def test_fault_injection_paths(wmc, monkeypatch):
    """WMC_FAULT_INJECT makes the library report a HIP failure from host code."""
    L = wmc.lib()
    monkeypatch.setenv("WMC_FAULT_INJECT", "launch")
    rc = L.wmc_compute(P(4096), P(1 << 20), wmc.Shape(1, 4, 4, 4, 16), None)
    assert rc == wmc.WMC_EHIP
    assert "injected" in L.wmc_last_error().decode()


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1903_07189_amd import wmc as W
    monkeypatch.setattr(W, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(W, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        W.lib()


def test_layer_and_fd_validation(wmc):
    L = wmc.lib()
    S = wmc.Shape(1, 8, 8, 8, 64)
    for K in (0, 17):
        assert L.wmc_layer_forward(P(4096), P(8192), K, P(1 << 20), None, S, None) == wmc.WMC_EINVAL
        assert "K must be" in L.wmc_last_error().decode()
    assert L.wmc_layer_forward(None, P(8192), 8, P(1 << 20), None, S, None) == wmc.WMC_EINVAL
    # output aliasing the input
    assert L.wmc_layer_forward(P(4096), P(1 << 22), 8, P(4096 + 8), None, S, None) == wmc.WMC_EINVAL
    # weight gradient without enough workspace
    assert L.wmc_layer_backward(P(4096), P(1 << 22), 8, P(1 << 23), P(1 << 24), None, P(1 << 25),
                                P(1 << 26), 4, S, None) == wmc.WMC_ENOMEM
    # nothing requested: a no-op
    assert L.wmc_layer_backward(P(4096), P(1 << 22), 8, P(1 << 23), P(1 << 24), None, None,
                                None, 0, S, None) == wmc.WMC_OK
    # finite-difference comparator
    assert L.wmc_fd_compute(P(4096), P(1 << 20), -1.0, S, None) == wmc.WMC_EINVAL
    assert L.wmc_fd_flow(P(4096), P(1 << 20), -1, 0.1, 1e-12, None, 0, S, None) == wmc.WMC_EINVAL
    assert L.wmc_fd_flow(P(4096), P(1 << 20), 5, 0.1, 1e-12, P(1 << 21), 8, S, None) == wmc.WMC_ENOMEM


def test_default_checkpoint_period_policy():
    """Every state is kept while K plane sets fit the budget, else ceil(sqrt(K))."""
    from paper_1903_07189_amd import wmc as W
    set_c4 = 16 * 512 * 512 * 4
    assert W.default_ckpt_every(20, set_c4) == 1
    assert W.default_ckpt_every(30, 32 * 256 * 256 * 4) == 1
    big = 4096 * 4096 * 4
    assert W.default_ckpt_every(200, big) == 15
    assert W.default_ckpt_every(1, big) == 1
    budget = W.KEEP_ALL_STATES_BYTES
    assert W.default_ckpt_every(4, budget // 4) == 1
    assert W.default_ckpt_every(4, budget // 4 + 1) == 2


def test_binding_shape_checks_on_host(wmc):
    """The binding's shape checks (run before any call into the library):
    an array passed with one layout must have exactly that shape, and a
    checkpoint buffer exactly the plane sets its solve stored."""
    import torch
    ref = torch.empty((2, 5, 7))
    wmc.require_shape(None, ref.shape, "u0")
    wmc.require_shape(torch.empty((2, 5, 7)), ref.shape, "u0")
    for bad in [(1, 5, 7), (2, 4, 7), (2, 5, 8), (3, 5, 7)]:
        with pytest.raises(ValueError, match="g_out has shape"):
            wmc.require_shape(torch.empty(bad), ref.shape, "g_out")
    assert wmc.checkpoint_sets(20, 5) == 4
    assert wmc.checkpoint_sets(20, 2) == 10
    assert wmc.checkpoint_sets(21, 5) == 5
    assert wmc.checkpoint_sets(0, 5) == 1       # a solve of 0 steps still returns one set
    with pytest.raises(ValueError):
        wmc.checkpoint_sets(20, 0)


def test_bw_probe_validation(wmc):
    """The bandwidth probe rejects bad arguments on the host, before any HIP
    call."""
    L = wmc.lib()
    A, B, O = P(1 << 40), P(1 << 41), P(1 << 42)
    assert L.wmc_bw_probe(2, A, B, O, 1024, 0, None) == wmc.WMC_EINVAL
    assert L.wmc_bw_probe(0, A, None, O, 1024, 4, None) == wmc.WMC_EINVAL
    assert L.wmc_bw_probe(0, A, None, O, 1022, 0, None) == wmc.WMC_EINVAL
    assert L.wmc_bw_probe(0, A, None, O, 0, 0, None) == wmc.WMC_EINVAL
    assert L.wmc_bw_probe(1, A, None, O, 1024, 0, None) == wmc.WMC_EINVAL
    assert L.wmc_bw_probe(0, P((1 << 40) + 4), None, O, 1024, 0, None) == wmc.WMC_EINVAL
    assert "aligned" in L.wmc_last_error().decode()
    assert L.wmc_bw_probe(1, A, B, P((1 << 40) + 1024), 1024, 1, None) == wmc.WMC_EINVAL
    assert "overlaps" in L.wmc_last_error().decode()

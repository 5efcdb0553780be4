"""C-ABI contract of the compute entry points on a real device (needs
gfx950): every documented error status of drc_cae_forward, _backward,
_step, _set_params and _calibrate_fp8 is returned on the host, before
anything is enqueued (the output buffers keep their sentinel values).

Cases: sizes that are not multiples of 8, n <= 0, misaligned pointers, a
workspace one byte short, calls before drc_cae_set_params, and the
precision / activation forms a call does not implement.
"""
import ctypes

import pytest
import torch

from paper_1910_02480_amd import binding as B
from paper_1910_02480_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
OK, ARG, SHAPE, UNSUP, WS, HIP, STATE = 0, 1, 2, 3, 4, 5, 6


@pytest.fixture(scope="module")
def L():
    return B.lib()


@pytest.fixture(scope="module")
def params():
    return torch.from_numpy(synth.init_params(0)).to(DEV)


def _handle(compute, final_relu=0):
    d = B.drc_cae_default_desc(B.DTYPES[compute])
    d.final_relu = final_relu
    return B.drc_cae_create(d)


def _aligned(nbytes):
    buf = torch.empty(nbytes + 512, dtype=torch.uint8, device=DEV)
    off = (-buf.data_ptr()) % 256
    return buf[off:off + nbytes + 256]


def _ws(h, n, H, W, flags):
    return _aligned(B.drc_cae_workspace_size(h, n, H, W, flags))


def _p(t, byte_off=0):
    return t.data_ptr() + byte_off


def _sentinel(t):
    t.fill_(-7.0)
    torch.cuda.synchronize()


def _untouched(t):
    torch.cuda.synchronize()
    return bool(torch.all(t == -7.0))


@pytest.mark.parametrize("compute", ["f32", "bf16", "fp8"])
def test_forward_contract(L, params, compute):
    h = _handle(compute)
    try:
        n, H, W = 2, 32, 32
        x = torch.from_numpy(synth.radiance_maps(n, H, W)).to(DEV)
        y = torch.empty((n, H, W, 3), device=DEV)
        ws = _ws(h, n, H, W, B.DRC_WS_FORWARD | B.DRC_WS_CALIBRATE)
        need = B.drc_cae_workspace_size(h, n, H, W, B.DRC_WS_FORWARD)
        _sentinel(y)
        fwd = lambda *a: L.drc_cae_forward(h, *a, None)  # noqa: E731
        # before set_params
        assert fwd(_p(x), _p(y), n, H, W, None, _p(ws), ws.numel()) == STATE
        B.drc_cae_set_params(h, params)
        if compute == "fp8":
            assert fwd(_p(x), _p(y), n, H, W, None, _p(ws), ws.numel()) == STATE  # not calibrated
            assert L.drc_cae_calibrate_fp8(h, _p(x), n, 20, W, _p(ws), ws.numel(), None) == SHAPE
            assert L.drc_cae_calibrate_fp8(h, _p(x, 4), n, H, W, _p(ws), ws.numel(), None) == ARG
            assert L.drc_cae_calibrate_fp8(h, _p(x), n, H, W, _p(ws, 16), ws.numel(), None) == ARG
            assert L.drc_cae_calibrate_fp8(h, _p(x), n, H, W, _p(ws), 0, None) == WS
            B.drc_cae_calibrate_fp8(h, x, ws)
        for bad_h, bad_w in ((36, 32), (32, 12), (4, 32), (32, 0)):
            assert fwd(_p(x), _p(y), n, bad_h, bad_w, None, _p(ws), ws.numel()) == SHAPE, (bad_h, bad_w)
        for bad_n in (0, -1):
            assert fwd(_p(x), _p(y), bad_n, H, W, None, _p(ws), ws.numel()) == SHAPE
        assert fwd(None, _p(y), n, H, W, None, _p(ws), ws.numel()) == ARG
        assert fwd(_p(x), None, n, H, W, None, _p(ws), ws.numel()) == ARG
        assert fwd(_p(x, 4), _p(y), n, H, W, None, _p(ws), ws.numel()) == ARG
        assert fwd(_p(x), _p(y, 8), n, H, W, None, _p(ws), ws.numel()) == ARG
        assert fwd(_p(x), _p(y), n, H, W, _p(ws, 16), _p(ws), ws.numel()) == ARG  # d_saved misaligned
        if need > 0:
            assert fwd(_p(x), _p(y), n, H, W, None, _p(ws), need - 1) == WS
            assert fwd(_p(x), _p(y), n, H, W, None, _p(ws, 128), ws.numel()) == ARG
        assert _untouched(y), "a rejected call wrote its output"
        assert fwd(_p(x), _p(y), n, H, W, None, _p(ws), ws.numel()) == OK
        torch.cuda.synchronize()
        assert torch.isfinite(y).all()
    finally:
        B.drc_cae_destroy(h)


@pytest.mark.parametrize("compute", ["f32", "bf16"])
def test_backward_and_step_contract(L, params, compute):
    h = _handle(compute)
    try:
        n, H, W = 2, 32, 32
        x, t = (torch.from_numpy(a).to(DEV) for a in synth.training_batch(n, H))
        dy = torch.full((n, H, W, 3), 1e-3, device=DEV)
        dp = torch.empty(B.drc_cae_num_params(h), device=DEV)
        dx = torch.empty_like(x)
        nbytes, _ = B.drc_cae_saved_size(h, n, H, W)
        saved = _aligned(nbytes)
        ws = _ws(h, n, H, W, B.DRC_WS_BACKWARD | B.DRC_WS_STEP)
        need_b = B.drc_cae_workspace_size(h, n, H, W, B.DRC_WS_BACKWARD)
        need_s = B.drc_cae_workspace_size(h, n, H, W, B.DRC_WS_STEP)
        bwd = lambda *a: L.drc_cae_backward(h, *a, None)  # noqa: E731
        args = lambda **k: [k.get("x", _p(x)), k.get("dy", _p(dy)), k.get("saved", _p(saved)),  # noqa: E731
                            k.get("dp", _p(dp)), k.get("dx", _p(dx)), k.get("n", n), k.get("H", H),
                            k.get("W", W), k.get("ws", _p(ws)), k.get("nb", ws.numel())]
        _sentinel(dp)
        assert bwd(*args()) == STATE  # before set_params
        B.drc_cae_set_params(h, params)
        assert L.drc_cae_set_params(h, None, None) == ARG
        assert L.drc_cae_set_params(h, _p(params, 2), None) == ARG
        assert bwd(*args(H=40, W=36)) == SHAPE
        assert bwd(*args(n=0)) == SHAPE
        assert bwd(*args(x=None)) == ARG
        assert bwd(*args(saved=None)) == ARG
        assert bwd(*args(dp=None)) == ARG
        assert bwd(*args(dy=_p(dy, 4))) == ARG
        assert bwd(*args(dx=_p(dx, 4))) == ARG
        assert bwd(*args(saved=_p(saved, 16))) == ARG
        assert bwd(*args(nb=need_b - 1)) == WS
        assert _untouched(dp)
        # the step
        p = params.clone()
        m, v = torch.zeros_like(p), torch.zeros_like(p)
        loss = torch.full((1,), -7.0, device=DEV)
        adam = B.drc_adam_cfg(6e-5, 0.9, 0.999, 1e-8)
        step = lambda **k: L.drc_cae_step(  # noqa: E731
            h, k.get("p", _p(p)), _p(m), _p(v), k.get("t", 1), ctypes.byref(k.get("adam", adam)),
            k.get("x", _p(x)), _p(t), _p(loss), None, k.get("n", n), H, k.get("W", W), _p(ws),
            k.get("nb", ws.numel()), None)
        assert step(t=0) == ARG
        assert step(adam=B.drc_adam_cfg(0.0, 0.9, 0.999, 1e-8)) == ARG
        assert step(adam=B.drc_adam_cfg(1e-3, 1.0, 0.999, 1e-8)) == ARG
        assert step(n=-3) == SHAPE
        assert step(W=20) == SHAPE
        assert step(x=_p(x, 4)) == ARG
        assert step(p=_p(p, 4)) == ARG
        assert step(nb=need_s - 1) == WS
        assert L.drc_cae_step(h, _p(p), _p(m), _p(v), 1, None, _p(x), _p(t), _p(loss), None, n, H, W, _p(ws),
                              ws.numel(), None) == ARG
        torch.cuda.synchronize()
        assert torch.equal(p, params) and float(loss) == -7.0
        assert step() == OK
        torch.cuda.synchronize()
        assert float(loss) > 0 and not torch.equal(p, params)
        y = torch.empty((n, H, W, 3), device=DEV)
        B.drc_cae_forward(h, x, y, saved, _ws(h, n, H, W, B.DRC_WS_FORWARD))
        assert bwd(*args()) == OK
        torch.cuda.synchronize()
        assert torch.isfinite(dp).all() and torch.isfinite(dx).all()
    finally:
        B.drc_cae_destroy(h)


def test_inference_only_forms_rejected(L, params):
    """FP8 handles and final_relu = 1 are inference only: backward and step
    return DRC_ERR_UNSUPPORTED; calibrate_fp8 on a non-FP8 handle is a call
    order error."""
    n, H, W = 1, 16, 16
    x = torch.from_numpy(synth.radiance_maps(n, H, W)).to(DEV)
    buf = _aligned(1 << 22)
    for compute, fr in (("fp8", 0), ("bf16", 1), ("f32", 1)):
        h = _handle(compute, fr)
        try:
            B.drc_cae_set_params(h, params)
            if compute == "fp8":
                B.drc_cae_calibrate_fp8(h, x, _ws(h, n, H, W, B.DRC_WS_CALIBRATE))
            assert L.drc_cae_backward(h, _p(x), _p(buf), _p(buf), _p(buf), None, n, H, W, _p(buf), buf.numel(),
                                      None) == UNSUP
            adam = B.drc_adam_cfg(6e-5, 0.9, 0.999, 1e-8)
            assert L.drc_cae_step(h, _p(buf), _p(buf), _p(buf), 1, ctypes.byref(adam), _p(x), _p(buf), _p(buf),
                                  None, n, H, W, _p(buf), buf.numel(), None) == UNSUP
            if compute != "fp8":
                assert L.drc_cae_calibrate_fp8(h, _p(x), n, H, W, _p(buf), buf.numel(), None) == STATE
        finally:
            B.drc_cae_destroy(h)
    assert B.drc_last_error()

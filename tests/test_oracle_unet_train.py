"""Pins of the FP64 oracle of the paper's network in training form (Sec. 4.3
and 5): batch-statistics batch normalisation, running-statistics update,
L1 loss and every parameter gradient, against the same network assembled
from PyTorch float64 library layers (conv2d, batch_norm in training mode,
leaky_relu, max_pool2d, bilinear interpolate, cat) and its autograd; the
blocks' backward rules against autograd one by one; and closed forms of
batch norm's gradient (its bias-invariance: a conv bias in front of a
batch-statistics norm gets a zero gradient, and dz sums to zero per
channel)."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import unet as U
from oracle import unet_train as UT
from paper_1910_02480_amd import synth


def _nchw(a):
    return torch.from_numpy(np.ascontiguousarray(np.moveaxis(a, -1, 1)))


def _nhwc(t):
    return np.moveaxis(t.detach().numpy(), 1, -1)


def _torch_train(params, x, t):
    P = [{k: torch.tensor(np.asarray(v, np.float64), requires_grad=k in ("w", "b", "gamma", "beta"))
          for k, v in q.items()} for q in params]
    xt = _nchw(x.astype(np.float64)).requires_grad_(True)
    it = iter(range(len(P)))
    running = []

    def block(h, bn=True):
        q = P[next(it)]
        h = F.conv2d(h, q["w"].permute(0, 3, 1, 2), q["b"], padding=1)
        if bn:
            mean, var = q["mean"].detach().clone(), q["var"].detach().clone()
            h = F.batch_norm(h, mean, var, q["gamma"], q["beta"], training=True, momentum=0.1, eps=1e-5)
            running.append((mean.numpy(), var.numpy()))
        else:
            running.append(None)
        return F.leaky_relu(h, 0.01)

    up = lambda h: F.interpolate(h, scale_factor=2, mode="bilinear", align_corners=False)  # noqa: E731
    s1 = block(block(xt))
    s2 = block(block(F.max_pool2d(s1, 2)))
    s3 = block(block(F.max_pool2d(s2, 2)))
    m = block(block(F.max_pool2d(s3, 2)))
    d3 = block(block(torch.cat([up(m), s3], 1)))
    d2 = block(block(torch.cat([up(d3), s2], 1)))
    d1 = block(block(torch.cat([up(d2), s1], 1), False), False)
    q = P[-1]
    y = F.relu(F.conv2d(d1, q["w"][:, :, None, None], q["b"]))
    loss = F.l1_loss(y, _nchw(t.astype(np.float64)))
    loss.backward()
    return loss.item(), P, _nhwc(y), xt.grad, running


@pytest.mark.parametrize("n,H,W", [(2, 16, 16), (3, 8, 24)])
def test_training_step_matches_torch_autograd(n, H, W):
    params = synth.unet_params(0)
    x, t = synth.training_batch(n, H, W)
    loss, grads, dx, y, running = UT.loss_and_grad(params, x, t)
    lt, P, yt, dxt, rt = _torch_train(params, x, t)
    np.testing.assert_allclose(y, yt, rtol=1e-11, atol=1e-12)
    assert abs(loss - lt) <= 1e-12
    gnorm = np.linalg.norm(UT.flat(grads))
    for k, q in enumerate(P):
        for name in ("w", "b", "gamma", "beta"):
            if name not in q:
                continue
            # absolute, scaled by the whole gradient: the conv bias in front of
            # a batch-statistics norm has an exactly-zero gradient (rounding on both sides)
            np.testing.assert_allclose(grads[k][name], q[name].grad.numpy(), rtol=1e-9, atol=1e-12 * gnorm,
                                       err_msg=f"layer {k} {name}")
    np.testing.assert_allclose(dx, _nhwc(dxt), rtol=1e-9, atol=1e-14)
    for a, b in zip(running, rt):
        assert (a is None) == (b is None)
        if a is not None:
            np.testing.assert_allclose(a[0], b[0], rtol=1e-12, atol=1e-15)
            np.testing.assert_allclose(a[1], b[1], rtol=1e-12, atol=1e-15)


def test_batch_norm_bias_invariance():
    """Adding a constant to a conv bias in front of a batch-statistics norm
    changes nothing downstream: its gradient is zero and so is the per-channel
    sum of dz."""
    params = synth.unet_params(1)
    x, t = synth.training_batch(2, 8)
    l0, g0, _, y0, _ = UT.loss_and_grad(params, x, t)
    p2 = [dict(q) for q in params]
    p2[3] = dict(p2[3])
    p2[3]["b"] = p2[3]["b"] + np.float32(0.25)
    l1_, _, _, y1, _ = UT.loss_and_grad(p2, x, t)
    np.testing.assert_allclose(y1, y0, rtol=1e-10, atol=1e-12)
    gnorm = np.linalg.norm(UT.flat(g0))
    for k, q in enumerate(params):
        if "gamma" in q:
            assert np.abs(g0[k]["b"]).max() <= 1e-12 * gnorm, k


def test_block_backward_rules_vs_autograd():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 6, 8, 5))
    dy = rng.standard_normal((2, 3, 4, 5))
    xt = _nchw(x).requires_grad_(True)
    F.max_pool2d(xt, 2).backward(_nchw(dy))
    np.testing.assert_array_equal(UT._max_pool2_bwd(x, dy), _nhwc(xt.grad))
    dy2 = rng.standard_normal((2, 12, 16, 5))
    xt = _nchw(x).requires_grad_(True)
    F.interpolate(xt, scale_factor=2, mode="bilinear", align_corners=False).backward(_nchw(dy2))
    np.testing.assert_allclose(UT._upsample2_bwd(dy2), _nhwc(xt.grad), rtol=1e-12, atol=1e-12)
    # adjointness of the upsampling pair
    lhs = np.sum(U.upsample2(x) * dy2)
    rhs = np.sum(x * UT._upsample2_bwd(dy2))
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)
    w = rng.standard_normal((4, 3, 3, 5))
    dz = rng.standard_normal((2, 6, 8, 4))
    xt = _nchw(x).requires_grad_(True)
    wt = torch.from_numpy(np.moveaxis(w, -1, 1).copy()).requires_grad_(True)
    F.conv2d(xt, wt, padding=1).backward(_nchw(dz))
    dw, db, dx = UT._conv3x3_bwd(x, w, dz)
    np.testing.assert_allclose(dw, np.moveaxis(wt.grad.numpy(), 1, -1), rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(dx, _nhwc(xt.grad), rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(db, dz.sum(axis=(0, 1, 2)), rtol=1e-12)


def test_inference_form_is_the_running_statistics_forward():
    """With the running statistics the training oracle's layer list and
    parameter dicts give the inference oracle's network (same LAYERS)."""
    assert UT.LAYERS == U.LAYERS


def test_branch_conditioning_with_own_decisions_is_exact():
    """Conditioned on its own forward's activations and output, the oracle
    returns exactly its unconditioned loss, output and gradients (the
    conditioning only fixes which piece is differentiated)."""
    params = synth.unet_params(2)
    x, t = synth.training_batch(2, 16)
    l0, g0, dx0, y0, _ = UT.loss_and_grad(params, x, t)
    _, cache, _ = UT.forward_train(params, x)
    acts = [UT._leaky(r["pre"]) for r in cache["layers"]]
    l1_, g1, dx1, y1, _ = UT.loss_and_grad(params, x, t, cond={"a": acts, "y": y0})
    assert l1_ == l0
    np.testing.assert_array_equal(y1, y0)
    np.testing.assert_array_equal(UT.flat(g1), UT.flat(g0))
    np.testing.assert_array_equal(dx1, dx0)
    # a flipped branch changes the gradient (the conditioning is used)
    acts[3] = acts[3].copy()
    acts[3][0, 0, 0, 0] = -acts[3][0, 0, 0, 0]
    _, g2, _, _, _ = UT.loss_and_grad(params, x, t, cond={"a": acts, "y": y0})
    assert not np.array_equal(UT.flat(g2), UT.flat(g0))

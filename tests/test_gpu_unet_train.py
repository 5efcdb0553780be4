"""GPU parity of the paper's network in training form (drc_unet_train_step,
FP32, needs gfx950) against the FP64 training oracle (oracle/unet_train.py,
pinned to PyTorch float64 autograd by test_oracle_unet_train.py).

Checked per step: the forward output (batch statistics) and the loss, the
running statistics written back into the parameters, the gradient of every
trainable tensor (normwise per tensor; the conv bias in front of a
batch-statistics norm has an exactly-zero gradient, so there only its size
against the layer's weight gradient is bounded), zero gradients and
untouched moments for the running-statistics entries, and Adam on the GPU's
own gradient against the oracle's Adam.

Gradient protocol: the network is piecewise smooth (LeakyReLU, max-pool,
output ReLU, L1), and an FP32 forward lands on the other side of a kink for
units within its rounding error of one; each such unit changes its
gradient by a full-size amount (unconditioned, the FP32 gradients are
~6e-4 normwise off the FP64 ones). So the oracle takes the GPU forward's
branch decisions (its activations, read from the workspace) as data, as in
the autoencoder's backward tests. Gates: y and loss <= 2e-5 relative,
gradients <= 1e-4 normwise (FP32 accumulation over up to 4.6 k terms per
output and through 14 batch-norm backward projections).
"""
import numpy as np
import pytest
import torch

from oracle import unet_train as UT
from paper_1910_02480_amd import binding as B
from paper_1910_02480_amd import synth
from tests.helpers import max_rel_per_map, normwise

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _unflat(vec, like):
    out, k = [], 0
    for q in like:
        d = {}
        for name in ("w", "b", "gamma", "beta", "mean", "var"):
            if name in q:
                size = np.asarray(q[name]).size
                d[name] = vec[k:k + size].reshape(np.shape(q[name]))
                k += size
        out.append(d)
    assert k == vec.size
    return out


def _acts(ws, n, H, W):
    """The GPU forward's activations of the 3x3 layers (float64 NHWC)."""
    div = (1, 1, 2, 2, 4, 4, 8, 8, 4, 4, 2, 2, 1, 1)
    cout = (64, 64, 128, 128, 256, 256, 256, 256, 256, 256, 128, 128, 64, 64)
    out = []
    for l, off in enumerate(B.drc_unet_train_act_offsets(n, H, W)):
        cnt = n * (H // div[l]) * (W // div[l]) * cout[l]
        raw = ws[off: off + 4 * cnt].cpu().view(torch.float32).numpy().astype(np.float64)
        out.append(raw.reshape(n, H // div[l], W // div[l], cout[l]))
    return out


def _step(params_flat, x, t, steps=1, want_acts=False):
    n, H, W, _ = x.shape
    p = torch.from_numpy(params_flat.copy()).to(DEV)
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    xd, td = torch.from_numpy(x).to(DEV), torch.from_numpy(t).to(DEV)
    ws = torch.empty(B.drc_unet_train_workspace_size(n, H, W) + 256, dtype=torch.uint8, device=DEV)
    ws = ws[(-ws.data_ptr()) % 256:]
    loss = torch.zeros(1, device=DEV)
    dp = torch.empty_like(p)
    y = torch.empty((n, H, W, 3), device=DEV)
    adam = B.drc_adam_cfg(6e-5, 0.9, 0.999, 1e-8)
    out = []
    for s in range(steps):
        print(f"[unet train] n={n} H={H} W={W} step {s}", flush=True)
        B.drc_unet_train_step(p, m, v, s + 1, adam, xd, td, loss, dp, y, ws)
        torch.cuda.synchronize()
        out.append((float(loss), dp.cpu().numpy().copy(), y.cpu().numpy().copy(), p.cpu().numpy().copy(),
                    m.cpu().numpy().copy(), v.cpu().numpy().copy()))
    if want_acts:
        return out, _acts(ws, n, H, W)
    return out


@pytest.mark.parametrize("n,H,W", [(4, 16, 16), (3, 8, 24), (8, 32, 32)])
def test_train_step_vs_oracle(n, H, W):
    params = synth.unet_params(0)
    flat = synth.unet_flat(params)
    x, t = synth.training_batch(n, H, W)
    ((loss, dp, y, p1, m1, v1),), acts = _step(flat, x, t, want_acts=True)
    lo, grads, _, yo, running = UT.loss_and_grad(params, x, t, cond={"a": acts, "y": y})
    ymr = max_rel_per_map(y, yo).max()
    print(f"unet train {n}x{H}x{W}: y max_rel {ymr:.2e}, loss {loss:.6e} vs {lo:.6e}")
    assert ymr <= 2e-5
    assert abs(loss - lo) <= 2e-5 * abs(lo)
    g = _unflat(dp.astype(np.float64), params)
    errs = []
    for k, (gq, oq) in enumerate(zip(g, grads)):
        ew = normwise(gq["w"], oq["w"])
        e = [ew]
        msg = f"layer {k}: dW {ew:.2e}"
        if "gamma" in oq:
            eg, eb = normwise(gq["gamma"], oq["gamma"]), normwise(gq["beta"], oq["beta"])
            msg += f" dgamma {eg:.2e} dbeta {eb:.2e}"
            e += [eg, eb]
            # the conv bias in front of the batch norm: zero in exact arithmetic
            assert np.abs(gq["b"]).max() <= 1e-5 * np.linalg.norm(oq["w"]), msg
            assert not gq["mean"].any() and not gq["var"].any(), msg
        else:
            eb = normwise(gq["b"], oq["b"])
            msg += f" db {eb:.2e}"
            e.append(eb)
        print(msg)
        errs.append((max(e), msg))
    worst = max(errs)
    assert worst[0] <= 1e-4, worst[1]
    # running statistics written back; their moments untouched
    pn = _unflat(p1.astype(np.float64), params)
    mq = _unflat(m1, params)
    for k, r in enumerate(running):
        if r is None:
            continue
        np.testing.assert_allclose(pn[k]["mean"], r[0], rtol=1e-5, atol=1e-6, err_msg=f"layer {k} mean")
        np.testing.assert_allclose(pn[k]["var"], r[1], rtol=1e-5, atol=1e-6, err_msg=f"layer {k} var")
        assert not mq[k]["mean"].any() and not mq[k]["var"].any()
    # Adam on the GPU's own gradient (trainable entries)
    theta, mm, vv = UT_adam(flat.astype(np.float64), dp.astype(np.float64))
    tr = _trainable_mask(params)
    np.testing.assert_allclose(p1[tr], theta[tr], rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(m1[tr], mm[tr], rtol=1e-5, atol=1e-12)
    np.testing.assert_allclose(v1[tr], vv[tr], rtol=1e-5, atol=1e-18)


def UT_adam(theta, g, lr=6e-5, b1=0.9, b2=0.999, eps=1e-8):
    """PyTorch's first Adam step from zero moments (the oracle's form)."""
    from oracle import oracle as O
    return O.adam(theta, np.zeros_like(theta), np.zeros_like(theta), g, 1, lr, b1, b2, eps)


def _trainable_mask(params):
    parts = []
    for q in params:
        parts += [np.ones(q["w"].size, bool), np.ones(q["b"].size, bool)]
        if "gamma" in q:
            parts += [np.ones(q["gamma"].size, bool), np.ones(q["beta"].size, bool),
                      np.zeros(q["mean"].size, bool), np.zeros(q["var"].size, bool)]
    return np.concatenate(parts)


def test_train_steps_deterministic_and_descending():
    """Two runs of three steps are bitwise equal, and the loss falls on a
    fixed batch (32 maps of 32 x 32, the paper's map size and batch)."""
    params = synth.unet_params(0)
    flat = synth.unet_flat(params)
    x, t = synth.training_batch(32, 32)
    a = _step(flat, x, t, steps=3)
    b = _step(flat, x, t, steps=3)
    for (la, *ra), (lb, *rb) in zip(a, b):
        assert la == lb
        for u, w in zip(ra, rb):
            np.testing.assert_array_equal(u, w)
    losses = [s[0] for s in a]
    print("unet train 32x32x32 losses", losses)
    assert np.all(np.isfinite(losses)) and losses[2] < losses[0]


def test_train_contract():
    L = B.lib()
    adam = B.drc_adam_cfg(6e-5, 0.9, 0.999, 1e-8)
    buf = torch.empty(1 << 20, device=DEV)
    p = buf.data_ptr()
    sz = B._SZ()
    assert L.drc_unet_train_workspace_size(1, 16, 16, sz) == 2          # n < 2
    assert L.drc_unet_train_workspace_size(2, 12, 16, sz) == 2          # not a multiple of 8
    assert L.drc_unet_train_step(p, p, p, 1, None, p, p, p, None, None, 2, 16, 16, p, 1 << 22, None) == 1
    assert L.drc_unet_train_step(p, p, p, 0, adam, p, p, p, None, None, 2, 16, 16, p, 1 << 22, None) == 1
    assert L.drc_unet_train_step(p + 4, p, p, 1, adam, p, p, p, None, None, 2, 16, 16, p, 1 << 22, None) == 1
    assert L.drc_unet_train_step(p, p, p, 1, adam, p, p, p, None, None, 2, 16, 16, p, 16, None) == 4

"""Pins for the oracle's whole network, loss, gradient and optimiser (CPU only).

* forward  : composition of PyTorch float64 library layers; positive
             homogeneity with zero biases; per-map independence;
* L1       : closed form and PyTorch's l1_loss with autograd;
* backward : PyTorch float64 autograd; central finite differences on a
             2 x 8 x 8 batch with kink detection; zero-channel invariant
             (ablation by zeroed channels, Sec. 6.2);
* Adam     : closed-form first step and torch.optim.Adam (the optimiser the
             paper trains with, Sec. 5).
"""
import json
import os

import numpy as np
import pytest
import torch
import torch.nn.functional as F

from paper_1910_02480_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _torch_net(params_t, x_t, final_relu=False):
    """The same autoencoder assembled from PyTorch float64 layers (NCHW)."""
    from oracle.oracle import layer_slices
    sl = layer_slices()
    Ws, Bs = [], []
    for (ws, bs, shp) in sl:
        Ws.append(params_t[ws].reshape(shp))
        Bs.append(params_t[bs])
    conv = lambda a, k: F.conv2d(a, Ws[k].permute(0, 3, 1, 2), Bs[k], stride=2, padding=1)
    tconv = lambda a, k: F.conv_transpose2d(a, Ws[k].permute(3, 0, 1, 2), Bs[k], stride=2,
                                            padding=1, output_padding=1)
    x = x_t.permute(0, 3, 1, 2)
    h1 = F.relu(conv(x, 0))
    h2 = F.relu(conv(h1, 1))
    h3 = F.relu(conv(h2, 2))
    u3 = F.relu(tconv(h3, 3))
    u2 = F.relu(tconv(torch.cat([u3, h2], 1), 4))
    y = tconv(torch.cat([u2, h1], 1), 5)
    if final_relu:
        y = F.relu(y)
    return y.permute(0, 2, 3, 1)


@pytest.fixture(scope="module")
def params():
    return synth.init_params(0).astype(np.float64)


def test_param_layout(oracle):
    assert oracle.num_params() == 206819 == synth.param_count()
    sl = oracle.layer_slices()
    assert sl[0][0].start == 0 and sl[-1][1].stop == 206819


@pytest.mark.parametrize("final_relu", [False, True])
def test_forward_vs_torch(oracle, params, final_relu):
    x = synth.radiance_maps(3, 16, 16).astype(np.float64)
    got = oracle.forward(params, x, final_relu)["y"]
    ref = _torch_net(torch.from_numpy(params), torch.from_numpy(x), final_relu).numpy()
    np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-10)


def test_forward_nonsquare_vs_torch(oracle, params):
    x = synth.radiance_maps(2, 8, 24).astype(np.float64)
    got = oracle.forward(params, x)["y"]
    ref = _torch_net(torch.from_numpy(params), torch.from_numpy(x)).numpy()
    np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-10)


def test_positive_homogeneity(oracle, params):
    p = params.copy()
    for (_, bs, _) in oracle.layer_slices():
        p[bs] = 0.0
    x = synth.radiance_maps(2, 16, 16).astype(np.float64)
    y1 = oracle.forward(p, x)["y"]
    y2 = oracle.forward(p, 2.5 * x)["y"]
    np.testing.assert_allclose(y2, 2.5 * y1, rtol=1e-12, atol=1e-12)


def test_per_map_independence(oracle, params):
    x = synth.radiance_maps(4, 16, 16).astype(np.float64)
    yb = oracle.forward(params, x)["y"]
    for k in range(4):
        np.testing.assert_array_equal(oracle.forward(params, x[k:k + 1])["y"][0], yb[k])


def test_l1_closed_form_and_autograd(oracle):
    r = np.random.default_rng(0)
    y = r.standard_normal((2, 8, 8, 3))
    t = r.standard_normal((2, 8, 8, 3))
    t[0, 0, 0, 0] = y[0, 0, 0, 0]          # a kink: sign(0) = 0
    loss, dy = oracle.l1(y, t)
    assert abs(loss - np.abs(y - t).mean()) < 1e-14
    yt = torch.tensor(y, requires_grad=True)
    F.l1_loss(yt, torch.from_numpy(t)).backward()
    np.testing.assert_array_equal(dy, yt.grad.numpy())
    assert dy[0, 0, 0, 0] == 0.0
    assert set(np.unique(np.abs(dy) * y.size)) <= {0.0, 1.0}


@pytest.mark.parametrize("final_relu", [False, True])
def test_backward_vs_torch_autograd(oracle, params, final_relu):
    x, t = synth.training_batch(2, 16)
    x = x.astype(np.float64)
    loss, dp, dx, _ = oracle.loss_and_grad(params, x, t, final_relu, want_dx=True)
    pt = torch.tensor(params, requires_grad=True)
    xt = torch.tensor(x, requires_grad=True)
    y = _torch_net(pt, xt, final_relu)
    lt = F.l1_loss(y, torch.from_numpy(t.astype(np.float64)))
    lt.backward()
    assert abs(loss - lt.item()) < 1e-12
    np.testing.assert_allclose(dp, pt.grad.numpy(), rtol=1e-9, atol=1e-13)
    np.testing.assert_allclose(dx, xt.grad.numpy(), rtol=1e-9, atol=1e-13)


def _masks(acts):
    return {k: (acts[k] > 0) for k in ("h1", "h2", "h3", "u3", "u2")}


def _same_pattern(oracle, params, x, t, ref_masks, ref_sign):
    a = oracle.forward(params, x)
    m = _masks(a)
    same = all(np.array_equal(m[k], ref_masks[k]) for k in m)
    return same and np.array_equal(np.sign(a["y"] - t), ref_sign)


def test_finite_differences_2x8x8(oracle, params):
    """Analytic FP64 gradient vs central differences on N=2 maps of 8x8.

    Covers every input coordinate, every bias, 1024 seeded weights per layer
    (every weight of a smaller layer) and 8 random directions. Kink detection: a step is used only if the ReLU
    masks and the loss sign pattern at theta +- h equal those at theta; past
    a kink the step shrinks (1e-5, 1e-6, 1e-7 relative), and a coordinate
    that crosses a kink at every step is skipped and counted.
    """
    x, t = synth.training_batch(2, 8)
    x = x.astype(np.float64)
    t = t.astype(np.float64)
    loss0, dp, dx, acts = oracle.loss_and_grad(params, x, t, want_dx=True)
    m0, s0 = _masks(acts), np.sign(acts["y"] - t)
    gmax = max(np.abs(dp).max(), np.abs(dx).max())

    def L(p, xx):
        return oracle.l1(oracle.forward(p, xx)["y"], t)[0]

    def check(get_p_x, theta, analytic):
        # Central differences with the largest step whose mask/sign pattern
        # matches the pattern at theta on both sides; shrink past kinks.
        for rel in (1e-5, 1e-6, 1e-7):
            h = rel * max(1.0, abs(theta))
            pp, xp = get_p_x(theta + h)
            pm, xm = get_p_x(theta - h)
            if (_same_pattern(oracle, pp, xp, t, m0, s0)
                    and _same_pattern(oracle, pm, xm, t, m0, s0)):
                fd = (L(pp, xp) - L(pm, xm)) / (2 * h)
                err = abs(fd - analytic)
                assert err <= 1e-6 * abs(analytic) + 1e-8 * gmax, (theta, fd, analytic)
                return err
        return None

    skipped = 0
    r = np.random.default_rng(123)
    # every input coordinate
    flat = x.reshape(-1)
    for k in range(flat.size):
        def gx(v, k=k):
            xx = flat.copy()
            xx[k] = v
            return params, xx.reshape(x.shape)
        skipped += check(gx, flat[k], dx.reshape(-1)[k]) is None
    # every bias and a sample of weights per layer
    coords = []
    for (ws, bs, _) in oracle.layer_slices():
        coords += list(range(bs.start, bs.stop))
        nw = ws.stop - ws.start
        coords += list(r.choice(np.arange(ws.start, ws.stop), size=min(1024, nw), replace=False))
    for k in coords:
        def gp(v, k=k):
            pp = params.copy()
            pp[k] = v
            return pp, x
        skipped += check(gp, params[k], dp[k]) is None
    # random directions over all parameters and inputs jointly
    for _ in range(8):
        dpv = r.standard_normal(params.shape)
        dxv = r.standard_normal(x.shape)
        an = float(dpv @ dp + np.sum(dxv * dx))
        def gd(s):
            return params + s * dpv, x + s * dxv
        res = check(gd, 0.0, an)
        skipped += res is None
    checks = flat.size + len(coords) + 8
    print(f"finite differences: {checks} checks, {skipped} skipped at kinks")
    assert skipped <= 5 + checks // 200


def test_zero_channel_ablation_invariant(oracle, params):
    """Zeroed input channels (the paper's ablation, Sec. 6.2) get exactly zero E1 weight gradient."""
    x, t = synth.training_batch(2, 16)
    x = x.astype(np.float64)
    x[..., 3:6] = 0.0        # normals removed
    x[..., 6] = 0.0          # distance removed
    _, dp, _, acts = oracle.loss_and_grad(params, x, t)
    ws, _, shp = oracle.layer_slices()[0]
    dW1 = dp[ws].reshape(shp)
    assert np.all(dW1[..., 3:7] == 0.0)
    assert np.any(dW1[..., 0:3] != 0.0)
    p2 = params.copy()
    w1 = p2[ws].reshape(shp)
    w1[..., 3:7] += 0.5
    np.testing.assert_array_equal(oracle.forward(p2, x)["y"], acts["y"])


def test_mask_override_matches_natural_masks(oracle, params):
    x, t = synth.training_batch(2, 16)
    a = oracle.forward(params, x)
    m = _masks(a)
    a2 = oracle.forward(params, x, masks=m)
    for k in a:
        np.testing.assert_array_equal(a[k], a2[k])
    _, dy = oracle.l1(a["y"], t)
    g1, _ = oracle.backward(params, x, a, dy)
    g2, _ = oracle.backward(params, x, a2, dy, masks=m)
    np.testing.assert_array_equal(g1, g2)
    # flipping a mask entry changes the forward exactly at that unit
    m2 = dict(m)
    h1m = m["h1"].copy()
    idx = np.argwhere(h1m)[0]
    h1m[tuple(idx)] = False
    m2["h1"] = h1m
    a3 = oracle.forward(params, x, masks=m2)
    assert a3["h1"][tuple(idx)] == 0.0


def test_adam_first_step_closed_form(oracle):
    r = np.random.default_rng(1)
    g = r.standard_normal(1000) * 10.0 ** r.uniform(-6, 1, 1000)
    th = r.standard_normal(1000)
    lr, eps = 6e-5, 1e-8
    th1, m1, v1 = oracle.adam(th, np.zeros(1000), np.zeros(1000), g, 1, lr=lr, eps=eps)
    np.testing.assert_allclose(th1, th - lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(m1, 0.1 * g, rtol=1e-14)
    np.testing.assert_allclose(v1, 0.001 * g * g, rtol=1e-14)


def test_adam_vs_torch_optim(oracle):
    r = np.random.default_rng(2)
    th = r.standard_normal(500)
    pt = torch.tensor(th, requires_grad=True)
    opt = torch.optim.Adam([pt], lr=6e-5, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(500)
    v = np.zeros(500)
    cur = th.copy()
    for step in range(1, 6):
        g = r.standard_normal(500)
        pt.grad = torch.from_numpy(g.copy())
        opt.step()
        cur, m, v = oracle.adam(cur, m, v, g, step)
        np.testing.assert_allclose(cur, pt.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_paper_constants_fixture():
    """The network I/O and optimiser settings stated in the paper (cited fixture)."""
    with open(os.path.join(GOLDEN, "paper_constants.json")) as f:
        c = json.load(f)
    assert c["input_channels"] == synth.IN_CH == 7
    assert c["output_channels"] == synth.OUT_CH == 3
    assert c["input_channel_order"] == ["R", "G", "B", "Nx", "Ny", "Nz", "D"]
    assert c["adam_lr"] == 6e-5

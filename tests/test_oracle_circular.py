"""Pins for the oracle's circular-azimuth-padding variant (CPU only).

A lat-long map of a hemisphere (Sec. 4.3) is periodic in azimuth, so the
width can wrap around instead of being zero-padded (rows keep zero
padding). The variant is pinned by:

* conv     : PyTorch float64 conv2d of the input padded circularly in the
             width by torch's own circular pad (a different construction);
* tconv    : PyTorch float64 conv_transpose2d without width padding, whose
             two edge columns are folded onto the wrapped output columns;
             adjointness with the circular conv;
* network  : shift equivariance (rolling the input by 8 columns rolls every
             activation by the corresponding number of columns, exactly);
             the zero-padded network differs only near the left and right
             borders; PyTorch autograd of the closed forms above for the
             parameter and input gradients.
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from paper_1910_02480_amd import synth


def _rng(seed):
    return np.random.default_rng(seed)


def _conv_circ_torch(x, wt, b):
    """x [N,H,W,C] -> [N,H/2,W/2,Co]: circular pad of the width, zero pad of the rows."""
    xt = x.permute(0, 3, 1, 2)
    xt = F.pad(xt, (1, 1, 0, 0), mode="circular")
    y = F.conv2d(xt, wt.permute(0, 3, 1, 2), b, stride=2, padding=(1, 0))
    return y.permute(0, 2, 3, 1)


def _tconv_circ_torch(x, wt, b):
    """Transposed conv with no width padding (output width 2W + 1): column f of
    that output is output column (f - 1) mod 2W, so column 0 folds onto 2W - 1."""
    xt = x.permute(0, 3, 1, 2)
    full = F.conv_transpose2d(xt, wt.permute(3, 0, 1, 2), None, stride=2, padding=(1, 0),
                              output_padding=(1, 0))
    w2 = 2 * x.shape[2]
    assert full.shape[-1] == w2 + 1
    out = full[..., 1:].clone()
    out[..., w2 - 1] = out[..., w2 - 1] + full[..., 0]
    if b is not None:
        out = out + b.view(1, -1, 1, 1)
    return out.permute(0, 2, 3, 1)


@pytest.mark.parametrize("n,h,w,ci,co", [(2, 8, 8, 3, 5), (1, 6, 10, 4, 2), (2, 4, 16, 7, 32)])
def test_conv_circular_vs_torch_pad(oracle, n, h, w, ci, co):
    r = _rng(1)
    x, wt, b = r.standard_normal((n, h, w, ci)), r.standard_normal((co, 3, 3, ci)), r.standard_normal(co)
    got = oracle.conv_s2(x, wt, b, circular=True)
    ref = _conv_circ_torch(torch.from_numpy(x), torch.from_numpy(wt), torch.from_numpy(b)).numpy()
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)
    # only the left border column of the output sees the wrap (tap kw = 0 at q = 0)
    zero = oracle.conv_s2(x, wt, b)
    np.testing.assert_array_equal(got[:, :, 1:], zero[:, :, 1:])
    assert not np.allclose(got[:, :, 0], zero[:, :, 0])


@pytest.mark.parametrize("n,h,w,ci,co", [(2, 4, 4, 3, 5), (1, 3, 5, 4, 2), (2, 2, 8, 6, 3)])
def test_tconv_circular_vs_torch_fold(oracle, n, h, w, ci, co):
    r = _rng(2)
    x, wt, b = r.standard_normal((n, h, w, ci)), r.standard_normal((co, 3, 3, ci)), r.standard_normal(co)
    got = oracle.tconv_s2(x, wt, b, circular=True)
    ref = _tconv_circ_torch(torch.from_numpy(x), torch.from_numpy(wt), torch.from_numpy(b)).numpy()
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)
    zero = oracle.tconv_s2(x, wt, b)
    np.testing.assert_array_equal(got[:, :, :-1], zero[:, :, :-1])
    assert not np.allclose(got[:, :, -1], zero[:, :, -1])


@pytest.mark.parametrize("h,w,ci,co", [(8, 8, 3, 4), (6, 12, 2, 5)])
def test_circular_adjointness(oracle, h, w, ci, co):
    """<conv_c(x; W), y> = <x, tconv_c(y; W^T)> with W^T[ci][kh][kw][co] = W[co][kh][kw][ci]."""
    r = _rng(3)
    x = r.standard_normal((2, h, w, ci))
    y = r.standard_normal((2, h // 2, w // 2, co))
    wt = r.standard_normal((co, 3, 3, ci))
    lhs = np.sum(oracle.conv_s2(x, wt, circular=True) * y)
    rhs = np.sum(x * oracle.tconv_s2(y, np.transpose(wt, (3, 1, 2, 0)), circular=True))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


@pytest.fixture(scope="module")
def params():
    return synth.init_params(0).astype(np.float64)


def test_network_shift_equivariance(oracle, params):
    """Rolling the input by 8 columns rolls y by 8, h1 and u2 by 4, h2 and u3
    by 2 and h3 by 1 column, bit for bit (each sum meets the same terms in the
    same order)."""
    x = synth.radiance_maps(2, 16, 32).astype(np.float64)
    a = oracle.forward(params, x, circular=True)
    b = oracle.forward(params, np.roll(x, 8, axis=2), circular=True)
    for k, s in (("h1", 4), ("h2", 2), ("h3", 1), ("u3", 2), ("u2", 4), ("y", 8)):
        np.testing.assert_array_equal(b[k], np.roll(a[k], s, axis=2), err_msg=k)
    # the zero-padded network is not equivariant, and differs near the borders only
    z = oracle.forward(params, x)
    assert not np.allclose(z["y"], a["y"])
    np.testing.assert_allclose(z["y"][:, :, 12:20], a["y"][:, :, 12:20], rtol=0, atol=0)


def _torch_net_circ(params_t, x_t):
    from oracle.oracle import layer_slices
    Ws, Bs = [], []
    for (ws, bs, shp) in layer_slices():
        Ws.append(params_t[ws].reshape(shp))
        Bs.append(params_t[bs])
    conv = lambda a, k: _conv_circ_torch(a, Ws[k], Bs[k])  # noqa: E731
    tconv = lambda a, k: _tconv_circ_torch(a, Ws[k], Bs[k])  # noqa: E731
    h1 = F.relu(conv(x_t, 0))
    h2 = F.relu(conv(h1, 1))
    h3 = F.relu(conv(h2, 2))
    u3 = F.relu(tconv(h3, 3))
    u2 = F.relu(tconv(torch.cat([u3, h2], 3), 4))
    return tconv(torch.cat([u2, h1], 3), 5)


def test_network_forward_and_backward_vs_torch(oracle, params):
    x, t = synth.training_batch(2, 16)
    x = x.astype(np.float64)
    loss, dp, dx, acts = oracle.loss_and_grad(params, x, t, want_dx=True, circular=True)
    pt = torch.tensor(params, requires_grad=True)
    xt = torch.tensor(x, requires_grad=True)
    y = _torch_net_circ(pt, xt)
    np.testing.assert_allclose(acts["y"], y.detach().numpy(), rtol=1e-11, atol=1e-12)
    lt = F.l1_loss(y, torch.from_numpy(t.astype(np.float64)))
    lt.backward()
    assert abs(loss - lt.item()) < 1e-12
    np.testing.assert_allclose(dp, pt.grad.numpy(), rtol=1e-9, atol=1e-13)
    np.testing.assert_allclose(dx, xt.grad.numpy(), rtol=1e-9, atol=1e-13)
    # and the zero-padded gradient differs
    _, dpz, _, _ = oracle.loss_and_grad(params, x, t)
    assert not np.allclose(dpz, dp)

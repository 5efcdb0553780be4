"""Pins for the oracle's single layers (CPU only).

Each operator of the autoencoder (Sec. 4.3: 3x3 convolutions downsampling by
2, 3x3 transposed convolutions upsampling by 2) is checked against things
other than itself: PyTorch's float64 library convolutions, SciPy's 2-D
correlation, exact delta kernels, adjointness and linearity.
"""
import numpy as np
import pytest
import scipy.signal
import torch
import torch.nn.functional as F


def _rng(seed):
    return np.random.default_rng(seed)


def _torch_conv(x, wt, b):
    # W[co][kh][kw][ci] -> conv2d weight [co][ci][kh][kw]
    xt = torch.from_numpy(x).permute(0, 3, 1, 2)
    w = torch.from_numpy(wt).permute(0, 3, 1, 2)
    y = F.conv2d(xt, w, None if b is None else torch.from_numpy(b), stride=2, padding=1)
    return y.permute(0, 2, 3, 1).numpy()


def _torch_tconv(x, wt, b):
    # W[co][kh][kw][ci] -> conv_transpose2d weight [ci][co][kh][kw]
    xt = torch.from_numpy(x).permute(0, 3, 1, 2)
    w = torch.from_numpy(wt).permute(3, 0, 1, 2)
    y = F.conv_transpose2d(xt, w, None if b is None else torch.from_numpy(b),
                           stride=2, padding=1, output_padding=1)
    return y.permute(0, 2, 3, 1).numpy()


@pytest.mark.parametrize("n,h,w,ci,co", [(1, 8, 8, 1, 1), (2, 8, 16, 3, 5),
                                         (3, 16, 8, 7, 32), (1, 6, 10, 4, 2)])
def test_conv_vs_torch(oracle, n, h, w, ci, co):
    r = _rng(10 + ci)
    x = r.standard_normal((n, h, w, ci))
    wt = r.standard_normal((co, 3, 3, ci))
    b = r.standard_normal(co)
    np.testing.assert_allclose(oracle.conv_s2(x, wt, b), _torch_conv(x, wt, b),
                               rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("n,h,w,ci,co", [(1, 4, 4, 1, 1), (2, 4, 8, 3, 5),
                                         (1, 8, 4, 128, 3), (2, 3, 5, 6, 4)])
def test_tconv_vs_torch(oracle, n, h, w, ci, co):
    r = _rng(20 + ci)
    x = r.standard_normal((n, h, w, ci))
    wt = r.standard_normal((co, 3, 3, ci))
    b = r.standard_normal(co)
    np.testing.assert_allclose(oracle.tconv_s2(x, wt, b), _torch_tconv(x, wt, b),
                               rtol=1e-12, atol=1e-12)


def test_conv_vs_scipy_correlate(oracle):
    """Single channel: stride-2 conv == 'same' correlation subsampled at even pixels."""
    r = _rng(3)
    x = r.standard_normal((12, 10))
    k = r.standard_normal((3, 3))
    ref = scipy.signal.correlate2d(x, k, mode="same", boundary="fill")[::2, ::2]
    got = oracle.conv_s2(x[None, :, :, None], k[None, :, :, None])[0, :, :, 0]
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_conv_delta_kernel_subsamples(oracle):
    r = _rng(4)
    x = r.standard_normal((2, 8, 8, 5))
    wt = np.zeros((5, 3, 3, 5))
    for c in range(5):
        wt[c, 1, 1, c] = 1.0
    np.testing.assert_array_equal(oracle.conv_s2(x, wt), x[:, ::2, ::2, :])


def test_conv_corner_tap_shifts(oracle):
    """Tap (0,0) reads x[2p-1, 2q-1]: output row/col 0 sees the zero padding."""
    r = _rng(5)
    x = r.standard_normal((1, 8, 8, 2))
    wt = np.zeros((2, 3, 3, 2))
    wt[0, 0, 0, 0] = 1.0
    wt[1, 2, 2, 1] = 1.0
    y = oracle.conv_s2(x, wt)
    exp0 = np.zeros((4, 4))
    exp0[1:, 1:] = x[0, 1:-1:2, 1:-1:2, 0]
    np.testing.assert_array_equal(y[0, :, :, 0], exp0)
    np.testing.assert_array_equal(y[0, :, :, 1], x[0, 1::2, 1::2, 1])


def test_tconv_delta_kernel_zero_inserts(oracle):
    r = _rng(6)
    x = r.standard_normal((2, 4, 4, 3))
    wt = np.zeros((3, 3, 3, 3))
    for c in range(3):
        wt[c, 1, 1, c] = 1.0
    y = oracle.tconv_s2(x, wt)
    exp = np.zeros((2, 8, 8, 3))
    exp[:, ::2, ::2, :] = x
    np.testing.assert_array_equal(y, exp)


@pytest.mark.parametrize("h,w,ci,co", [(8, 8, 3, 4), (16, 8, 32, 64), (6, 10, 7, 2)])
def test_adjointness(oracle, h, w, ci, co):
    """<conv(x;W), g> == <x, tconv(g; W^T)> with W^T[ci][kh][kw][co] = W[co][kh][kw][ci]."""
    r = _rng(7 + ci)
    x = r.standard_normal((2, h, w, ci))
    wt = r.standard_normal((co, 3, 3, ci))
    g = r.standard_normal((2, h // 2, w // 2, co))
    lhs = np.sum(oracle.conv_s2(x, wt) * g)
    wT = np.ascontiguousarray(wt.transpose(3, 1, 2, 0))
    rhs = np.sum(x * oracle.tconv_s2(g, wT))
    assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(lhs))


def test_linearity(oracle):
    r = _rng(8)
    x1, x2 = r.standard_normal((2, 2, 8, 8, 6))
    w1, w2 = r.standard_normal((2, 4, 3, 3, 6))
    a, c = 0.7, -1.3
    for op in (oracle.conv_s2, oracle.tconv_s2):
        np.testing.assert_allclose(op(a * x1 + c * x2, w1),
                                   a * op(x1, w1) + c * op(x2, w1), rtol=1e-11, atol=1e-11)
        np.testing.assert_allclose(op(x1, a * w1 + c * w2),
                                   a * op(x1, w1) + c * op(x1, w2), rtol=1e-11, atol=1e-11)


def test_brute_force_dense_matrix(oracle):
    """Tiny conv: every output element equals an explicit sum over padded input."""
    r = _rng(9)
    x = r.standard_normal((1, 6, 6, 2))
    wt = r.standard_normal((3, 3, 3, 2))
    b = r.standard_normal(3)
    xp = np.zeros((1, 8, 8, 2))
    xp[:, 1:7, 1:7, :] = x
    y = oracle.conv_s2(x, wt, b)
    for p in range(3):
        for q in range(3):
            for co in range(3):
                s = b[co]
                for kh in range(3):
                    for kw in range(3):
                        s += float(wt[co, kh, kw] @ xp[0, 2 * p + kh, 2 * q + kw])
                assert abs(y[0, p, q, co] - s) < 1e-12


def test_layer_backward_vs_autograd(oracle):
    r = _rng(11)
    for kind in ("conv", "tconv"):
        x = r.standard_normal((2, 8, 6, 5))
        wt = r.standard_normal((4, 3, 3, 5))
        b = r.standard_normal(4)
        xt = torch.tensor(x, requires_grad=True)
        wtt = torch.tensor(wt, requires_grad=True)
        bt = torch.tensor(b, requires_grad=True)
        if kind == "conv":
            y = F.conv2d(xt.permute(0, 3, 1, 2), wtt.permute(0, 3, 1, 2), bt, stride=2, padding=1)
            bwd = oracle.conv_s2_bwd
        else:
            y = F.conv_transpose2d(xt.permute(0, 3, 1, 2), wtt.permute(3, 0, 1, 2), bt,
                                   stride=2, padding=1, output_padding=1)
            bwd = oracle.tconv_s2_bwd
        y = y.permute(0, 2, 3, 1)
        g = r.standard_normal(tuple(y.shape))
        (y * torch.from_numpy(g)).sum().backward()
        dw, db, dx = bwd(x, wt, g)
        np.testing.assert_allclose(dw, wtt.grad.numpy(), rtol=1e-11, atol=1e-11)
        np.testing.assert_allclose(db, bt.grad.numpy(), rtol=1e-11, atol=1e-11)
        np.testing.assert_allclose(dx, xt.grad.numpy(), rtol=1e-11, atol=1e-11)

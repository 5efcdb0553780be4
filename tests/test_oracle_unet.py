"""Pins of the FP64 oracle of the paper's own network (Sec. 4.3 / 5):
each building block against PyTorch's float64 library routine (the
framework of Sec. 5), brute force for the convolution, the whole network
against a composition of library layers, and the model size Sec. 5 states."""
import json
import os

import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import unet as U
from paper_1910_02480_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


def _nchw(a):
    return torch.from_numpy(np.ascontiguousarray(np.moveaxis(a, -1, 1)))


def _nhwc(t):
    return np.moveaxis(t.numpy(), 1, -1)


def test_conv3x3_matches_library_and_brute_force():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 5, 6, 3))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = U.conv3x3(x, w, b)
    ref = F.conv2d(_nchw(x), torch.from_numpy(np.moveaxis(w, -1, 1).copy()), torch.from_numpy(b), padding=1)
    np.testing.assert_allclose(y, _nhwc(ref), rtol=1e-12, atol=1e-12)
    # brute force at one output position next to the border
    n, i, j, co = 1, 0, 5, 2
    s = b[co]
    for kh in range(3):
        for kw in range(3):
            ii, jj = i + kh - 1, j + kw - 1
            if 0 <= ii < 5 and 0 <= jj < 6:
                s += (x[n, ii, jj] * w[co, kh, kw]).sum()
    assert abs(y[n, i, j, co] - s) < 1e-12


def test_blocks_match_library():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 8, 6, 5))
    p = {"gamma": rng.uniform(0.5, 2, 5), "beta": rng.standard_normal(5), "mean": rng.standard_normal(5),
         "var": rng.uniform(0.1, 2, 5)}
    ref = F.batch_norm(_nchw(x), torch.from_numpy(p["mean"]), torch.from_numpy(p["var"]),
                       torch.from_numpy(p["gamma"]), torch.from_numpy(p["beta"]), training=False, eps=1e-5)
    np.testing.assert_allclose(U.batch_norm(x, p), _nhwc(ref), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(U.leaky_relu(x), _nhwc(F.leaky_relu(_nchw(x))), rtol=0, atol=0)
    np.testing.assert_allclose(U.max_pool2(x), _nhwc(F.max_pool2d(_nchw(x), 2)), rtol=0, atol=0)
    up = F.interpolate(_nchw(x), scale_factor=2, mode="bilinear", align_corners=False)
    np.testing.assert_allclose(U.upsample2(x), _nhwc(up), rtol=1e-13, atol=1e-13)


def _torch_forward(params, x):
    t = _nchw(x)
    p = iter(params)

    def block(h, bn=True):
        q = next(p)
        h = F.conv2d(h, torch.from_numpy(np.moveaxis(q["w"].astype(np.float64), -1, 1).copy()),
                     torch.from_numpy(q["b"].astype(np.float64)), padding=1)
        if bn:
            h = F.batch_norm(h, *(torch.from_numpy(q[k].astype(np.float64)) for k in ("mean", "var", "gamma", "beta")),
                             training=False, eps=1e-5)
        return F.leaky_relu(h, 0.01)

    up = lambda h: F.interpolate(h, scale_factor=2, mode="bilinear", align_corners=False)
    s1 = block(block(t))
    s2 = block(block(F.max_pool2d(s1, 2)))
    s3 = block(block(F.max_pool2d(s2, 2)))
    m = block(block(F.max_pool2d(s3, 2)))
    d3 = block(block(torch.cat([up(m), s3], 1)))
    d2 = block(block(torch.cat([up(d3), s2], 1)))
    d1 = block(block(torch.cat([up(d2), s1], 1), False), False)
    q = next(p)
    y = F.conv2d(d1, torch.from_numpy(q["w"].astype(np.float64))[:, :, None, None],
                 torch.from_numpy(q["b"].astype(np.float64)))
    return _nhwc(F.relu(y))


@pytest.mark.parametrize("H,W", [(32, 32), (16, 24)])
def test_forward_matches_library_composition(H, W):
    params = synth.unet_params(0)
    x = synth.radiance_maps(2, H, W).astype(np.float64)
    y = U.forward(params, x)
    np.testing.assert_allclose(y, _torch_forward(params, x), rtol=1e-10, atol=1e-10)
    assert y.shape == (2, H, W, 3) and np.all(y >= 0) and np.any(y > 0)
    # maps are independent
    np.testing.assert_allclose(U.forward(params, x[1:]), y[1:], rtol=1e-12, atol=1e-12)


def test_model_size_is_the_stated_20_mb():
    g = json.load(open(GOLDEN))
    weights = sum(co * ci * (1 if n == "out" else 9) + co for n, ci, co, _ in U.LAYERS)
    mb = weights * 4 / 1e6
    assert abs(mb - g["model_size_mb"]) / g["model_size_mb"] < 0.05, mb
    assert U.LAYERS == tuple((n, ci, co, bn) for n, ci, co, bn in synth.UNET_LAYERS)

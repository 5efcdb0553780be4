"""Cache-point interpolation weights on the GPU against the FP64 oracle
(Sec. 4.2, Eqs. 4-6 with the text's reading).

Indices are integer work and must match exactly. Probabilities: each
weight is a few FP32 roundings from its exact value (distance, 1 - d/r,
normal dot product and norms, product and sum: at most ~10 u relative, or
~u absolute where 1 - d/r cancels), and normalising adds about as much
again, so every probability (at most 1) is within 32 u = 1.9e-6 of the
oracle's (u = 2^-24).
"""
import numpy as np
import pytest
import torch

from oracle import interp as I
from paper_1910_02480_amd import binding as B
from paper_1910_02480_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
ATOL = 32 * 2.0 ** -24


def _gpu(normals, r, cache_normals, eps):
    Hi, Wi, _ = normals.shape
    nd = torch.from_numpy(np.ascontiguousarray(normals, dtype=np.float32)).to(DEV)
    cd = torch.from_numpy(np.ascontiguousarray(cache_normals, dtype=np.float32)).to(DEV)
    idx = torch.full((Hi, Wi, 4), -7, dtype=torch.int32, device=DEV)
    prob = torch.full((Hi, Wi, 4), float("nan"), device=DEV)
    print(f"[interp] Hi={Hi} Wi={Wi} r={r} eps={eps}", flush=True)
    B.drc_interp_weights(nd, r, cd, eps, idx, prob)
    torch.cuda.synchronize()
    return idx.cpu().numpy(), prob.cpu().double().numpy()


def _inputs(Hi, Wi, r, seed=5):
    n = synth.gbuffer_normals(Hi, Wi, seed)
    Gy, Gx = I.grid_shape(Hi, Wi, r)
    cn = n[::r, ::r][:Gy, :Gx].copy()        # a cache point's normal is its pixel's
    cn[::3, ::2] = np.random.default_rng(seed).standard_normal(cn[::3, ::2].shape)  # and some others
    return n, cn


@pytest.mark.parametrize("Hi,Wi,r,eps", [(64, 64, 8, 1e-4), (37, 53, 5, 1e-3), (1, 1, 1, 1e-4), (9, 9, 4, 0.0),
                                         (100, 7, 3, 1e-4), (50, 70, 64, 0.0), (1080, 1920, 16, 1e-4)])
def test_interp_matches_oracle(Hi, Wi, r, eps):
    n, cn = _inputs(Hi, Wi, r)
    idx_g, p_g = _gpu(n, r, cn, eps)
    idx_o, p_o = I.weights(n.astype(np.float64), r, cn.astype(np.float64), eps)
    np.testing.assert_array_equal(idx_g, idx_o)
    np.testing.assert_allclose(p_g, p_o, atol=ATOL, rtol=0)
    present = idx_g >= 0
    assert np.all(p_g[~present] == 0)
    np.testing.assert_allclose(p_g.sum(-1), 1.0, atol=4 * ATOL)


def test_interp_special_cases():
    r, eps = 4, 1e-3
    n = np.zeros((9, 9, 3), np.float32)
    n[..., 2] = 1.0
    cn = np.zeros((3, 3, 3), np.float32)
    cn[..., 2] = 1.0
    cn[0, 1] = (0.0, 0.0, -2.0)
    n[1, 1] = 0.0                                   # background pixel
    idx, p = _gpu(n, r, cn, eps)
    tot = 2 + 4 * eps                               # pixel on cache point (1, 1), aligned normals
    np.testing.assert_allclose(p[4, 4], [(2 + eps) / tot, eps / tot, eps / tot, eps / tot], atol=ATOL)
    np.testing.assert_allclose(p[6, 2], 0.25, atol=ATOL)  # cell centre, equal normals
    w = np.array([0.75 * 1 + 0.75 + eps, 0.25 + eps, eps, eps])  # (x=1, y=0): corner (1, 0) faces away
    np.testing.assert_allclose(p[0, 1], w / w.sum(), atol=ATOL)
    d = np.hypot([1, 3, 1, 3], [1, 1, 3, 3])
    wp = np.maximum(0, 1 - d / r) + eps             # zero normal: w_n = 0
    np.testing.assert_allclose(p[1, 1], wp / wp.sum(), atol=ATOL)

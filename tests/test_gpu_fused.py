"""Whole-network BF16 forward (one kernel, activations in LDS) against the
layer-by-layer path and the FP64 oracle (needs gfx950).

Both paths use the same weight packs, K order and rounding, so their
outputs must agree bit for bit on every map; the oracle bounds the error
of either at the BF16 gate (max |y - r| / max |r| <= 1e-2 per map).
"""
import numpy as np
import pytest
import torch

from paper_1910_02480_amd import synth
from tests.helpers import max_rel_per_map

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def params():
    return synth.init_params(0)


# 64x64: one workgroup per CU, so 300 maps loop past the grid; 32x32: two per CU
@pytest.mark.parametrize("H,n", [(64, 1), (64, 3), (64, 300), (32, 1), (32, 600)])
def test_fused_matches_layer_path_bitwise(params, H, n):
    from paper_1910_02480_amd.cae import CAE
    print(f"[fused] H={H} n={n}", flush=True)
    cae = CAE("bf16", torch.from_numpy(params).to(DEV), device=DEV)
    x = torch.from_numpy(synth.radiance_maps(n, H, H, seed=11)).to(DEV)
    y_fused = cae.forward(x).cpu().numpy()
    cae.set_fused(False)
    y_layer = cae.forward(x).cpu().numpy()
    cae.set_fused(True)
    assert np.isfinite(y_fused).all()
    np.testing.assert_array_equal(y_fused, y_layer)


@pytest.mark.parametrize("H", [64, 32])
def test_fused_vs_oracle(oracle, params, H):
    from paper_1910_02480_amd.cae import CAE
    cae = CAE("bf16", torch.from_numpy(params).to(DEV), device=DEV)
    x = synth.radiance_maps(4, H, H, seed=12)
    y = cae.forward(torch.from_numpy(x).to(DEV)).cpu().numpy()
    r = oracle.forward(params, x[:2])["y"]
    assert max_rel_per_map(y[:2], r).max() <= 1e-2


def test_fused_final_relu_and_repeat(params):
    """Final ReLU variant, and a second call on fewer maps reuses the scratch
    slots without carrying anything over."""
    from paper_1910_02480_amd.cae import CAE
    cae = CAE("bf16", torch.from_numpy(params).to(DEV), device=DEV, final_relu=True)
    x = torch.from_numpy(synth.radiance_maps(20, 64, 64, seed=13)).to(DEV)
    a = cae.forward(x).cpu().numpy()
    b = cae.forward(x[:5]).cpu().numpy()
    cae.set_fused(False)
    c = cae.forward(x).cpu().numpy()
    np.testing.assert_array_equal(a, c)
    np.testing.assert_array_equal(b, c[:5])
    assert (a >= 0).all()

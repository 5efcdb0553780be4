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


@pytest.mark.parametrize("H,recompute", [(64, False), (64, True), (32, False), (32, True)])
def test_fused_saving_forward_and_backward_bitwise(params, H, recompute):
    """A saving forward writes the same activations, and a backward (with or
    without recompute, which also runs fused) the same gradients, as the
    layer path."""
    from paper_1910_02480_amd.cae import CAE
    print(f"[fused-save] H={H} recompute={recompute}", flush=True)
    n = 40
    x = torch.from_numpy(synth.radiance_maps(n, H, H, seed=14)).to(DEV)
    dy = torch.from_numpy(np.random.default_rng(15).standard_normal((n, H, H, 3)).astype(np.float32)).to(DEV)
    out = {}
    for fused in (True, False):
        cae = CAE("bf16", torch.from_numpy(params).to(DEV), device=DEV, recompute=recompute)
        cae.set_fused(fused)
        saved, offsets = cae.saved_buffer(n, H, H)
        saved.zero_()
        y = cae.forward(x, saved=saved)
        dp, _ = cae.backward(x, dy, saved)
        torch.cuda.synchronize()
        out[fused] = (y.cpu().numpy(), saved.cpu().numpy(), dp.cpu().numpy(), offsets)
    np.testing.assert_array_equal(out[True][0], out[False][0])
    np.testing.assert_array_equal(out[True][1], out[False][1])
    _check_grads(out[True][2], out[False][2])


def _check_grads(g_fused, g_layer):
    """Weight gradients bitwise equal; bias gradients (summed inside the fused
    data-gradient kernel, in another fixed order) equal up to float32
    summation rounding."""
    from oracle.oracle import layer_slices
    for ws, bs, _ in layer_slices():
        np.testing.assert_array_equal(g_fused[ws], g_layer[ws])
        ref = g_layer[bs]
        np.testing.assert_allclose(g_fused[bs], ref, rtol=1e-5, atol=1e-6 * max(np.abs(ref).max(), 1e-30))


def test_fused_training_step_matches_layer_path(params):
    """drc_cae_step (forward, L1, recomputing backward, Adam) gives the same
    loss and gradients through either path (bias gradients up to summation
    order), and Adam then moves every weight identically."""
    from oracle.oracle import layer_slices
    from paper_1910_02480_amd.cae import CAE, Trainer
    xt, tg = synth.training_batch(16, 64)
    xt, tg = torch.from_numpy(xt).to(DEV), torch.from_numpy(tg).to(DEV)
    res = {}
    for fused in (True, False):
        cae = CAE("bf16", device=DEV, recompute=True)
        cae.set_fused(fused)
        tr = Trainer(cae, torch.from_numpy(params).to(DEV).clone())
        dp = torch.empty_like(tr.params)
        loss = float(tr.step(xt, tg, dparams=dp))
        res[fused] = (loss, dp.cpu().numpy(), tr.params.cpu().numpy())
    assert res[True][0] == res[False][0]
    _check_grads(res[True][1], res[False][1])
    for ws, _, _ in layer_slices():
        np.testing.assert_array_equal(res[True][2][ws], res[False][2][ws])


# BF16 128x128: D3 and D2 in the banded tail kernel (h3, h2 in; u2 out) against the layer path
@pytest.mark.parametrize("n", [1, 3, 300])
def test_fused_tail_128_matches_layer_path_bitwise(params, n):
    from paper_1910_02480_amd.cae import CAE
    print(f"[fused-tail] H=128 n={n}", flush=True)
    cae = CAE("bf16", torch.from_numpy(params).to(DEV), device=DEV)
    x = torch.from_numpy(synth.radiance_maps(n, 128, 128, seed=23)).to(DEV)
    y_tail = cae.forward(x).cpu().numpy()
    cae.set_fused(False)
    y_layer = cae.forward(x).cpu().numpy()
    assert np.isfinite(y_tail).all()
    np.testing.assert_array_equal(y_tail, y_layer)


# FP8 (e4m3, per-tensor scales): the whole-network kernel against the FP8 layer path
@pytest.mark.parametrize("H,n", [(64, 1), (64, 3), (64, 600), (32, 1), (32, 1100)])
def test_fused_fp8_matches_layer_path_bitwise(params, H, n):
    from paper_1910_02480_amd.cae import CAE
    print(f"[fused-fp8] H={H} n={n}", flush=True)
    cae = CAE("fp8", torch.from_numpy(params).to(DEV), device=DEV)
    cae.calibrate_fp8(torch.from_numpy(synth.radiance_maps(16, 64, 64, seed=3)).to(DEV))
    x = torch.from_numpy(synth.radiance_maps(n, H, H, seed=21)).to(DEV)
    y_fused = cae.forward(x).cpu().numpy()
    cae.set_fused(False)
    y_layer = cae.forward(x).cpu().numpy()
    assert np.isfinite(y_fused).all()
    np.testing.assert_array_equal(y_fused, y_layer)


def test_fused_fp8_repeatable_at_full_batch(params):
    """4096 maps of 64x64 (16 maps per workgroup): three whole-network FP8
    forwards are bitwise equal to each other and to the FP8 layer path. The
    zero block that taps outside the map read shares its LDS bytes with the
    staged input, so it is cleared again after E1 for every map; a clear
    that some wave could overtake with its first read made later maps
    depend on the instruction schedule."""
    from paper_1910_02480_amd.cae import CAE
    n, H = 4096, 64
    print(f"[fused-fp8] repeat H={H} n={n}", flush=True)
    cae = CAE("fp8", torch.from_numpy(params).to(DEV), device=DEV)
    x = torch.from_numpy(synth.radiance_maps(n, H, H, seed=21)).to(DEV)
    cae.calibrate_fp8(x[:256])
    ys = [cae.forward(x).cpu().numpy() for _ in range(3)]
    cae.set_fused(False)
    y_layer = cae.forward(x).cpu().numpy()
    for y in ys:
        np.testing.assert_array_equal(y, y_layer)


def test_fused_fp8_accuracy_reported(oracle, params):
    """FP8 error against the FP64 oracle over 64 maps of 64x64 (reported,
    not gated by the BF16 bound: e4m3 keeps 3 mantissa bits)."""
    from paper_1910_02480_amd.cae import CAE
    from tests.helpers import mean_rel_per_map
    cae = CAE("fp8", torch.from_numpy(params).to(DEV), device=DEV)
    cae.calibrate_fp8(torch.from_numpy(synth.radiance_maps(64, 64, 64, seed=3)).to(DEV))
    x = synth.radiance_maps(64, 64, 64, seed=22)
    y = cae.forward(torch.from_numpy(x).to(DEV)).cpu().numpy()
    r = oracle.forward(params, x)["y"]
    mx, mn = max_rel_per_map(y, r), mean_rel_per_map(y, r)
    print(f"FP8 fused, 64 maps of 64x64: max_rel max {mx.max():.3e} p99 {np.percentile(mx, 99):.3e}, "
          f"mean_rel mean {mn.mean():.3e}")
    assert mx.max() < 0.25 and mn.mean() < 0.1

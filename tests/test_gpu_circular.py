"""GPU parity of the circular-azimuth-padding variant (needs gfx950).

Handles created with pad_w = DRC_PAD_CIRCULAR treat the width as periodic
(a lat-long map of the hemisphere wraps around in azimuth, Sec. 4.3): every
gather of the layer kernels, the data gradients and the weight gradients
wraps columns. Checked against the oracle's circular variant (itself pinned
on the CPU by torch closed forms, adjointness and shift equivariance):

* forward y: FP32 <= 1e-5, BF16 <= 1e-2 max relative error per map, and
  each stored BF16 activation the RNE rounding of the exact layer output on
  the GPU's own inputs; FP8 reported with the zero-padding bound;
* shift equivariance on the GPU itself: rolling the input by 8 columns rolls
  y by 8 columns bit for bit (FP32, BF16, FP8);
* gradients by the mask-conditioned protocol of the backward tests (FP32
  <= 1e-5, BF16 <= 1e-2 normwise per tensor), including a batch whose weight
  gradients run several strips per chunk;
* the whole-network kernels (zero padding only) are refused.
"""
import numpy as np
import pytest
import torch

from paper_1910_02480_amd import synth
from tests.helpers import layer_params, max_rel_per_map, mean_rel_per_map, normwise, round_to, saved_acts

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
NAMES = ("E1", "E2", "E3", "D3", "D2", "D1")


@pytest.fixture(scope="module")
def params():
    return synth.init_params(0)


@pytest.fixture(scope="module")
def params_dev(params):
    return torch.from_numpy(params).to(DEV)


def _cae(compute, params_dev, calib_x=None, **kw):
    from paper_1910_02480_amd.cae import CAE
    c = CAE(compute, params_dev, device=DEV, circular=True, **kw)
    if compute == "fp8":
        c.calibrate_fp8(calib_x)
    return c


def _run(cae, x_np, want_saved=False):
    x = torch.from_numpy(x_np).to(DEV)
    n, H, W, _ = x_np.shape
    saved, off = cae.saved_buffer(n, H, W) if want_saved else (None, None)
    y = cae.forward(x, saved=saved)
    torch.cuda.synchronize()
    return y.cpu().numpy(), saved, off


@pytest.mark.parametrize("compute,gate", [("f32", 1e-5), ("bf16", 1e-2)])
@pytest.mark.parametrize("n,H,W", [(2, 8, 8), (3, 32, 32), (2, 64, 64), (1, 16, 128), (2, 40, 24),
                                   (1, 128, 128)])
def test_forward_vs_oracle(oracle, params, params_dev, compute, gate, n, H, W):
    x = synth.radiance_maps(n, H, W, seed=7)
    y, _, _ = _run(_cae(compute, params_dev), x)
    r = oracle.forward(params, x, circular=True)["y"]
    mr = max_rel_per_map(y, r)
    print(f"{compute} {n}x{H}x{W} circular: max_rel {mr.max():.3e}, mean_rel {mean_rel_per_map(y, r).mean():.3e}")
    assert mr.max() <= gate
    # the test can tell the variants apart: the zero-padded result is further off
    rz = oracle.forward(params, x)["y"]
    assert max_rel_per_map(rz, r).max() > 10 * gate


def _layer_refs_circ(oracle, params, x, acts, compute):
    def W(k):
        w, b = layer_params(params, k)
        return round_to(w, compute), b.astype(np.float64)

    refs = {}
    refs["h1"] = oracle.conv_s2(round_to(x, compute), *W(0), circular=True)
    refs["h2"] = oracle.conv_s2(acts["h1"], *W(1), circular=True)
    refs["h3"] = oracle.conv_s2(acts["h2"], *W(2), circular=True)
    refs["u3"] = oracle.tconv_s2(acts["h3"], *W(3), circular=True)
    refs["u2"] = oracle.tconv_s2(np.concatenate([acts["u3"], acts["h2"]], -1), *W(4), circular=True)
    refs["y"] = oracle.tconv_s2(np.concatenate([acts["u2"], acts["h1"]], -1), *W(5), circular=True)
    for k in ("h1", "h2", "h3", "u3", "u2"):
        refs[k] = np.maximum(refs[k], 0.0)
    return refs


def _half_ulp_bf16(v):
    a = np.abs(v)
    e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    return np.where(a > 0, 2.0 ** (e - 8), 0.0)


@pytest.mark.parametrize("n,H,W", [(2, 32, 32), (1, 64, 64), (1, 128, 128), (2, 24, 40)])
def test_layers_bf16_round_to_nearest_even(oracle, params, params_dev, n, H, W):
    x = synth.radiance_maps(n, H, W, seed=11)
    y, saved, off = _run(_cae("bf16", params_dev), x, want_saved=True)
    acts = saved_acts(saved, off, n, H, W, "bf16")
    refs = _layer_refs_circ(oracle, params, x, acts, "bf16")
    for name in ("h1", "h2", "h3", "u3", "u2"):
        g, r = acts[name], refs[name]
        err = np.abs(g - r)
        tol = _half_ulp_bf16(r) * (1 + 1e-3) + 1e-6 * np.abs(r).max()
        assert np.mean(err <= tol) >= 0.999, name
        assert np.all(err <= 2 * _half_ulp_bf16(r) + 1e-5 * np.abs(r).max()), name
    assert max_rel_per_map(y, refs["y"]).max() <= 1e-5


def test_fp8_forward_reported(oracle, params, params_dev):
    calib = torch.from_numpy(synth.radiance_maps(64, 32, 32, seed=11)).to(DEV)
    cae = _cae("fp8", params_dev, calib_x=calib)
    x = synth.radiance_maps(8, 32, 32)
    y, _, _ = _run(cae, x)
    r = oracle.forward(params, x, circular=True)["y"]
    mr = max_rel_per_map(y, r)
    print(f"fp8 8x32x32 circular: max_rel max {mr.max():.3e}, mean_rel {mean_rel_per_map(y, r).mean():.3e}")
    assert np.all(np.isfinite(y)) and mr.max() <= 0.25


@pytest.mark.parametrize("compute", ["f32", "bf16", "fp8"])
def test_shift_equivariance_bitwise(params_dev, compute):
    """Rolling the input by 8 columns rolls y by 8 columns, bit for bit: every
    output meets the same products in the same order."""
    x = synth.radiance_maps(3, 32, 64, seed=5)
    calib = torch.from_numpy(x).to(DEV) if compute == "fp8" else None
    cae = _cae(compute, params_dev, calib_x=calib)
    y0, _, _ = _run(cae, x)
    y1, _, _ = _run(cae, np.ascontiguousarray(np.roll(x, 8, axis=2)))
    np.testing.assert_array_equal(y1, np.roll(y0, 8, axis=2))


def _masked_oracle_grad(oracle, params, x, acts, dy):
    masks = {k: acts[k] > 0 for k in ("h1", "h2", "h3", "u3", "u2")}
    a = oracle.forward(params, x, masks=masks, circular=True)
    return oracle.backward(params, x, a, dy, masks=masks, want_dx=True, circular=True)


@pytest.mark.parametrize("compute,gate", [("f32", 1e-5), ("bf16", 1e-2)])
@pytest.mark.parametrize("n,H,W", [(2, 8, 8), (4, 32, 32), (2, 64, 64), (3, 40, 24), (64, 64, 64)])
def test_backward_mask_conditioned(oracle, params, params_dev, compute, gate, n, H, W):
    """n = 64 at 64 x 64: the weight-gradient kernels run several strips per
    chunk, as at the training batch."""
    x, _ = synth.training_batch(n, H, W)
    dy = np.random.default_rng(5).standard_normal((n, H, W, 3)).astype(np.float32)
    cae = _cae(compute, params_dev)
    xd, dyd = torch.from_numpy(x).to(DEV), torch.from_numpy(dy).to(DEV)
    saved, off = cae.saved_buffer(n, H, W)
    cae.forward(xd, saved=saved)
    dp, dx = cae.backward(xd, dyd, saved, want_dx=True)
    torch.cuda.synchronize()
    dp, dx = dp.cpu().numpy(), dx.cpu().numpy()
    acts = saved_acts(saved, off, n, H, W, compute)
    dp_ref, dx_ref = _masked_oracle_grad(oracle, params, x, acts, dy)
    for k, (ws, bs, _) in enumerate(oracle.layer_slices()):
        ew, eb = normwise(dp[ws], dp_ref[ws]), normwise(dp[bs], dp_ref[bs])
        print(f"{compute} {n}x{H}x{W} circular {NAMES[k]}: dW {ew:.2e} db {eb:.2e}")
        assert ew <= gate and eb <= gate, NAMES[k]
    assert normwise(dx, dx_ref) <= gate


@pytest.mark.parametrize("compute", ["f32", "bf16"])
def test_training_step_loss_and_recompute(oracle, params, params_dev, compute):
    """A training step (recompute on) gives the loss of the circular forward,
    and the same parameters as the step without recompute."""
    from paper_1910_02480_amd.cae import Trainer
    x, t = synth.training_batch(8, 32)
    xd, td = torch.from_numpy(x).to(DEV), torch.from_numpy(t).to(DEV)
    y, _, _ = _run(_cae(compute, params_dev), x)
    loss_ref, _ = oracle.l1(y, t)
    outs = []
    for rc in (False, True):
        tr = Trainer(_cae(compute, params_dev, recompute=rc), params_dev.clone())
        loss = float(tr.step(xd, td))
        assert abs(loss - loss_ref) <= 1e-6 * abs(loss_ref)
        outs.append(tr.params.cpu().numpy())
    np.testing.assert_array_equal(outs[0], outs[1])


def test_whole_network_kernels_refused(params_dev):
    from paper_1910_02480_amd import binding as B
    cae = _cae("bf16", params_dev)
    with pytest.raises(B.DrcError) as e:
        cae.set_fused(True)
    assert e.value.status == 3
    cae.set_fused(False)

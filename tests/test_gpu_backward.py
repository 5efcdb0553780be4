"""GPU parity of the backward pass and the training step (needs gfx950).

Gradient protocol. The network is piecewise linear, so its gradient jumps
where a ReLU pre-activation or an L1 residual crosses zero; a forward pass
in any finite precision lands on the other side of such a kink for units
within its rounding error of zero. The oracle therefore takes the GPU
forward's ReLU masks (read from the saved activations, a > 0) as data, and
both sides get the same dL/dy. Gates (normwise per parameter tensor):
FP32 <= 1e-5, BF16 <= 1e-2. Adam is checked in isolation on the GPU's own
gradient.
"""
import numpy as np
import pytest
import torch

from paper_1910_02480_amd import synth
from tests.helpers import normwise, saved_acts

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
NAMES = ("E1", "E2", "E3", "D3", "D2", "D1")


@pytest.fixture(scope="module")
def params():
    return synth.init_params(0)


def _cae(compute, params, recompute=False):
    from paper_1910_02480_amd.cae import CAE
    return CAE(compute, torch.from_numpy(params).to(DEV), device=DEV, recompute=recompute)


def _fwd_bwd(cae, x_np, dy_np, want_dx=True):
    n, H, W, _ = x_np.shape
    x = torch.from_numpy(x_np).to(DEV)
    dy = torch.from_numpy(dy_np).to(DEV)
    saved, off = cae.saved_buffer(n, H, W)
    y = cae.forward(x, saved=saved)
    dp, dx = cae.backward(x, dy, saved, want_dx=want_dx)
    torch.cuda.synchronize()
    return (y.cpu().numpy(), dp.cpu().numpy(), None if dx is None else dx.cpu().numpy(), saved, off)


def _masked_oracle_grad(oracle, params, x, acts, dy):
    masks = {k: acts[k] > 0 for k in ("h1", "h2", "h3", "u3", "u2")}
    a = oracle.forward(params, x, masks=masks)
    dp, dx = oracle.backward(params, x, a, dy, masks=masks, want_dx=True)
    return dp, dx


@pytest.mark.parametrize("compute,gate", [("f32", 1e-5), ("bf16", 1e-2)])
@pytest.mark.parametrize("n,H,W", [(2, 8, 8), (4, 32, 32), (2, 64, 64), (3, 40, 24)])
def test_backward_mask_conditioned(oracle, params, compute, gate, n, H, W):
    x, t = synth.training_batch(n, H, W)
    dy = np.random.default_rng(5).standard_normal((n, H, W, 3)).astype(np.float32)
    cae = _cae(compute, params)
    y, dp, dx, saved, off = _fwd_bwd(cae, x, dy)
    acts = saved_acts(saved, off, n, H, W, compute)
    dp_ref, dx_ref = _masked_oracle_grad(oracle, params, x, acts, dy)
    for k, (ws, bs, _) in enumerate(oracle.layer_slices()):
        ew, eb = normwise(dp[ws], dp_ref[ws]), normwise(dp[bs], dp_ref[bs])
        print(f"{compute} {n}x{H}x{W} {NAMES[k]}: dW {ew:.2e} db {eb:.2e}")
        assert ew <= gate and eb <= gate, NAMES[k]
    edx = normwise(dx, dx_ref)
    print(f"{compute} dx {edx:.2e}")
    assert edx <= gate


def test_backward_f32_vs_oracle_gradient_2x8x8(oracle, params):
    """The 2 x 8 x 8 case whose oracle gradient is pinned to FP64 central
    finite differences on the CPU: the FP32 GPU gradient matches it."""
    x, t = synth.training_batch(2, 8)
    cae = _cae("f32", params)
    y, _, _, saved, off = _fwd_bwd(cae, x, np.zeros((2, 8, 8, 3), np.float32), want_dx=False)
    loss, dy = oracle.l1(y, t)
    _, dp, dx, saved, off = _fwd_bwd(cae, x, dy.astype(np.float32))
    acts = saved_acts(saved, off, 2, 8, 8, "f32")
    dp_ref, dx_ref = _masked_oracle_grad(oracle, params, x, acts, dy)
    assert normwise(dp, dp_ref) <= 1e-5
    assert normwise(dx, dx_ref) <= 1e-5


@pytest.mark.parametrize("compute", ["f32", "bf16"])
def test_recompute_bitwise_equal(params, compute):
    x, _ = synth.training_batch(4, 32)
    dy = np.random.default_rng(1).standard_normal((4, 32, 32, 3)).astype(np.float32)
    _, g0, dx0, _, _ = _fwd_bwd(_cae(compute, params, recompute=False), x, dy)
    _, g1, dx1, _, off = _fwd_bwd(_cae(compute, params, recompute=True), x, dy)
    assert off[2] == off[3] == off[4] == -1
    np.testing.assert_array_equal(g0, g1)
    np.testing.assert_array_equal(dx0, dx1)


def test_backward_determinism(params):
    x, _ = synth.training_batch(8, 64)
    dy = np.random.default_rng(2).standard_normal((8, 64, 64, 3)).astype(np.float32)
    cae = _cae("bf16", params)
    _, g0, _, _, _ = _fwd_bwd(cae, x, dy)
    _, g1, _, _, _ = _fwd_bwd(cae, x, dy)
    np.testing.assert_array_equal(g0, g1)


@pytest.mark.parametrize("compute", ["f32", "bf16"])
def test_zero_channel_ablation(params, compute):
    """Zeroed input channels (the paper's ablation, Sec. 6.2) receive exactly
    zero E1 weight gradient, and their E1 weights do not affect y."""
    x, t = synth.training_batch(2, 32)
    x[..., 3:7] = 0.0
    dy = np.random.default_rng(3).standard_normal((2, 32, 32, 3)).astype(np.float32)
    cae = _cae(compute, params)
    y0, dp, _, _, _ = _fwd_bwd(cae, x, dy, want_dx=False)
    dW1 = dp[:32 * 9 * 7].reshape(32, 3, 3, 7)
    assert np.all(dW1[..., 3:7] == 0.0)
    assert np.any(dW1[..., :3] != 0.0)
    p2 = params.copy()
    p2[:32 * 9 * 7].reshape(32, 3, 3, 7)[..., 3:7] += 0.25
    y1, _, _, _, _ = _fwd_bwd(_cae(compute, p2), x, dy, want_dx=False)
    np.testing.assert_array_equal(y0, y1)


@pytest.mark.parametrize("compute,gate", [("f32", 1e-5), ("bf16", 1e-2)])
def test_training_step(oracle, params, compute, gate):
    """drc_cae_step: L1 loss, gradient and PyTorch-form Adam update."""
    from paper_1910_02480_amd.cae import CAE, Trainer
    n, H = 4, 64
    x, t = synth.training_batch(n, H)
    p = torch.from_numpy(params.copy()).to(DEV)
    cae = CAE(compute, device=DEV, recompute=True)
    tr = Trainer(cae, p)
    xd, td = torch.from_numpy(x).to(DEV), torch.from_numpy(t).to(DEV)
    g = torch.empty_like(p)
    loss = tr.step(xd, td, dparams=g).item()
    torch.cuda.synchronize()
    g = g.cpu().numpy()
    # loss and gradient vs the oracle at the same parameters (mask-conditioned
    # on a GPU forward with those parameters)
    cae2 = _cae(compute, params)
    y, _, _, saved, off = _fwd_bwd(cae2, x, np.zeros((n, H, H, 3), np.float32), want_dx=False)
    acts = saved_acts(saved, off, n, H, H, compute)
    loss_ref, dy_ref = oracle.l1(y, t)
    assert abs(loss - loss_ref) <= 1e-6 * loss_ref
    loss_o = oracle.l1(oracle.forward(params, x)["y"], t)[0]
    assert abs(loss - loss_o) <= gate * loss_o
    masks = {k: acts[k] > 0 for k in ("h1", "h2", "h3", "u3", "u2")}
    a = oracle.forward(params, x, masks=masks)
    # same residual signs as the GPU forward
    dp_ref, _ = oracle.backward(params, x, a, dy_ref, masks=masks)
    for k, (ws, bs, _) in enumerate(oracle.layer_slices()):
        assert normwise(g[ws], dp_ref[ws]) <= gate, NAMES[k]
        assert normwise(g[bs], dp_ref[bs]) <= gate, NAMES[k]
    # Adam in isolation: the update the GPU applied, from the gradient it used
    th_ref, m_ref, v_ref = oracle.adam(params, np.zeros_like(params), np.zeros_like(params), g, 1)
    th = p.cpu().numpy().astype(np.float64)
    ulp = np.spacing(np.abs(th_ref).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(th - th_ref) <= 2 * ulp + 1e-6 * np.abs(th_ref - params))
    np.testing.assert_allclose(tr.m.cpu().numpy(), m_ref, rtol=1e-6, atol=1e-30)
    np.testing.assert_allclose(tr.v.cpu().numpy(), v_ref, rtol=1e-5, atol=1e-30)


def test_training_reduces_loss(params):
    """A few BF16 steps on the lobe-target pairs lower the L1 loss."""
    from paper_1910_02480_amd.cae import CAE, Trainer
    x, t = synth.training_batch(32, 32)
    p = torch.from_numpy(params.copy()).to(DEV)
    tr = Trainer(CAE("bf16", device=DEV, recompute=True), p, lr=1e-3)
    xd, td = torch.from_numpy(x).to(DEV), torch.from_numpy(t).to(DEV)
    losses = [tr.step(xd, td).item() for _ in range(20)]
    print("losses", losses[0], losses[-1])
    assert losses[-1] < 0.7 * losses[0]


def test_autograd_function(params):
    """CAEFunction routes torch autograd through drc_cae_backward."""
    from paper_1910_02480_amd.cae import CAE, CAEFunction
    x, t = synth.training_batch(2, 32)
    p = torch.from_numpy(params).to(DEV).requires_grad_(True)
    cae = CAE("f32", p.detach(), device=DEV)
    xd = torch.from_numpy(x).to(DEV).requires_grad_(True)
    y = CAEFunction.apply(xd, p, cae)
    loss = torch.nn.functional.l1_loss(y, torch.from_numpy(t).to(DEV))
    loss.backward()
    dy = (torch.sign(y.detach() - torch.from_numpy(t).to(DEV)) / y.numel())
    dp, dx = cae.backward(xd.detach(), dy, *_saved_again(cae, xd.detach()), want_dx=True)
    np.testing.assert_allclose(p.grad.cpu().numpy(), dp.cpu().numpy(), rtol=1e-6, atol=1e-12)
    np.testing.assert_allclose(xd.grad.cpu().numpy(), dx.cpu().numpy(), rtol=1e-6, atol=1e-12)


def _saved_again(cae, x):
    n, H, W, _ = x.shape
    saved, _ = cae.saved_buffer(n, H, W)
    cae.forward(x, saved=saved)
    return (saved,)


def test_autograd_function_tracks_params(params):
    """CAEFunction computes with the current values of params: an in-place
    update is repacked before the next forward, and a tensor the handle was
    not packed from is rejected."""
    from paper_1910_02480_amd.cae import CAE, CAEFunction
    x, _ = synth.training_batch(2, 32)
    xd = torch.from_numpy(x).to(DEV)
    p = torch.from_numpy(params.copy()).to(DEV).requires_grad_(True)
    cae = CAE("f32", p.detach(), device=DEV)
    y0 = CAEFunction.apply(xd, p, cae).detach().clone()
    with torch.no_grad():
        p.mul_(2.0)
    y1 = CAEFunction.apply(xd, p, cae).detach()
    ref = CAE("f32", p.detach().clone(), device=DEV).forward(xd)
    torch.cuda.synchronize()
    assert not torch.equal(y0, y1)
    assert torch.equal(y1, ref)
    other = p.detach().clone().requires_grad_(True)
    with pytest.raises(ValueError):
        CAEFunction.apply(xd, other, cae)

"""GPU parity at the batch sizes the benchmark runs (needs gfx950).

The weight gradients sum over every pixel of the batch in chunks of strips
(drc_cae_wgrad_schedule); small batches run one strip per chunk, the
benchmark's batches several, with the next strip's loads issued during the
current strip's MFMAs. These tests compare that multi-strip schedule (and a
ragged last chunk) with the FP64 oracle, mask-conditioned as in
test_gpu_backward.py (the oracle takes the GPU forward's ReLU masks and the
same dL/dy; gates normwise per parameter tensor: FP32 1e-5, BF16 1e-2), and
check a sample of the 6000-map mixed frame against the oracle.
"""
import math

import numpy as np
import pytest
import torch

from paper_1910_02480_amd import binding as B
from paper_1910_02480_amd import synth
from tests.helpers import max_rel_per_map, mean_rel_per_map, normwise, saved_acts

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
NAMES = ("E1", "E2", "E3", "D3", "D2", "D1")
ACTS = ("h1", "h2", "h3", "u3", "u2")


@pytest.fixture(scope="module")
def params():
    return synth.init_params(0)


def _strips(n, H, layer):
    """Strips of the layer's weight-gradient reduction over a batch."""
    kind, R, spc, chunks = B.drc_cae_wgrad_schedule(B.DRC_BF16, layer, n, H, H)
    rows = (H // 2, H // 4, H // 8, H // 8, H // 4, H // 2)[layer]
    return kind, spc, chunks, n * math.ceil(rows / R)


def _check_grads(oracle, params, g, dp_ref, gate, tag):
    for k, (ws, bs, _) in enumerate(oracle.layer_slices()):
        ew, eb = normwise(g[ws], dp_ref[ws]), normwise(g[bs], dp_ref[bs])
        print(f"{tag} {NAMES[k]}: dW {ew:.2e} db {eb:.2e}", flush=True)
        assert ew <= gate and eb <= gate, (tag, NAMES[k], ew, eb)


@pytest.mark.parametrize("compute,gate", [("bf16", 1e-2), ("f32", 1e-5)])
def test_step_gradient_at_training_batch(oracle, params, compute, gate):
    """drc_cae_step on 256 training pairs of 64x64 (recompute on): loss and
    gradient against the oracle. In BF16 every layer's weight gradient runs
    at least 2 strips per chunk at this batch."""
    n, H = 256, 64
    if compute == "bf16":
        for l in range(6):
            kind, spc, chunks, total = _strips(n, H, l)
            assert kind == 2 and spc >= 2, (NAMES[l], kind, spc)
    from paper_1910_02480_amd.cae import CAE, Trainer
    x, t = synth.training_batch(n, H)
    p = torch.from_numpy(params.copy()).to(DEV)
    tr = Trainer(CAE(compute, device=DEV, recompute=True), p)
    xd, td = torch.from_numpy(x).to(DEV), torch.from_numpy(t).to(DEV)
    g = torch.empty_like(p)
    loss = tr.step(xd, td, dparams=g).item()
    torch.cuda.synchronize()
    g = g.cpu().numpy()
    # the GPU forward at the same parameters, its masks and its residual signs
    cae = CAE(compute, torch.from_numpy(params).to(DEV), device=DEV)
    saved, off = cae.saved_buffer(n, H, H)
    y = cae.forward(xd, saved=saved).cpu().numpy()
    acts = saved_acts(saved, off, n, H, H, compute)
    loss_ref, dy_ref = oracle.l1(y, t)
    assert abs(loss - loss_ref) <= 1e-6 * loss_ref
    masks = {k: acts[k] > 0 for k in ACTS}
    a = oracle.forward(params, x, masks=masks)
    dp_ref, _ = oracle.backward(params, x, a, dy_ref, masks=masks)
    _check_grads(oracle, params, g, dp_ref, gate, f"step {compute} {n}x{H}x{H}")


@pytest.mark.parametrize("n", [1024, 700])
def test_backward_bf16_large_batch(oracle, params, n):
    """drc_cae_backward on n maps of 64x64 in BF16 (activations saved): every
    layer at 4 to 8 strips per chunk; at n = 700 every layer's last chunk is
    short (total strips not a multiple of the chunk)."""
    H = 64
    for l in range(6):
        kind, spc, chunks, total = _strips(n, H, l)
        assert kind == 2 and spc >= 4, (NAMES[l], spc)
        if n == 700:
            assert total % spc != 0 and chunks == -(-total // spc), (NAMES[l], total, spc)
    from paper_1910_02480_amd.cae import CAE
    x, _ = synth.training_batch(n, H)
    dy = (np.random.default_rng(11).standard_normal((n, H, H, 3)) / (n * H * H * 3)).astype(np.float32)
    cae = CAE("bf16", torch.from_numpy(params).to(DEV), device=DEV)
    xd, dyd = torch.from_numpy(x).to(DEV), torch.from_numpy(dy).to(DEV)
    saved, off = cae.saved_buffer(n, H, H)
    cae.forward(xd, saved=saved)
    dp, dx = cae.backward(xd, dyd, saved, want_dx=True)
    torch.cuda.synchronize()
    g, dx = dp.cpu().numpy(), dx.cpu().numpy()
    acts = saved_acts(saved, off, n, H, H, "bf16")
    masks = {k: acts[k] > 0 for k in ACTS}
    a = oracle.forward(params, x, masks=masks)
    dp_ref, dx_ref = oracle.backward(params, x, a, dy, masks=masks, want_dx=True)
    _check_grads(oracle, params, g, dp_ref, 1e-2, f"backward bf16 {n}x{H}x{H}")
    e = normwise(dx, dx_ref)
    print(f"dx {e:.2e}")
    assert e <= 1e-2


def test_mixed_frame_6000_sampled(oracle, params):
    """The benchmark's 6000-map frame (50 % 32x32, 35 % 64x64, 15 % 128x128,
    shuffled by seed 2), one captured-graph launch and two replays (the
    128x128 chain on the handle's side stream beside the whole-network
    launches); 4 maps of each size, drawn by seed, against the oracle map by
    map (max_rel <= 1e-2), and every map of every launch bitwise equal to
    uniform forwards of its size class on one stream."""
    from paper_1910_02480_amd.cae import CAE
    res = synth.mixed_resolutions(6000)
    x, xo, yo = synth.mixed_frame(res)
    ny = int(yo[-1] + res[-1] * res[-1] * 3)
    cae = CAE("bf16", torch.from_numpy(params).to(DEV), device=DEV)
    maps = [(int(r), int(r), int(xo[m]), int(yo[m])) for m, r in enumerate(res)]
    plan = B.drc_cae_plan_create(cae.h, maps)
    try:
        ws = torch.empty(B.drc_cae_plan_workspace_size(plan) + 256, dtype=torch.uint8, device=DEV)
        ws = ws[(-ws.data_ptr()) % 256:]
        xd = torch.from_numpy(x).to(DEV)
        yd = torch.full((ny,), float("nan"), device=DEV)
        stream = torch.cuda.Stream(device=DEV)
        torch.cuda.synchronize()
        ys = []
        for rep in range(3):
            print(f"[frame 6000] launch {rep}", flush=True)
            with torch.cuda.stream(stream):
                yd.fill_(float("nan"))
                B.drc_cae_plan_launch(plan, xd, yd, ws)
            torch.cuda.synchronize()
            ys.append(yd.cpu().numpy())
        assert B.drc_cae_plan_captures(plan) == 1
    finally:
        B.drc_cae_plan_destroy(plan)
    y = ys[0]
    assert np.all(np.isfinite(y))
    for r in (32, 64, 128):
        idx = np.flatnonzero(res == r)
        xs = torch.from_numpy(np.stack([x[xo[m]:xo[m] + r * r * 7].reshape(r, r, 7) for m in idx])).to(DEV)
        ref = cae.forward(xs).cpu().numpy().reshape(len(idx), -1)
        for k, yk in enumerate(ys):
            got = np.stack([yk[yo[m]:yo[m] + r * r * 3] for m in idx])
            np.testing.assert_array_equal(got, ref, err_msg=f"{r}x{r} class, launch {k}")
    rng = np.random.default_rng(7)
    for r in (32, 64, 128):
        pick = rng.choice(np.flatnonzero(res == r), size=4, replace=False)
        xs = np.stack([x[xo[m]:xo[m] + r * r * 7].reshape(r, r, 7) for m in pick])
        ref = oracle.forward(params, xs)["y"]
        got = np.stack([y[yo[m]:yo[m] + r * r * 3].reshape(r, r, 3) for m in pick])
        mx, mn = max_rel_per_map(got, ref), mean_rel_per_map(got, ref)
        print(f"{r}x{r} maps {pick.tolist()}: max_rel {mx.max():.2e}, mean_rel {mn.max():.2e}", flush=True)
        assert mx.max() <= 1e-2, (r, pick, mx)

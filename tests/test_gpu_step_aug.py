"""The training step on augmented maps with the augmentation in the loaders
(drc_cae_step_aug, needs gfx950).

Sec. 5 trains on rotated and flipped maps. drc_cae_step_aug reads x and the
target through the rotation / mirror in the whole-network forward's input
staging, E1's weight gradient and the loss, instead of writing augmented
copies first. It must equal drc_augment followed by drc_cae_step bit for bit
(loss, gradient, parameters and Adam moments, over consecutive steps), at
the training batch (256 maps of 64x64, whose weight gradients run several
strips per chunk) and at 32x32, with and without activation recompute. The
augmentation itself is checked against the oracle in test_gpu_augment.py.
"""
import numpy as np
import pytest
import torch

from paper_1910_02480_amd import binding as B
from paper_1910_02480_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _rolls(n, W, seed):
    r = np.random.default_rng(seed)
    roll = r.integers(-3 * W, 3 * W, n).astype(np.int32)
    flip = r.integers(0, 2, n).astype(np.int32)
    roll[0], flip[0] = 0, 0          # identity
    roll[1], flip[1] = W // 4, 1     # a quarter turn, mirrored
    return torch.from_numpy(roll).to(DEV), torch.from_numpy(flip).to(DEV)


@pytest.mark.parametrize("n,H,recompute", [(256, 64, True), (256, 64, False), (24, 32, True), (5, 64, True)])
def test_step_aug_equals_augment_then_step(n, H, recompute):
    from paper_1910_02480_amd.cae import CAE, Trainer, augment
    p0 = torch.from_numpy(synth.init_params(0)).to(DEV)
    xs, ts = synth.training_batch(n, H)
    x, t = torch.from_numpy(xs).to(DEV), torch.from_numpy(ts).to(DEV)
    a = Trainer(CAE("bf16", device=DEV, recompute=recompute), p0.clone())
    b = Trainer(CAE("bf16", device=DEV, recompute=recompute), p0.clone())
    ga = torch.empty_like(p0)
    gb = torch.empty_like(p0)
    for step in range(2):
        roll, flip = _rolls(n, H, 10 + step)
        print(f"[step_aug] n={n} H={H} recompute={recompute} step {step}", flush=True)
        la = float(a.step(x, t, dparams=ga, roll=roll, flip=flip))
        xa, ta = augment(x, t, roll, flip)
        lb = float(b.step(xa, ta, dparams=gb))
        torch.cuda.synchronize()
        assert la == lb, (step, la, lb)
        assert torch.equal(ga, gb), step
        assert torch.equal(a.params, b.params) and torch.equal(a.m, b.m) and torch.equal(a.v, b.v), step
    # the augmentation changed the step (an identity roll everywhere would not)
    c = Trainer(CAE("bf16", device=DEV, recompute=recompute), p0.clone())
    c.step(x, t)
    c.step(x, t)
    assert not torch.equal(c.params, a.params)


def test_step_aug_unsupported_forms():
    from paper_1910_02480_amd.cae import CAE, Trainer
    p0 = torch.from_numpy(synth.init_params(0)).to(DEV)
    roll, flip = _rolls(4, 16, 1)
    cases = [(CAE("f32", device=DEV), 32), (CAE("bf16", device=DEV), 16), (CAE("bf16", device=DEV, circular=True), 32)]
    off = CAE("bf16", device=DEV)
    off.set_fused(False)
    cases.append((off, 64))
    for cae, H in cases:
        xs, ts = synth.training_batch(4, H)
        tr = Trainer(cae, p0.clone())
        with pytest.raises(B.DrcError) as e:
            tr.step(torch.from_numpy(xs).to(DEV), torch.from_numpy(ts).to(DEV), roll=roll, flip=flip)
        assert e.value.status == 3, str(e.value)
        assert torch.equal(tr.params, p0)

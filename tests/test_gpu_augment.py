"""Training augmentation on the GPU against the FP64 oracle (Sec. 5 rotations
and flips read as azimuth rotations and mirrors of the hemispherical map).

Moved values (R, G, B, Nz, D, targets) must be bit-exact copies. The rotated
normal components carry the FP32 sine and cosine of 2 pi k / W (a few ulp
each) and two products and a sum: within 8 ulp(1) = 9.5e-7 of the exact
value for normals of length <= 1.
"""
import numpy as np
import pytest
import torch

from oracle import augment as A
from paper_1910_02480_amd import binding as B
from paper_1910_02480_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
ATOL = 8 * 2.0 ** -23


def _gpu(x, t, roll, flip):
    n, H, W, _ = x.shape
    xd = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(DEV)
    td = None if t is None else torch.from_numpy(np.ascontiguousarray(t, dtype=np.float32)).to(DEV)
    rd = torch.tensor(np.asarray(roll, dtype=np.int32), device=DEV)
    fd = torch.tensor(np.asarray(flip, dtype=np.int32), device=DEV)
    xo = torch.full_like(xd, float("nan"))
    to = None if td is None else torch.full_like(td, float("nan"))
    print(f"[augment] n={n} H={H} W={W}", flush=True)
    B.drc_augment(xd, td, rd, fd, xo, to)
    torch.cuda.synchronize()
    return xo.cpu().numpy(), None if to is None else to.cpu().numpy()


def _check(x, t, roll, flip):
    xo, to = _gpu(x, t, roll, flip)
    ro, rt = A.augment(x.astype(np.float64), None if t is None else t.astype(np.float64), roll, flip)
    exact = [0, 1, 2, 5, 6]
    np.testing.assert_array_equal(xo[..., exact], ro[..., exact].astype(np.float32))
    np.testing.assert_allclose(xo[..., 3:5], ro[..., 3:5], atol=ATOL, rtol=0)
    if t is not None:
        np.testing.assert_array_equal(to, rt.astype(np.float32))


@pytest.mark.parametrize("n,H,W", [(6, 64, 64), (5, 32, 32), (3, 7, 5), (2, 1, 1), (2, 128, 128), (4, 8, 100)])
def test_augment_matches_oracle(n, H, W):
    x, t = synth.training_batch(n, H, W)
    rng = np.random.default_rng(n * 1000 + W)
    roll = rng.integers(-3 * W, 3 * W, n)
    flip = rng.integers(0, 2, n)
    roll[0], flip[0] = 0, 0              # identity
    roll[1 % n], flip[1 % n] = W, 1      # a full turn, mirrored
    _check(x, t, roll, flip)


def test_augment_without_targets_and_quarter_turns():
    x, _ = synth.training_batch(4, 16, 16)
    _check(x, None, [4, 8, 12, -4], [0, 0, 1, 1])


def test_full_batch_256x64x64():
    """The bench's batch: 256 training maps of 64 x 64, every map checked."""
    x, t = synth.training_batch(256, 64, 64)
    rng = np.random.default_rng(7)
    _check(x, t, rng.integers(0, 64, 256), rng.integers(0, 2, 256))

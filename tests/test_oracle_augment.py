"""Pins of the FP64 augmentation oracle (Sec. 5 rotation and flipping, read
as azimuth rotations and mirrors of the hemispherical map): group laws,
geometry of the moved directions, and values that must not change."""
import numpy as np
import pytest

from oracle import augment as A
from paper_1910_02480_amd import synth


def _maps(n=3, H=8, W=12):
    x = synth.radiance_maps(n, H, W).astype(np.float64)
    t = np.random.default_rng(0).random((n, H, W, 3))
    return x, t


def _dirs(H, W):
    th = (np.arange(H) + 0.5) * np.pi / (2 * H)
    ph = (np.arange(W) + 0.5) * 2 * np.pi / W
    T, P = np.meshgrid(th, ph, indexing="ij")
    return np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], -1)


def test_identity_and_full_turn():
    x, t = _maps()
    for k in (0, 12, -24):
        xo, to = A.augment(x, t, [k] * 3, [0] * 3)
        np.testing.assert_allclose(xo, x, atol=1e-14)
        np.testing.assert_array_equal(to, t)


def test_group_laws():
    x, t = _maps()
    n, H, W, _ = x.shape
    # two rolls add up
    a, _ = A.augment(*A.augment(x, t, [3, 5, 7], [0] * 3), [4, 2, 11], [0] * 3)
    b, _ = A.augment(x, t, [7, 7, 18], [0] * 3)
    np.testing.assert_allclose(a, b, atol=1e-13)
    # a mirror is its own inverse, for any k
    for k in (0, 5):
        m1, tt = A.augment(x, t, [k] * n, [1] * n)
        m2, t2 = A.augment(m1, tt, [k] * n, [1] * n)
        np.testing.assert_allclose(m2, x, atol=1e-13)
        np.testing.assert_array_equal(t2, t)
    # roll k then mirror 0 = mirror k
    r, tr = A.augment(x, t, [4] * n, [0] * n)
    f1, t1 = A.augment(r, tr, [0] * n, [1] * n)
    f2, t2 = A.augment(x, t, [-4] * n, [1] * n)
    np.testing.assert_allclose(f1, f2, atol=1e-13)
    np.testing.assert_array_equal(t1, t2)


@pytest.mark.parametrize("k,flip", [(0, 0), (3, 0), (5, 1), (0, 1), (11, 1)])
def test_map_of_its_own_directions_stays_consistent(k, flip):
    # A map whose normal channel holds each pixel's own view direction is
    # carried onto itself: the moved vectors still point at their pixels.
    H, W = 6, 12
    d = _dirs(H, W)
    x = np.zeros((1, H, W, 7))
    x[0, ..., 3:6] = d
    x[0, ..., 0] = np.arange(W)[None, :]     # column tag in R
    xo, _ = A.augment(x, None, [k], [flip])
    np.testing.assert_allclose(xo[0, ..., 3:6], d, atol=1e-13)
    # the column tag moved to the documented column
    u = np.arange(W)
    dst = (u + k) % W if not flip else (k - 1 - u) % W
    np.testing.assert_array_equal(xo[0, 0, dst, 0], u)


def test_values_that_do_not_change():
    x, t = _maps()
    xo, to = A.augment(x, t, [1, 6, 9], [1, 0, 1])
    # per row, R G B Nz D and the targets are permutations of the input row
    for m in range(3):
        for v in range(x.shape[1]):
            for c in (0, 1, 2, 5, 6):
                np.testing.assert_array_equal(np.sort(xo[m, v, :, c]), np.sort(x[m, v, :, c]))
            np.testing.assert_array_equal(np.sort(to[m, v].ravel()), np.sort(t[m, v].ravel()))
    # rotations and mirrors keep the length of the normals (per row, as multisets)
    np.testing.assert_allclose(np.sort(np.linalg.norm(xo[..., 3:6], axis=-1), axis=-1),
                               np.sort(np.linalg.norm(x[..., 3:6], axis=-1), axis=-1), rtol=1e-14)
    # a quarter turn maps (Nx, Ny) to (-Ny, Nx)
    q, _ = A.augment(x, None, [3, 3, 3], [0, 0, 0])
    W = x.shape[2]
    src = (np.arange(W) - 3) % W
    np.testing.assert_allclose(q[..., 3], -x[:, :, src, 4], atol=1e-15)
    np.testing.assert_allclose(q[..., 4], x[:, :, src, 3], atol=1e-15)

"""Pins of the FP64 interpolation-weight oracle (Sec. 4.2, Eqs. 4-6, with
the prose's reading of Eqs. 5 and 6) against hand-computed special cases,
symmetry and brute force."""
import numpy as np
import pytest

from oracle import interp as I


def _flat(Hi, Wi, r, n=(0.0, 0.0, 1.0)):
    Gy, Gx = I.grid_shape(Hi, Wi, r)
    return np.broadcast_to(np.array(n), (Hi, Wi, 3)).copy(), np.broadcast_to(np.array(n), (Gy, Gx, 3)).copy()


def test_pixel_on_a_cache_point():
    # Aligned normals: the cache point under the pixel has w_p = 1, w_n = 1,
    # w = 2 + eps; the other three corners are a grid spacing or more away
    # (w_p = 0), w = eps.
    r, eps = 4, 1e-3
    n, cn = _flat(9, 9, r)
    idx, prob = I.weights(n, r, cn, eps)
    Gx = 3
    assert list(idx[4, 4]) == [1 * Gx + 1, 1 * Gx + 2, 2 * Gx + 1, 2 * Gx + 2]
    tot = 2 + 4 * eps
    np.testing.assert_allclose(prob[4, 4], [(2 + eps) / tot, eps / tot, eps / tot, eps / tot], rtol=1e-14)


def test_cell_centre_is_symmetric():
    r = 4
    n, cn = _flat(9, 9, r)
    _, prob = I.weights(n, r, cn, 1e-4)
    np.testing.assert_allclose(prob[2, 2], 0.25, rtol=1e-14)
    # w_p = 1 - sqrt(8) / 4 at each corner; aligned normals double it
    wp = 1 - np.sqrt(8) / 4
    assert wp > 0


def test_hand_computed_weights():
    # pixel (x=1, y=0), r = 4: corners (0,0) at distance 1, (1,0) at 3,
    # (0,1) at sqrt(17) > 4, (1,1) at 5; cache normals tilted.
    r, eps = 4, 0.01
    n, cn = _flat(9, 9, r)
    cn[0, 0] = (0.0, 0.6, 0.8)     # dot with +Z: 0.8
    cn[0, 1] = (0.0, 0.0, -2.0)    # opposite: w_n = 0
    idx, prob = I.weights(n, r, cn, eps)
    w = np.array([0.75 * 0.8 + 0.75 + eps, 0.25 * 0.0 + 0.25 + eps, eps, eps])
    np.testing.assert_allclose(prob[0, 1], w / w.sum(), rtol=1e-14)


def test_image_edges_and_degenerate_normals():
    r = 4
    Hi, Wi = 7, 10                 # grid 2 x 3: corners beyond x = 8 or y = 4 are absent
    n, cn = _flat(Hi, Wi, r)
    idx, prob = I.weights(n, r, cn, 1e-3)
    assert list(idx[6, 9]) == [1 * 3 + 2, -1, -1, -1]
    np.testing.assert_allclose(prob[6, 9], [1.0, 0, 0, 0])
    assert np.all(prob[idx < 0] == 0)
    np.testing.assert_allclose(prob.sum(-1), 1.0, rtol=1e-14)
    # zero-length pixel normal: w_n = 0, so only w_p + eps remains
    n[1, 1] = 0.0
    _, p0 = I.weights(n, r, cn, 0.0)
    d = np.hypot([1, 3, 1, 3], [1, 1, 3, 3])
    wp = np.maximum(0, 1 - d / r)
    np.testing.assert_allclose(p0[1, 1], wp / wp.sum(), rtol=1e-14)
    # every weight zero (eps = 0, pixel a grid spacing or more from its only corner)
    n, cn = _flat(8, 8, 8)
    _, p1 = I.weights(n, 8, cn, 0.0)
    np.testing.assert_allclose(p1[7, 7], [1.0, 0, 0, 0])


def test_neighbourhood_holds_every_point_with_positive_position_weight():
    # brute force over all cache points: every point closer than r lies
    # among the four corners, and the corners' probabilities follow Eq. 4.
    rng = np.random.default_rng(0)
    Hi, Wi, r, eps = 11, 13, 3, 1e-3
    Gy, Gx = I.grid_shape(Hi, Wi, r)
    n = rng.standard_normal((Hi, Wi, 3))
    cn = rng.standard_normal((Gy, Gx, 3))
    idx, prob = I.weights(n, r, cn, eps)
    for y in range(Hi):
        for x in range(Wi):
            w = {}
            for gy in range(Gy):
                for gx in range(Gx):
                    d = np.hypot(x - gx * r, y - gy * r)
                    if d < r:
                        assert gy * Gx + gx in idx[y, x]
                    if gy * Gx + gx in idx[y, x]:
                        a = n[y, x] / np.linalg.norm(n[y, x])
                        b = cn[gy, gx] / np.linalg.norm(cn[gy, gx])
                        wp = max(0.0, 1 - d / r)
                        w[gy * Gx + gx] = wp * max(0.0, a @ b) + wp + eps
            tot = sum(w.values())
            for k in range(4):
                if idx[y, x, k] >= 0:
                    assert abs(prob[y, x, k] - w[idx[y, x, k]] / tot) < 1e-14

"""FP64 oracle of the interpolation weights between cache points (Sec. 4.2,
Eqs. 4-6): per image pixel, the probability of sampling each nearby cache
point's radiance map.

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU
baseline leg use it to check and time the HIP path; the product path never
imports it. It shares no code with the HIP library.

Readings (the printed formulas and the prose disagree; the prose is taken):
* position weight w_p = max(0, 1 - dist / r): largest at the cache point and
  zero one grid spacing away (Eq. 5 prints dist / r, which would grow with
  distance);
* normal weight w_n = max(0, n_i . n) of the unit normals: maximal when the
  normals agree and zero when their dot product is negative, as the prose
  says (Eq. 6 prints one minus that); a zero-length normal gives 0;
* w = w_p w_n + w_p + eps (Eq. 4), over the four cache points at the
  corners of the grid cell holding the pixel (the only ones where w_p can be
  non-zero) that lie inside the image; the weights are normalised to
  probabilities, and if they all vanish (eps = 0) the present corners are
  equally likely.
Grid: cache point (gy, gx) sits on pixel (gx r, gy r), for every such pixel
inside the Hi x Wi image; distances are in pixels between integer pixel
coordinates. Corner k of pixel (x, y) is (x // r + (k & 1), y // r + (k >> 1));
absent corners get index -1 and probability 0.
"""
from __future__ import annotations

import numpy as np


def grid_shape(Hi, Wi, r):
    return (Hi - 1) // r + 1, (Wi - 1) // r + 1


def _unit(n):
    n = np.asarray(n, dtype=np.float64)
    ln = np.linalg.norm(n, axis=-1, keepdims=True)
    return np.where(ln > 0, n / np.where(ln > 0, ln, 1.0), 0.0)


def weights(normals, r, cache_normals, eps):
    """normals [Hi, Wi, 3], cache_normals [Gy, Gx, 3] -> (idx [Hi, Wi, 4]
    int64 = gy * Gx + gx or -1, prob [Hi, Wi, 4] float64)."""
    Hi, Wi, _ = normals.shape
    Gy, Gx = grid_shape(Hi, Wi, r)
    assert cache_normals.shape[:2] == (Gy, Gx)
    n = _unit(normals)
    cn = _unit(cache_normals).reshape(-1, 3)
    y, x = np.meshgrid(np.arange(Hi), np.arange(Wi), indexing="ij")
    idx = np.full((Hi, Wi, 4), -1, dtype=np.int64)
    w = np.zeros((Hi, Wi, 4))
    for k in range(4):
        gx = x // r + (k & 1)
        gy = y // r + (k >> 1)
        ok = (gx < Gx) & (gy < Gy)
        dist = np.hypot(x - gx * r, y - gy * r)
        wp = np.maximum(0.0, 1.0 - dist / r)
        i = np.where(ok, gy * Gx + gx, 0)
        wn = np.maximum(0.0, np.einsum("hwc,hwc->hw", cn[i], n))
        w[..., k] = np.where(ok, wp * wn + wp + eps, 0.0)
        idx[..., k] = np.where(ok, i, -1)
    tot = w.sum(-1, keepdims=True)
    present = (idx >= 0).astype(np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        prob = np.where(tot > 0, w / np.where(tot > 0, tot, 1.0), present / present.sum(-1, keepdims=True))
    return idx, prob

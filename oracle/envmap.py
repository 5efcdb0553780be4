"""FP64 oracle of the step after the autoencoder: sampling the predicted
radiance map R as an environment map (Sec. 3, the multiple-importance-
sampling paragraph after Eq. 2; map projection of Sec. 4.3).

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU
baseline leg use it to check and time the HIP path; the product path never
imports it. It shares no code with the HIP library.

What is computed, per map of H rows x W columns (NHWC, 3 channels R, G, B):

* The map is a hemispherical latitude-longitude projection with the surface
  normal along +Z (Sec. 4.3). Row v spans polar angles
  [v, v + 1] * (pi/2) / H from the normal (row 0 at the zenith); column u
  spans azimuths [u, u + 1] * 2 pi / W.
* Pixel weight f[v, u] = max(0, Y(R[v, u])) * sin(theta_v), with Y the
  luminance of ITU-R BT.709 primaries (0.2126 R + 0.7152 G + 0.0722 B) and
  theta_v the polar angle of the row centre: a piecewise-constant density
  over the (u, v) unit square whose mass per pixel is proportional to
  luminance times the pixel's solid angle.
* Marginal distribution over rows (row sums of f) and one conditional
  distribution over columns per row, both as inclusive CDFs (the value at
  index k is the probability of indices 0..k). A row (or map) whose weights
  all vanish gets the uniform CDF (k + 1) / n.
* Sampling by inversion: xi1 picks the row, xi2 the column within it, and the
  fractional position inside the chosen pixel is the linear interpolation
  of the CDF, so (u_c, v_c) is distributed with the piecewise-constant
  density p(u_c, v_c) = p(v) p(u | v) H W.
* Direction in the map frame: theta = v_c pi / 2, phi = u_c 2 pi,
  d = (sin theta cos phi, sin theta sin phi, cos theta); its density with
  respect to solid angle is p(u_c, v_c) / (pi^2 sin theta), since
  d omega = sin theta d theta d phi = pi^2 sin theta du dv.

Random numbers are inputs (xi in [0, 1)).
"""
from __future__ import annotations

import numpy as np

# ITU-R BT.709 relative luminance of linear R, G, B
LUMA = (0.2126, 0.7152, 0.0722)


def pixel_weights(rgb):
    """f[n, v, u] = max(0, luminance) * sin(row-centre polar angle), float64."""
    rgb = np.asarray(rgb, dtype=np.float64)
    n, H, W, c = rgb.shape
    assert c == 3
    lum = LUMA[0] * rgb[..., 0] + LUMA[1] * rgb[..., 1] + LUMA[2] * rgb[..., 2]
    theta = (np.arange(H) + 0.5) * (np.pi / 2) / H
    return np.maximum(lum, 0.0) * np.sin(theta)[None, :, None]


def _inclusive_cdf(w, axis):
    """Inclusive CDF along an axis of non-negative weights; uniform where all vanish."""
    w = np.moveaxis(w, axis, -1)
    k = w.shape[-1]
    s = np.cumsum(w, axis=-1)
    tot = s[..., -1:]
    uni = np.broadcast_to((np.arange(k) + 1.0) / k, s.shape)
    with np.errstate(invalid="ignore", divide="ignore"):
        cdf = np.where(tot > 0, s / np.where(tot > 0, tot, 1.0), uni)
    return np.moveaxis(cdf, -1, axis), tot[..., 0]


def build(rgb):
    """Sampling tables of each map.

    Returns (cdf_u [n, H, W], cdf_v [n, H], total [n]): conditional column
    CDFs per row, the marginal row CDF, and the sum of all pixel weights
    (0 means the whole map fell back to the uniform distribution).
    """
    f = pixel_weights(rgb)
    cdf_u, rowsum = _inclusive_cdf(f, axis=2)
    cdf_v, total = _inclusive_cdf(rowsum, axis=1)
    return cdf_u, cdf_v, total


def _probs(cdf):
    """Per-index probabilities from an inclusive CDF (last axis)."""
    return np.diff(cdf, axis=-1, prepend=0.0)


def _invert(cdf, xi):
    """Index k with cdf[k-1] <= xi < cdf[k] and the fraction of xi inside it."""
    k = int(np.searchsorted(cdf, xi, side="right"))
    k = min(k, len(cdf) - 1)
    lo = cdf[k - 1] if k > 0 else 0.0
    p = cdf[k] - lo
    frac = (xi - lo) / p if p > 0 else 0.0
    return k, min(max(frac, 0.0), 1.0), p


def sample(cdf_u, cdf_v, xi):
    """Directions sampled from each map.

    xi: [n, S, 2] uniforms in [0, 1). Returns (dir [n, S, 3], pdf [n, S]
    with respect to solid angle, pix [n, S] = v * W + u). Pure-Python loop
    over samples: for small cases.
    """
    cdf_u = np.asarray(cdf_u, dtype=np.float64)
    cdf_v = np.asarray(cdf_v, dtype=np.float64)
    xi = np.asarray(xi, dtype=np.float64)
    n, H, W = cdf_u.shape
    S = xi.shape[1]
    d = np.zeros((n, S, 3))
    pdf = np.zeros((n, S))
    pix = np.zeros((n, S), dtype=np.int64)
    for m in range(n):
        for s in range(S):
            v, fv, pv = _invert(cdf_v[m], xi[m, s, 0])
            u, fu, pu = _invert(cdf_u[m, v], xi[m, s, 1])
            theta = (v + fv) / H * (np.pi / 2)
            phi = (u + fu) / W * (2 * np.pi)
            st = np.sin(theta)
            d[m, s] = (st * np.cos(phi), st * np.sin(phi), np.cos(theta))
            pdf[m, s] = pv * pu * H * W / (np.pi ** 2 * st) if st > 0 else 0.0
            pix[m, s] = v * W + u
    return d, pdf, pix


def pdf(cdf_u, cdf_v, dirs):
    """Solid-angle density of directions dirs [n, S, 3] (map frame, any
    length) under each map's sampling distribution; 0 below the horizon
    (z < 0) and along the normal itself."""
    cdf_u = np.asarray(cdf_u, dtype=np.float64)
    cdf_v = np.asarray(cdf_v, dtype=np.float64)
    dirs = np.asarray(dirs, dtype=np.float64)
    n, H, W = cdf_u.shape
    x, y, z = dirs[..., 0], dirs[..., 1], dirs[..., 2]
    r = np.hypot(x, y)
    theta = np.arctan2(r, z)
    phi = np.mod(np.arctan2(y, x), 2 * np.pi)
    v = np.minimum((theta / (np.pi / 2) * H).astype(np.int64), H - 1)
    u = np.minimum((phi / (2 * np.pi) * W).astype(np.int64), W - 1)
    pv = _probs(cdf_v)
    pu = _probs(cdf_u)
    mi = np.arange(n)[:, None]
    p = pv[mi, v] * pu[mi, v, u] * H * W
    st = r / np.maximum(np.sqrt(r * r + z * z), 1e-300)
    with np.errstate(invalid="ignore", divide="ignore"):
        out = np.where((z >= 0) & (st > 0), p / (np.pi ** 2 * np.where(st > 0, st, 1.0)), 0.0)
    return out

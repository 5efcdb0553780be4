"""FP64 oracle of the training-data augmentation (Sec. 5: the data loader
applies combinations of rotation and flipping to the training maps).

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU
baseline leg use it to check and time the HIP path; the product path never
imports it. It shares no code with the HIP library.

Reading: on a hemispherical lat-long map (normal along +Z, Sec. 4.3) the
rotations and flips that keep the map physical are the rotations about the
normal and the mirror images through a plane containing it; a rotation that
moved the zenith (a vertical flip, say) would put the horizon at the top.
So a map is transformed by an azimuth map phi -> s phi + alpha with
s = +1 or -1 (flip) and alpha = 2 pi k / W (a whole number k of columns):
* pixels move: the value at column u goes to column (u + k) mod W, or
  (k - 1 - u) mod W when flipped (the column centres (u + 1/2) 2 pi / W map
  onto column centres);
* vector channels move with the scene: a normal with azimuth psi gets
  azimuth s psi + alpha, i.e. (Nx, Ny) is reflected (Ny -> -Ny) when
  flipped and then rotated by alpha; Nz, radiance and distance keep their
  values (normals are read as expressed in the map's frame);
* the target map (RGB) moves with its input.
"""
from __future__ import annotations

import numpy as np


def augment(x, t, roll, flip):
    """x [n, H, W, 7] (R, G, B, Nx, Ny, Nz, D), t [n, H, W, 3] or None,
    roll [n] integers (any value; taken mod W), flip [n] in {0, 1}.
    Returns (x_out, t_out) as float64."""
    x = np.asarray(x, dtype=np.float64)
    n, H, W, C = x.shape
    assert C == 7
    xo = np.empty_like(x)
    to = None if t is None else np.empty(np.shape(t), dtype=np.float64)
    for m in range(n):
        k = int(roll[m]) % W
        s = -1 if flip[m] else 1
        u = np.arange(W)
        dst = (u + k) % W if s > 0 else (k - 1 - u) % W
        src = x[m]
        a = 2.0 * np.pi * k / W
        nx, ny = src[..., 3], s * src[..., 4]
        moved = src.copy()
        moved[..., 3] = np.cos(a) * nx - np.sin(a) * ny
        moved[..., 4] = np.sin(a) * nx + np.cos(a) * ny
        xo[m][:, dst] = moved
        if to is not None:
            to[m][:, dst] = np.asarray(t[m], dtype=np.float64)
    return xo, to

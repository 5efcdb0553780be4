"""Seeded synthetic workloads for the radiance-cache autoencoder.

This module only draws random numbers and lays them out. It contains none of
the autoencoder's arithmetic, so it may feed both the HIP path and the FP64
oracle with identical FP32 arrays.

Stand-ins. The paper's training set (43 scenes, 16 000 map pairs; Sec. 5)
and its trained weights are not available, so every input here is synthetic,
with the shapes and value structure the paper describes:

* a cache point's input map has 7 channels in the order R, G, B, Nx, Ny, Nz,
  D (Sec. 4.3, network inputs) and the output map has 3 (R, G, B);
* 1-spp radiance maps are mostly dark with a few very bright pixels
  (Sec. 6.1), modelled as a lognormal with rare x100 "fireflies" and
  compressed with log1p;
* normals are unit vectors, distances are positive.

Every map ``m`` of a workload is drawn from its own generator
``numpy.random.default_rng([seed, m])`` (PCG64), so any subset of a large
batch can be regenerated exactly without generating the rest.
"""
from __future__ import annotations

import numpy as np

IN_CH = 7
OUT_CH = 3

# Layer shapes used for parameter initialisation (fan-in only).
# (name, input channels, output channels); every layer has a 3x3 kernel.
_INIT_LAYERS = (
    ("E1", 7, 32),
    ("E2", 32, 64),
    ("E3", 64, 128),
    ("D3", 128, 64),
    ("D2", 128, 32),
    ("D1", 64, 3),
)

SEED_WEIGHTS = 0
SEED_MAPS = 1
SEED_MIXED_PERM = 2
SEED_TRAIN = 3
SEED_ENVMAP = 4
SEED_GBUFFER = 5
SEED_UNET = 6


def param_count() -> int:
    return sum(co * 9 * ci + co for _, ci, co in _INIT_LAYERS)


def init_params(seed: int = SEED_WEIGHTS) -> np.ndarray:
    """Flat FP32 parameter vector, layers in order E1 E2 E3 D3 D2 D1.

    Each layer is its weight ``W[co][kh][kw][ci]`` (C order) followed by its
    bias ``b[co]``. Weights are Kaiming-normal with std sqrt(2 / (9 Cin)) for
    convolutions and transposed convolutions alike; biases are uniform in
    +-1/sqrt(9 Cin) so that the bias path is exercised. Values are drawn in
    float64 and cast to float32.
    """
    rng = np.random.default_rng(seed)
    parts = []
    for _, ci, co in _INIT_LAYERS:
        fan_in = 9 * ci
        w = rng.standard_normal((co, 3, 3, ci)) * np.sqrt(2.0 / fan_in)
        bound = 1.0 / np.sqrt(fan_in)
        b = rng.uniform(-bound, bound, size=(co,))
        parts.append(w.reshape(-1))
        parts.append(b)
    return np.concatenate(parts).astype(np.float32)


def _unit_normals(rng, h, w):
    g = rng.standard_normal((h, w, 3))
    return g / np.linalg.norm(g, axis=-1, keepdims=True)


def radiance_map(m: int, h: int, w: int, seed: int = SEED_MAPS,
                 firefly_p: float = 0.02) -> np.ndarray:
    """One noisy 1-spp cache-point map, float32 [h, w, 7].

    Draw order: RGB lognormal(mu=-1, sigma=1.5) [h,w,3]; firefly mask
    Bernoulli(p) [h,w] (all three RGB samples of a firefly pixel x100);
    distance U[0.1, 10] [h,w]; Gaussian [h,w,3] normalised to the unit
    sphere. RGB is stored as log1p of the radiance.
    """
    rng = np.random.default_rng([seed, m])
    rgb = rng.lognormal(mean=-1.0, sigma=1.5, size=(h, w, 3))
    fire = rng.random((h, w)) < firefly_p
    rgb[fire] *= 100.0
    rgb = np.log1p(rgb)
    dist = rng.uniform(0.1, 10.0, size=(h, w))
    nrm = _unit_normals(rng, h, w)
    out = np.empty((h, w, IN_CH), dtype=np.float32)
    out[..., 0:3] = rgb
    out[..., 3:6] = nrm
    out[..., 6] = dist
    return out


def radiance_maps(n: int, h: int, w: int | None = None, seed: int = SEED_MAPS,
                  start: int = 0) -> np.ndarray:
    """Maps ``start .. start+n-1`` of a workload, float32 NHWC [n, h, w, 7]."""
    w = h if w is None else w
    out = np.empty((n, h, w, IN_CH), dtype=np.float32)
    for k in range(n):
        out[k] = radiance_map(start + k, h, w, seed)
    return out


def _lobe_target(rng, h, w):
    """Smooth target: sum of 8 random cosine lobes on the upper hemisphere.

    Lat-long parameterisation of the hemisphere (normal along +Z):
    theta_i = (i + 1/2)/h * pi/2, phi_j = (j + 1/2)/w * 2 pi.
    """
    d = rng.standard_normal((8, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    d[:, 2] = np.abs(d[:, 2])
    e = rng.uniform(1.0, 8.0, size=(8,))
    a = rng.uniform(0.0, 1.0, size=(8, 3))
    th = (np.arange(h) + 0.5) / h * (np.pi / 2)
    ph = (np.arange(w) + 0.5) / w * (2 * np.pi)
    st, ct = np.sin(th)[:, None], np.cos(th)[:, None]
    omega = np.stack([st * np.cos(ph)[None, :], st * np.sin(ph)[None, :],
                      np.broadcast_to(ct, (h, w))], axis=-1)  # [h,w,3]
    cosang = np.maximum(omega @ d.T, 0.0)                       # [h,w,8]
    return (cosang ** e[None, None, :]) @ a                      # [h,w,3]


def training_pair(m: int, h: int, w: int, seed: int = SEED_TRAIN):
    """One (input [h,w,7], target [h,w,3]) float32 training pair.

    Draw order: lobes (directions, exponents, amplitudes); Gamma(k=4, theta=1)
    noise [h,w,3]; 1 % firefly mask [h,w]; distance; normals. Input RGB is
    target * G / 4 (x100 on firefly pixels); log1p is applied to the input RGB
    and to the target.
    """
    rng = np.random.default_rng([seed, m])
    t = _lobe_target(rng, h, w)
    g = rng.gamma(shape=4.0, scale=1.0, size=(h, w, 3))
    noisy = t * g / 4.0
    fire = rng.random((h, w)) < 0.01
    noisy[fire] *= 100.0
    dist = rng.uniform(0.1, 10.0, size=(h, w))
    nrm = _unit_normals(rng, h, w)
    x = np.empty((h, w, IN_CH), dtype=np.float32)
    x[..., 0:3] = np.log1p(noisy)
    x[..., 3:6] = nrm
    x[..., 6] = dist
    return x, np.log1p(t).astype(np.float32)


def training_batch(n: int, h: int, w: int | None = None, seed: int = SEED_TRAIN,
                   start: int = 0):
    w = h if w is None else w
    x = np.empty((n, h, w, IN_CH), dtype=np.float32)
    t = np.empty((n, h, w, OUT_CH), dtype=np.float32)
    for k in range(n):
        x[k], t[k] = training_pair(start + k, h, w, seed)
    return x, t


def predicted_map(m: int, h: int, w: int, seed: int = SEED_ENVMAP, noise: float = 0.05) -> np.ndarray:
    """A stand-in for one denoised output map, float32 [h, w, 3].

    Draw order: lobes as in ``training_pair`` (log1p applied), then Gaussian
    noise of standard deviation ``noise`` [h,w,3]. The noise lets a few
    values dip below zero, as the linear output layer's can.
    """
    rng = np.random.default_rng([seed, m])
    t = np.log1p(_lobe_target(rng, h, w))
    t += noise * rng.standard_normal((h, w, 3))
    return t.astype(np.float32)


def predicted_maps(n: int, h: int, w: int | None = None, seed: int = SEED_ENVMAP,
                   start: int = 0) -> np.ndarray:
    w = h if w is None else w
    out = np.empty((n, h, w, OUT_CH), dtype=np.float32)
    for k in range(n):
        out[k] = predicted_map(start + k, h, w, seed)
    return out


def gbuffer_normals(hi: int, wi: int, seed: int = SEED_GBUFFER, background: float = 0.05) -> np.ndarray:
    """Primary-hit normals of an hi x wi image, float32 [hi, wi, 3].

    A smooth height field z(x, y) (sum of 6 random sinusoids) gives the
    unit normals (-dz/dx, -dz/dy, 1) / norm; then a random ``background``
    fraction of pixels (rays that hit nothing) gets the zero vector.
    Draw order: amplitudes [6], frequencies [6, 2], phases [6], background
    mask [hi, wi].
    """
    rng = np.random.default_rng(seed)
    amp = rng.uniform(0.2, 1.0, 6)
    freq = rng.uniform(0.002, 0.05, (6, 2))
    ph = rng.uniform(0.0, 2 * np.pi, 6)
    y, x = np.meshgrid(np.arange(hi, dtype=np.float64), np.arange(wi, dtype=np.float64), indexing="ij")
    dzdx = np.zeros((hi, wi))
    dzdy = np.zeros((hi, wi))
    for k in range(6):
        c = amp[k] * np.cos(freq[k, 0] * x + freq[k, 1] * y + ph[k]) * 20.0
        dzdx += c * freq[k, 0]
        dzdy += c * freq[k, 1]
    n = np.stack([-dzdx, -dzdy, np.ones_like(dzdx)], -1)
    n /= np.linalg.norm(n, axis=-1, keepdims=True)
    n[rng.random((hi, wi)) < background] = 0.0
    return n.astype(np.float32)


# The paper's own network (U-Net-like, Sec. 4.3 / 5): (name, cin, cout,
# batch norm) in execution order, widths 64-128-256 with a 256-channel 4x4
# bottleneck; "out" is the 1x1 output convolution.
UNET_LAYERS = (
    ("enc1a", 7, 64, True), ("enc1b", 64, 64, True),
    ("enc2a", 64, 128, True), ("enc2b", 128, 128, True),
    ("enc3a", 128, 256, True), ("enc3b", 256, 256, True),
    ("mid_a", 256, 256, True), ("mid_b", 256, 256, True),
    ("dec3a", 512, 256, True), ("dec3b", 256, 256, True),
    ("dec2a", 384, 128, True), ("dec2b", 128, 128, True),
    ("dec1a", 192, 64, False), ("dec1b", 64, 64, False),
    ("out", 64, 3, False),
)


def unet_params(seed: int = SEED_UNET):
    """Random-init parameters of the U-Net, float32: a list of per-layer
    dicts {"w": [Cout, 3, 3, Cin] ([Cout, Cin] for the 1x1), "b": [Cout],
    and for batch-normalised layers "gamma", "beta", "mean", "var"}.

    Draw order per layer: w Kaiming-normal (std sqrt(2 / fan_in)), b
    U(+-1/sqrt(fan_in)), then gamma U[0.8, 1.2], beta U[-0.1, 0.1], mean
    U[-0.1, 0.1], var U[0.5, 1.5] (so that batch norm is not the identity).
    """
    rng = np.random.default_rng(seed)
    out = []
    for name, ci, co, bn in UNET_LAYERS:
        k = 1 if name == "out" else 9
        fan = k * ci
        w = rng.standard_normal((co, ci) if k == 1 else (co, 3, 3, ci)) * np.sqrt(2.0 / fan)
        d = {"w": w.astype(np.float32), "b": rng.uniform(-1, 1, co).astype(np.float32) / np.float32(np.sqrt(fan))}
        if bn:
            d["gamma"] = rng.uniform(0.8, 1.2, co).astype(np.float32)
            d["beta"] = rng.uniform(-0.1, 0.1, co).astype(np.float32)
            d["mean"] = rng.uniform(-0.1, 0.1, co).astype(np.float32)
            d["var"] = rng.uniform(0.5, 1.5, co).astype(np.float32)
        out.append(d)
    return out


def unet_flat(params) -> np.ndarray:
    """The flat float32 parameter vector of the U-Net: per layer W (C order),
    b, then gamma, beta, mean, var for batch-normalised layers."""
    parts = []
    for q in params:
        parts += [q["w"].reshape(-1), q["b"]]
        if "gamma" in q:
            parts += [q["gamma"], q["beta"], q["mean"], q["var"]]
    return np.concatenate(parts).astype(np.float32)


# Mixed-resolution frame: 50 % 32x32, 35 % 64x64, 15 % 128x128, shuffled.
MIXED_FRACTIONS = ((32, 0.50), (64, 0.35), (128, 0.15))


def mixed_resolutions(count: int = 6000, seed: int = SEED_MIXED_PERM) -> np.ndarray:
    """Per-map square resolution of a mixed frame, shuffled by ``seed``."""
    sizes = []
    remaining = count
    for k, (res, frac) in enumerate(MIXED_FRACTIONS):
        c = remaining if k == len(MIXED_FRACTIONS) - 1 else int(round(count * frac))
        sizes += [res] * c
        remaining -= c
    sizes = np.asarray(sizes, dtype=np.int32)
    rng = np.random.default_rng(seed)
    return sizes[rng.permutation(count)]


def mixed_frame(resolutions, seed: int = SEED_MAPS):
    """Packed NHWC input for a mixed frame.

    Returns (x_packed float32 [sum h*w*7], x_off int64 [count],
    y_off int64 [count]); offsets are element offsets of each map's first
    value in the packed input (7 ch) and output (3 ch) buffers.
    """
    res = np.asarray(resolutions, dtype=np.int64)
    pix = res * res
    x_off = np.concatenate([[0], np.cumsum(pix * IN_CH)[:-1]]).astype(np.int64)
    y_off = np.concatenate([[0], np.cumsum(pix * OUT_CH)[:-1]]).astype(np.int64)
    x = np.empty(int(pix.sum()) * IN_CH, dtype=np.float32)
    for m, r in enumerate(res):
        x[x_off[m]:x_off[m] + pix[m] * IN_CH] = radiance_map(m, int(r), int(r), seed).reshape(-1)
    return x, x_off, y_off

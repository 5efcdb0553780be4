"""FP64 oracle of the paper's own network (Sec. 4.3 and Sec. 5): a U-Net-like
convolutional autoencoder, inference form.

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU
baseline leg use it to check and time the HIP path; the product path never
imports it. It shares no code with the HIP library.

Structure as the text describes it (its figure is missing), with this
build's readings:
* encoder stages at 32, 16 and 8 pixels (for a 32 x 32 input) with widths
  64, 128, 256: each two 3x3 convolutions (stride 1, zero padding 1), each
  followed by batch normalisation and LeakyReLU; a 2x2 max-pool between
  stages; the bottleneck stage at 4 x 4 (minimum hidden size 4 x 4, three
  downsizing steps, base width K = 64) keeps 256 channels, which makes the
  model 19.3 MB of float32 parameters, the size Sec. 5 states (doubling it
  to 512 would make 31 MB);
* decoder stages: 2x2 bilinear upsampling (half-pixel centres, edge
  clamped), concatenation [upsampled | skip] with the encoder output of the
  same size, two 3x3 "deconvolutions" (stride 1, padding 1; with stride 1 a
  transposed convolution is a convolution with a flipped kernel, so the
  weights are stored as a convolution's) with batch normalisation and
  LeakyReLU; the last stage (the output stage) has no batch normalisation;
* a 1x1 convolution to 3 channels with ReLU.
* LeakyReLU slope 0.01 and batch-norm eps 1e-5 (PyTorch's defaults, the
  framework of Sec. 5); batch norm at inference uses the running mean and
  variance: y = gamma (x - mean) / sqrt(var + eps) + beta.

Parameters: a list of per-layer dicts {"w": [Cout, 3, 3, Cin] or [Cout, Cin]
for the 1x1, "b": [Cout], and for batch-normalised layers "gamma", "beta",
"mean", "var": [Cout]}, in execution order. Maps are NHWC.
"""
from __future__ import annotations

import numpy as np

BASE = 64
SLOPE = 0.01
BN_EPS = 1e-5

# (name, cin, cout, batch norm) in execution order; "out" is the 1x1 output convolution
LAYERS = (
    ("enc1a", 7, 64, True), ("enc1b", 64, 64, True),
    ("enc2a", 64, 128, True), ("enc2b", 128, 128, True),
    ("enc3a", 128, 256, True), ("enc3b", 256, 256, True),
    ("mid_a", 256, 256, True), ("mid_b", 256, 256, True),
    ("dec3a", 512, 256, True), ("dec3b", 256, 256, True),
    ("dec2a", 384, 128, True), ("dec2b", 128, 128, True),
    ("dec1a", 192, 64, False), ("dec1b", 64, 64, False),
    ("out", 64, 3, False),
)


def num_params():
    total = 0
    for name, ci, co, bn in LAYERS:
        k = 1 if name == "out" else 9
        total += co * ci * k + co + (4 * co if bn else 0)
    return total


def conv3x3(x, w, b):
    """Stride-1 3x3 cross-correlation with zero padding 1: x [n,H,W,Ci],
    w [Co,3,3,Ci] -> [n,H,W,Co]; a sum over the 9 taps of shifted matmuls."""
    n, H, W, ci = x.shape
    xp = np.zeros((n, H + 2, W + 2, ci))
    xp[:, 1:H + 1, 1:W + 1] = x
    y = np.zeros((n, H, W, w.shape[0]))
    for kh in range(3):
        for kw in range(3):
            y += xp[:, kh:kh + H, kw:kw + W] @ w[:, kh, kw, :].T
    return y + b


def batch_norm(x, p):
    return p["gamma"] * (x - p["mean"]) / np.sqrt(p["var"] + BN_EPS) + p["beta"]


def leaky_relu(x):
    return np.where(x > 0, x, SLOPE * x)


def max_pool2(x):
    n, H, W, c = x.shape
    return x.reshape(n, H // 2, 2, W // 2, 2, c).max(axis=(2, 4))


def upsample2(x):
    """2x bilinear upsampling with half-pixel centres: output index i reads
    source coordinate (i + 1/2) / 2 - 1/2, clamped to [0, size - 1]."""
    def axis_weights(size):
        src = np.maximum((np.arange(2 * size) + 0.5) / 2 - 0.5, 0.0)
        i0 = np.minimum(np.floor(src).astype(int), size - 1)
        i1 = np.minimum(i0 + 1, size - 1)
        return i0, i1, src - i0
    n, H, W, c = x.shape
    r0, r1, fr = axis_weights(H)
    c0, c1, fc = axis_weights(W)
    rows = x[:, r0] * (1 - fr)[None, :, None, None] + x[:, r1] * fr[None, :, None, None]
    return rows[:, :, c0] * (1 - fc)[None, None, :, None] + rows[:, :, c1] * fc[None, None, :, None]


def forward(params, x):
    """x [n, H, W, 7] (H, W multiples of 8) -> y [n, H, W, 3], float64."""
    x = np.asarray(x, dtype=np.float64)
    p = iter([{k: np.asarray(v, dtype=np.float64) for k, v in q.items()} for q in params])

    def block(h, bn=True):
        q = next(p)
        h = conv3x3(h, q["w"], q["b"])
        return leaky_relu(batch_norm(h, q) if bn else h)

    s1 = block(block(x))
    s2 = block(block(max_pool2(s1)))
    s3 = block(block(max_pool2(s2)))
    m = block(block(max_pool2(s3)))
    d3 = block(block(np.concatenate([upsample2(m), s3], axis=-1)))
    d2 = block(block(np.concatenate([upsample2(d3), s2], axis=-1)))
    d1 = block(block(np.concatenate([upsample2(d2), s1], axis=-1), bn=False), bn=False)
    q = next(p)
    return np.maximum(d1 @ q["w"].T + q["b"], 0.0)

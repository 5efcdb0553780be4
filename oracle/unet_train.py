"""FP64 oracle of the paper's own network in its training form (Sec. 4.3 and
Sec. 5): batch-statistics batch normalisation, the L1 loss and the gradient
of every trainable parameter.

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU
baseline leg use it to check and time the HIP path; the product path never
imports it. It shares no code with the HIP library.

The network is the one of ``oracle.unet`` (same layer list and parameter
dicts). In training, a batch-normalised layer normalises its convolution
output z with the statistics of the batch, per channel over (n, H, W):
    mu = mean(z), var = mean((z - mu)^2)          (biased, as PyTorch)
    q  = gamma (z - mu) / sqrt(var + eps) + beta,  a = LeakyReLU(q)
and updates its running statistics with momentum 0.1 (PyTorch's
BatchNorm2d): mean <- 0.9 mean + 0.1 mu, var <- 0.9 var + 0.1 var_unbiased
(var_unbiased = var M / (M - 1), M = n H W). The loss is the mean L1
distance of the output to the target (Sec. 4.3's L1 in the mean form used
for the autoencoder). Trainable parameters: every w and b, and gamma, beta;
the running statistics get a zero gradient.

The backward pass is written out layer by layer from the definitions
(reverse mode):
* output: y = relu(d1 W^T + b): dy_pre = dL/dy [y > 0];
* convolution (3x3, zero padding 1, cross-correlation): dW[co, kh, kw, ci] =
  sum over pixels of dz[p, co] x[p + (kh - 1, kw - 1), ci], db = sum dz,
  dx = the same shifts read backwards (each tap scatters dz W into the
  input positions it read);
* LeakyReLU: derivative 1 where q > 0, else the slope (0.01);
* batch norm (xhat = (z - mu) / sqrt(var + eps), M = n H W):
  dgamma = sum dq xhat, dbeta = sum dq,
  dz = gamma / sqrt(var + eps) (dq - mean(dq) - xhat mean(dq xhat));
* max-pool: the gradient goes to the first maximum of each window in
  row-major order;
* branch conditioning (optional): the LeakyReLU branches, the max-pool
  choices, the output ReLU and the loss signs can be taken from another
  forward's activations (the GPU's), so that a lower-precision forward that
  lands on the other side of a kink is compared with the derivative of the
  same piece;
* bilinear upsampling: the adjoint of the interpolation (every output pixel
  returns its gradient to the two-by-two sources it read, with the same
  weights);
* concatenation: the gradient is split by channels; a skip tensor's
  gradient is added to the gradient arriving through the encoder path.
"""
from __future__ import annotations

import numpy as np

from oracle.unet import BN_EPS, LAYERS, SLOPE, max_pool2, upsample2

MOMENTUM = 0.1


def _conv3x3(x, w, b):
    n, H, W, _ = x.shape
    xp = np.zeros((n, H + 2, W + 2, x.shape[3]))
    xp[:, 1:H + 1, 1:W + 1] = x
    y = np.zeros((n, H, W, w.shape[0]))
    for kh in range(3):
        for kw in range(3):
            y += xp[:, kh:kh + H, kw:kw + W] @ w[:, kh, kw, :].T
    return y + b


def _conv3x3_bwd(x, w, dz):
    """(dW, db, dx) of z = conv3x3(x, w) + b."""
    n, H, W, ci = x.shape
    xp = np.zeros((n, H + 2, W + 2, ci))
    xp[:, 1:H + 1, 1:W + 1] = x
    dw = np.zeros_like(w)
    dxp = np.zeros_like(xp)
    g = dz.reshape(-1, dz.shape[3])
    for kh in range(3):
        for kw in range(3):
            patch = xp[:, kh:kh + H, kw:kw + W].reshape(-1, ci)
            dw[:, kh, kw, :] = g.T @ patch
            dxp[:, kh:kh + H, kw:kw + W] += dz @ w[:, kh, kw, :]
    return dw, g.sum(axis=0), dxp[:, 1:H + 1, 1:W + 1]


def _leaky(q, on=None):
    return np.where(q > 0 if on is None else on, q, SLOPE * q)


def _leaky_grad(q, on=None):
    return np.where(q > 0 if on is None else on, 1.0, SLOPE)


def _windows(x):
    n, H, W, c = x.shape
    return x.reshape(n, H // 2, 2, W // 2, 2, c).transpose(0, 1, 3, 5, 2, 4).reshape(n, H // 2, W // 2, c, 4)


def _pool(x, by=None):
    """2x2 max-pool; with by (an array of the same shape), the value of x at
    the first maximum of by's window (the branch another forward took)."""
    if by is None:
        return max_pool2(x)
    first = np.argmax(_windows(np.asarray(by)), axis=-1)
    return np.take_along_axis(_windows(x), first[..., None], axis=-1)[..., 0]


def _max_pool2_bwd(x, dy):
    """Routes dy to the first maximum (row-major) of each 2x2 window of x."""
    n, H, W, c = x.shape
    win = _windows(x)
    first = np.argmax(win, axis=-1)  # numpy's argmax takes the first maximum
    onehot = np.zeros_like(win)
    np.put_along_axis(onehot, first[..., None], 1.0, axis=-1)
    g = onehot * dy[..., None]
    return g.reshape(n, H // 2, W // 2, c, 2, 2).transpose(0, 1, 4, 2, 5, 3).reshape(n, H, W, c)


def _upsample2_bwd(dy):
    """Adjoint of oracle.unet.upsample2 (half-pixel centres, clamped edges)."""
    def axis_weights(size):
        src = np.maximum((np.arange(2 * size) + 0.5) / 2 - 0.5, 0.0)
        i0 = np.minimum(np.floor(src).astype(int), size - 1)
        i1 = np.minimum(i0 + 1, size - 1)
        return i0, i1, src - i0
    n, H2, W2, c = dy.shape
    H, W = H2 // 2, W2 // 2
    r0, r1, fr = axis_weights(H)
    c0, c1, fc = axis_weights(W)
    cols = np.zeros((n, H2, W, c))
    for j in range(W2):  # columns first (the forward interpolates rows, then columns)
        cols[:, :, c0[j]] += dy[:, :, j] * (1 - fc[j])
        cols[:, :, c1[j]] += dy[:, :, j] * fc[j]
    out = np.zeros((n, H, W, c))
    for i in range(H2):
        out[:, r0[i]] += cols[:, i] * (1 - fr[i])
        out[:, r1[i]] += cols[:, i] * fr[i]
    return out


def forward_train(params, x, cond=None):
    """Training forward. Returns (y, cache, running) where running is the
    list of updated (mean, var) per batch-normalised layer (None elsewhere).

    cond (optional): the branch decisions of another (lower-precision)
    forward of the same network, so that both sides differentiate the same
    piece of this piecewise-smooth function: {"a": the 14 activations of the
    3x3 layers (LeakyReLU branch: a > 0; max-pool: the first maximum of a's
    window), "y": its output (ReLU branch y > 0; loss sign sign(y - t))}."""
    x = np.asarray(x, dtype=np.float64)
    P = [{k: np.asarray(v, dtype=np.float64) for k, v in q.items()} for q in params]
    cache = {"layers": [], "x": x, "cond": cond}
    running = []
    it = iter(range(len(P)))

    def block(h, bn=True):
        k = next(it)
        q = P[k]
        z = _conv3x3(h, q["w"], q["b"])
        rec = {"in": h, "z": z, "bn": bn}
        if bn:
            m = z.shape[0] * z.shape[1] * z.shape[2]
            mu = z.mean(axis=(0, 1, 2))
            var = ((z - mu) ** 2).mean(axis=(0, 1, 2))
            rstd = 1.0 / np.sqrt(var + BN_EPS)
            xhat = (z - mu) * rstd
            pre = q["gamma"] * xhat + q["beta"]
            rec.update(xhat=xhat, rstd=rstd)
            running.append(((1 - MOMENTUM) * q["mean"] + MOMENTUM * mu,
                            (1 - MOMENTUM) * q["var"] + MOMENTUM * var * m / (m - 1)))
        else:
            pre = z
            running.append(None)
        rec["pre"] = pre
        rec["on"] = None if cond is None else np.asarray(cond["a"][k]) > 0
        cache["layers"].append(rec)
        return _leaky(pre, rec["on"])

    by = (lambda k: None) if cond is None else (lambda k: cond["a"][k])
    s1 = block(block(x))
    p1 = _pool(s1, by(1))
    s2 = block(block(p1))
    p2 = _pool(s2, by(3))
    s3 = block(block(p2))
    p3 = _pool(s3, by(5))
    m = block(block(p3))
    d3 = block(block(np.concatenate([upsample2(m), s3], axis=-1)))
    d2 = block(block(np.concatenate([upsample2(d3), s2], axis=-1)))
    d1 = block(block(np.concatenate([upsample2(d2), s1], axis=-1), bn=False), bn=False)
    q = P[-1]
    ypre = d1 @ q["w"].T + q["b"]
    running.append(None)
    yon = ypre > 0 if cond is None else np.asarray(cond["y"]) > 0
    cache.update(s1=s1, s2=s2, s3=s3, d1=d1, ypre=ypre, yon=yon)
    return np.where(yon, ypre, 0.0), cache, running


def l1(y, t, y_sign=None):
    """(loss, dL/dy); y_sign: take sign(y_sign - t) for the gradient (the
    side of each residual's kink another forward is on)."""
    d = y - np.asarray(t, dtype=np.float64)
    sgn = np.sign(d if y_sign is None else np.asarray(y_sign, dtype=np.float64) - np.asarray(t, dtype=np.float64))
    return float(np.abs(d).mean()), sgn / d.size


def backward_train(params, cache, dy):
    """Gradients (list of dicts with w, b and, for batch-normalised layers,
    gamma, beta; mean and var get zeros) from a training forward's cache."""
    P = [{k: np.asarray(v, dtype=np.float64) for k, v in q.items()} for q in params]
    L = cache["layers"]
    grads = [None] * len(P)
    # output 1x1 convolution with ReLU
    g = dy * cache["yon"]
    q = P[-1]
    gf = g.reshape(-1, g.shape[-1])
    grads[-1] = {"w": gf.T @ cache["d1"].reshape(-1, cache["d1"].shape[-1]), "b": gf.sum(axis=0)}
    da = g @ q["w"]

    def block_bwd(k, da):
        rec, q = L[k], P[k]
        dq = da * _leaky_grad(rec["pre"], rec["on"])
        gr = {}
        if rec["bn"]:
            xhat, rstd = rec["xhat"], rec["rstd"]
            gr["gamma"] = (dq * xhat).sum(axis=(0, 1, 2))
            gr["beta"] = dq.sum(axis=(0, 1, 2))
            dxh = dq * q["gamma"]
            dz = rstd * (dxh - dxh.mean(axis=(0, 1, 2)) - xhat * (dxh * xhat).mean(axis=(0, 1, 2)))
            gr["mean"] = np.zeros_like(q["mean"])
            gr["var"] = np.zeros_like(q["var"])
        else:
            dz = dq
        gr["w"], gr["b"], din = _conv3x3_bwd(rec["in"], q["w"], dz)
        grads[k] = gr
        return din

    def split(d, c_up):
        return d[..., :c_up], d[..., c_up:]

    # decoder stage 1 (layers 12, 13), input [up(d2) | s1]
    d = block_bwd(12, block_bwd(13, da))
    dup, ds1 = split(d, 128)
    dd2 = _upsample2_bwd(dup)
    d = block_bwd(10, block_bwd(11, dd2))
    dup, ds2 = split(d, 256)
    dd3 = _upsample2_bwd(dup)
    d = block_bwd(8, block_bwd(9, dd3))
    dup, ds3 = split(d, 256)
    dm = _upsample2_bwd(dup)
    cond = cache["cond"]
    sel = (lambda k, s: s) if cond is None else (lambda k, s: np.asarray(cond["a"][k], dtype=np.float64))
    dp3 = block_bwd(6, block_bwd(7, dm))
    ds3 = ds3 + _max_pool2_bwd(sel(5, cache["s3"]), dp3)
    dp2 = block_bwd(4, block_bwd(5, ds3))
    ds2 = ds2 + _max_pool2_bwd(sel(3, cache["s2"]), dp2)
    dp1 = block_bwd(2, block_bwd(3, ds2))
    ds1 = ds1 + _max_pool2_bwd(sel(1, cache["s1"]), dp1)
    dx = block_bwd(0, block_bwd(1, ds1))
    return grads, dx


def loss_and_grad(params, x, t, cond=None):
    y, cache, running = forward_train(params, x, cond)
    loss, dy = l1(y, t, None if cond is None else cond["y"])
    grads, dx = backward_train(params, cache, dy)
    return loss, grads, dx, y, running


def flat(grads_or_params):
    """Flat vector in the layout of synth.unet_flat (w, b, gamma, beta, mean, var per layer)."""
    parts = []
    for q in grads_or_params:
        parts += [np.asarray(q["w"]).reshape(-1), np.asarray(q["b"])]
        if "gamma" in q:
            parts += [q["gamma"], q["beta"], q["mean"], q["var"]]
    return np.concatenate(parts)


assert tuple(c for _, _, c, _ in LAYERS)  # same layer list as the inference oracle

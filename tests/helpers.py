"""Shared test helpers: error metrics, reading the library's saved
activations, and rounding inputs to the compute precision with PyTorch's own
casts (so the oracle sees exactly the operands the GPU multiplies)."""
from __future__ import annotations

import numpy as np
import torch

ACT_SHAPES = (("h1", 2, 32), ("h2", 4, 64), ("h3", 8, 128), ("u3", 4, 64), ("u2", 2, 32))
TORCH_DT = {"f32": torch.float32, "bf16": torch.bfloat16, "fp8": torch.float8_e4m3fn}


def max_rel_per_map(y, r):
    """max_i |y_i - r_i| / max_i |r_i| for every map (leading axis)."""
    y = np.asarray(y, dtype=np.float64).reshape(len(y), -1)
    r = np.asarray(r, dtype=np.float64).reshape(len(r), -1)
    return np.abs(y - r).max(axis=1) / np.maximum(np.abs(r).max(axis=1), 1e-300)


def mean_rel_per_map(y, r):
    y = np.asarray(y, dtype=np.float64).reshape(len(y), -1)
    r = np.asarray(r, dtype=np.float64).reshape(len(r), -1)
    return np.abs(y - r).sum(axis=1) / np.maximum(np.abs(r).sum(axis=1), 1e-300)


def normwise(g, r):
    g = np.asarray(g, dtype=np.float64).ravel()
    r = np.asarray(r, dtype=np.float64).ravel()
    return np.linalg.norm(g - r) / max(np.linalg.norm(r), 1e-300)


def saved_acts(saved: torch.Tensor, offsets, n, H, W, compute, scales=None):
    """Decode the library's saved activations into float64 numpy arrays.

    FP8 activations are stored as e4m3(value * scale); scales maps the
    activation name to that scale.
    """
    out = {}
    dt = TORCH_DT[compute]
    esize = torch.tensor([], dtype=dt).element_size()
    for k, (name, div, c) in enumerate(ACT_SHAPES):
        if offsets[k] < 0:
            continue
        cnt = n * (H // div) * (W // div) * c
        # decode on the host: copy the raw bytes first, then reinterpret
        raw = saved[offsets[k]: offsets[k] + cnt * esize].cpu().view(dt).float().numpy()
        raw = raw.astype(np.float64).reshape(n, H // div, W // div, c)
        if compute == "fp8":
            raw = raw / scales[name]
        out[name] = raw
    return out


def round_to(a, compute, scale=1.0):
    """Round a float array to the compute precision with PyTorch's casts
    (RNE); FP8 values are scaled, rounded (saturating at 448) and unscaled."""
    t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32))
    if compute == "f32":
        return t.double().numpy()
    if compute == "bf16":
        return t.to(torch.bfloat16).double().numpy()
    q = (t * scale).clamp(-448.0, 448.0).to(torch.float8_e4m3fn).double()
    return (q / scale).numpy()


def layer_params(params, k):
    from oracle.oracle import layer_slices
    ws, bs, shp = layer_slices()[k]
    return params[ws].reshape(shp), params[bs]

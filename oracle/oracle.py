"""Python face of the FP64 oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU
baseline leg use it to check and time the HIP path; the product path never
imports it. It shares no code with the HIP library.

All arrays are NHWC; inputs may be float32 or float64 and are widened to
float64 before the call. Parameters use the flat layout E1 E2 E3 D3 D2 D1,
each layer ``W[co][kh][kw][ci]`` followed by ``b[co]``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# (input channels, output channels, kind) per layer, in parameter order.
LAYERS = ((7, 32, "conv"), (32, 64, "conv"), (64, 128, "conv"),
          (128, 64, "tconv"), (128, 32, "tconv"), (64, 3, "tconv"))
LAYER_NAMES = ("E1", "E2", "E3", "D3", "D2", "D1")


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain C, OpenMP, IEEE double)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_U8PP = ctypes.POINTER(ctypes.c_void_p)


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        L.orc_num_params.restype = ctypes.c_long
        L.orc_layer_offset.restype = ctypes.c_long
        L.orc_layer_offset.argtypes = [ctypes.c_int]
        sig = [_D, ctypes.c_long, ctypes.c_long, ctypes.c_long, ctypes.c_long,
               _D, _D, ctypes.c_long, _D]
        L.orc_conv_s2.argtypes = sig
        L.orc_tconv_s2.argtypes = sig
        L.orc_conv_s2_pad.argtypes = sig + [ctypes.c_int]
        L.orc_tconv_s2_pad.argtypes = sig + [ctypes.c_int]
        bsig = [_D, ctypes.c_long, ctypes.c_long, ctypes.c_long, ctypes.c_long,
                _D, ctypes.c_long, _D, _D, _D, _D]
        L.orc_conv_s2_bwd.argtypes = bsig
        L.orc_tconv_s2_bwd.argtypes = bsig
        L.orc_conv_s2_bwd_pad.argtypes = bsig + [ctypes.c_int]
        L.orc_tconv_s2_bwd_pad.argtypes = bsig + [ctypes.c_int]
        fsig = [_D, _D, ctypes.c_long, ctypes.c_long, ctypes.c_long,
                ctypes.c_int, _U8PP, _D, _D, _D, _D, _D, _D]
        L.orc_forward.argtypes = fsig
        L.orc_forward_pad.argtypes = fsig + [ctypes.c_int]
        bwsig = [_D, _D, ctypes.c_long, ctypes.c_long, ctypes.c_long,
                 ctypes.c_int, _U8PP, _D, _D, _D, _D, _D, _D, _D, _D, _D]
        L.orc_backward.argtypes = bwsig
        L.orc_backward_pad.argtypes = bwsig + [ctypes.c_int]
        L.orc_l1.restype = ctypes.c_double
        L.orc_l1.argtypes = [_D, _D, ctypes.c_long, _D]
        L.orc_adam.argtypes = [_D, _D, _D, _D, ctypes.c_long, ctypes.c_long,
                               ctypes.c_double, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double]
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return None if a is None else a.ctypes.data_as(_D)


def num_params() -> int:
    return int(lib().orc_num_params())


def layer_slices():
    """[(weight slice, bias slice, (cout, 3, 3, cin))] per layer."""
    out = []
    for k, (ci, co, _) in enumerate(LAYERS):
        off = int(lib().orc_layer_offset(k))
        nw = co * 9 * ci
        out.append((slice(off, off + nw), slice(off + nw, off + nw + co), (co, 3, 3, ci)))
    return out


def conv_s2(x, wt, b=None, circular=False):
    """Stride-2 3x3 convolution, x [N,H,W,Cin], wt [Cout,3,3,Cin] -> [N,H/2,W/2,Cout].
    circular: the width is periodic (columns taken mod W) instead of zero-padded."""
    x, wt = _f64(x), _f64(wt)
    n, h, w, ci = x.shape
    co = wt.shape[0]
    assert wt.shape == (co, 3, 3, ci)
    b = None if b is None else _f64(b)
    y = np.empty((n, h // 2, w // 2, co))
    lib().orc_conv_s2_pad(_p(x), n, h, w, ci, _p(wt), _p(b), co, _p(y), int(circular))
    return y


def tconv_s2(x, wt, b=None, circular=False):
    """Stride-2 3x3 transposed convolution -> [N,2H,2W,Cout] (circular: output
    columns taken mod 2W)."""
    x, wt = _f64(x), _f64(wt)
    n, h, w, ci = x.shape
    co = wt.shape[0]
    assert wt.shape == (co, 3, 3, ci)
    b = None if b is None else _f64(b)
    y = np.empty((n, 2 * h, 2 * w, co))
    lib().orc_tconv_s2_pad(_p(x), n, h, w, ci, _p(wt), _p(b), co, _p(y), int(circular))
    return y


def conv_s2_bwd(x, wt, g, want_dx=True, circular=False):
    x, wt, g = _f64(x), _f64(wt), _f64(g)
    n, h, w, ci = x.shape
    co = wt.shape[0]
    dw = np.empty_like(wt)
    db = np.empty(co)
    dx = np.empty_like(x) if want_dx else None
    lib().orc_conv_s2_bwd_pad(_p(x), n, h, w, ci, _p(wt), co, _p(g), _p(dw), _p(db), _p(dx), int(circular))
    return dw, db, dx


def tconv_s2_bwd(x, wt, g, want_dx=True, circular=False):
    x, wt, g = _f64(x), _f64(wt), _f64(g)
    n, h, w, ci = x.shape
    co = wt.shape[0]
    dw = np.empty_like(wt)
    db = np.empty(co)
    dx = np.empty_like(x) if want_dx else None
    lib().orc_tconv_s2_bwd_pad(_p(x), n, h, w, ci, _p(wt), co, _p(g), _p(dw), _p(db), _p(dx), int(circular))
    return dw, db, dx


ACT_NAMES = ("h1", "h2", "h3", "u3", "u2", "y")


def _mask_array(masks, keep):
    """Pack up to six optional uint8 masks into a void* array for the C side."""
    if masks is None:
        return None
    arr = (ctypes.c_void_p * 6)()
    for k, name in enumerate(ACT_NAMES):
        m = masks.get(name) if isinstance(masks, dict) else masks[k]
        if m is None:
            arr[k] = None
        else:
            m = np.ascontiguousarray(m, dtype=np.uint8)
            keep.append(m)
            arr[k] = m.ctypes.data
    return ctypes.cast(arr, _U8PP)


def forward(params, x, final_relu=False, masks=None, circular=False):
    """Whole autoencoder in FP64. Returns dict of h1,h2,h3,u3,u2,y.
    circular: every layer's width is periodic (circular azimuth padding)."""
    params, x = _f64(params), _f64(x)
    n, h, w, c = x.shape
    assert c == 7 and h % 8 == 0 and w % 8 == 0
    assert params.size == num_params()
    acts = {
        "h1": np.empty((n, h // 2, w // 2, 32)),
        "h2": np.empty((n, h // 4, w // 4, 64)),
        "h3": np.empty((n, h // 8, w // 8, 128)),
        "u3": np.empty((n, h // 4, w // 4, 64)),
        "u2": np.empty((n, h // 2, w // 2, 32)),
        "y": np.empty((n, h, w, 3)),
    }
    keep = []
    mp = _mask_array(masks, keep)
    lib().orc_forward_pad(_p(params), _p(x), n, h, w, int(final_relu), mp,
                          *[_p(acts[k]) for k in ACT_NAMES], int(circular))
    return acts


def l1(y, t):
    """(loss, dL/dy) with loss = mean |y - t| and dy = sign(y - t)/M."""
    y, t = _f64(y), _f64(t)
    dy = np.empty_like(y)
    loss = lib().orc_l1(_p(y), _p(t), y.size, _p(dy))
    return float(loss), dy


def backward(params, x, acts, dy, final_relu=False, masks=None, want_dx=False, circular=False):
    """dL/dparams (flat) and optionally dL/dx, from a forward's activations."""
    params, x, dy = _f64(params), _f64(x), _f64(dy)
    n, h, w, _ = x.shape
    a = {k: _f64(acts[k]) for k in ACT_NAMES}
    dparams = np.empty_like(params)
    dx = np.empty_like(x) if want_dx else None
    keep = []
    mp = _mask_array(masks, keep)
    lib().orc_backward_pad(_p(params), _p(x), n, h, w, int(final_relu), mp,
                           *[_p(a[k]) for k in ACT_NAMES], _p(dy), _p(dparams), _p(dx), int(circular))
    return dparams, dx


def loss_and_grad(params, x, t, final_relu=False, masks=None, want_dx=False, circular=False):
    acts = forward(params, x, final_relu, masks, circular)
    loss, dy = l1(acts["y"], t)
    dp, dx = backward(params, x, acts, dy, final_relu, masks, want_dx, circular)
    return loss, dp, dx, acts


def adam(theta, m, v, g, t, lr=6e-5, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (PyTorch's form) in FP64; returns new (theta, m, v)."""
    theta, m, v, g = (np.array(a, dtype=np.float64, copy=True) for a in (theta, m, v, g))
    lib().orc_adam(_p(theta), _p(m), _p(v), _p(g), theta.size, int(t), lr, beta1, beta2, eps)
    return theta, m, v

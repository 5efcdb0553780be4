"""ctypes binding of libdrc_cae.so: one Python function per C entry point,
with the same name, doing argument marshalling only (every step of the path
runs in the library's HIP kernels). PyTorch provides the device memory and
the stream; tensors must be contiguous float32 CUDA(HIP) tensors.

The library is loaded from this package directory. If it is missing, every
entry point raises: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdrc_cae.so")

DRC_OK = 0
STATUS_NAMES = {0: "DRC_OK", 1: "DRC_ERR_INVALID_ARG", 2: "DRC_ERR_SHAPE", 3: "DRC_ERR_UNSUPPORTED",
                4: "DRC_ERR_WORKSPACE", 5: "DRC_ERR_HIP", 6: "DRC_ERR_STATE"}
DRC_F32, DRC_BF16, DRC_FP8_E4M3 = 0, 1, 2
DTYPES = {"f32": DRC_F32, "bf16": DRC_BF16, "fp8": DRC_FP8_E4M3}
DRC_WS_FORWARD, DRC_WS_BACKWARD, DRC_WS_STEP, DRC_WS_CALIBRATE, DRC_WS_AUTOTUNE = 1, 2, 4, 8, 16


class DrcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class drc_cae_desc(ctypes.Structure):
    _fields_ = [("in_ch", ctypes.c_int), ("out_ch", ctypes.c_int), ("widths", ctypes.c_int * 3),
                ("compute", ctypes.c_int), ("final_relu", ctypes.c_int), ("pad_w", ctypes.c_int)]


DRC_PAD_ZERO, DRC_PAD_CIRCULAR = 0, 1


class drc_adam_cfg(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_double), ("beta1", ctypes.c_double), ("beta2", ctypes.c_double),
                ("eps", ctypes.c_double)]


class drc_map_desc(ctypes.Structure):
    _fields_ = [("h", ctypes.c_int), ("w", ctypes.c_int), ("x_off", ctypes.c_int64),
                ("y_off", ctypes.c_int64)]


_VP = ctypes.c_void_p
_I = ctypes.c_int
_SZ = ctypes.c_size_t
_SIGS = {
    "drc_cae_default_desc": (drc_cae_desc, [_I]),
    "drc_cae_create": (_I, [ctypes.POINTER(drc_cae_desc), ctypes.POINTER(_VP)]),
    "drc_cae_destroy": (None, [_VP]),
    "drc_cae_num_params": (_SZ, [_VP]),
    "drc_cae_set_params": (_I, [_VP, _VP, _VP]),
    "drc_cae_set_recompute": (_I, [_VP, _I]),
    "drc_cae_set_fused": (_I, [_VP, _I]),
    "drc_cae_saved_size": (_I, [_VP, _I, _I, _I, ctypes.POINTER(_SZ), ctypes.POINTER(ctypes.c_int64)]),
    "drc_cae_workspace_size": (_I, [_VP, _I, _I, _I, _I, ctypes.POINTER(_SZ)]),
    "drc_cae_forward": (_I, [_VP, _VP, _VP, _I, _I, _I, _VP, _VP, _SZ, _VP]),
    "drc_cae_backward": (_I, [_VP, _VP, _VP, _VP, _VP, _VP, _I, _I, _I, _VP, _SZ, _VP]),
    "drc_cae_step": (_I, [_VP, _VP, _VP, _VP, ctypes.c_int64, ctypes.POINTER(drc_adam_cfg), _VP, _VP,
                          _VP, _VP, _I, _I, _I, _VP, _SZ, _VP]),
    "drc_cae_step_aug": (_I, [_VP, _VP, _VP, _VP, ctypes.c_int64, ctypes.POINTER(drc_adam_cfg), _VP, _VP,
                              _VP, _VP, _VP, _VP, _I, _I, _I, _VP, _SZ, _VP]),
    "drc_cae_static_scratch_bytes": (_SZ, []),
    "drc_cae_forward_static": (_I, [_VP, _VP, _VP, _I, _I, _I, _VP]),
    "drc_cae_step_graph_create": (_I, [_VP, _VP, _VP, _VP, ctypes.POINTER(drc_adam_cfg), _VP, _VP, _VP, _VP,
                                       _I, _I, _I, _VP, _SZ, _VP, ctypes.POINTER(_VP)]),
    "drc_cae_step_graph_launch": (_I, [_VP, ctypes.c_int64]),
    "drc_cae_step_graph_captures": (_I, [_VP, ctypes.POINTER(ctypes.c_int64)]),
    "drc_cae_step_graph_destroy": (None, [_VP]),
    "drc_cae_calibrate_fp8": (_I, [_VP, _VP, _I, _I, _I, _VP, _SZ, _VP]),
    "drc_cae_get_fp8_scales": (_I, [_VP, ctypes.POINTER(ctypes.c_float), _VP]),
    "drc_cae_plan_create": (_I, [_VP, ctypes.POINTER(drc_map_desc), _I, ctypes.c_char_p,
                                 ctypes.POINTER(_VP)]),
    "drc_cae_plan_workspace_size": (_I, [_VP, ctypes.POINTER(_SZ)]),
    "drc_cae_plan_launch": (_I, [_VP, _VP, _VP, _VP, _SZ, _VP]),
    "drc_cae_plan_destroy": (None, [_VP]),
    "drc_cae_plan_captures": (_I, [_VP, ctypes.POINTER(ctypes.c_int64)]),
    "drc_envmap_build": (_I, [_VP, _I, _I, _I, _VP, _VP, _VP, _VP]),
    "drc_envmap_sample": (_I, [_VP, _VP, _I, _I, _I, _I, _VP, _VP, _VP, _VP, _VP]),
    "drc_envmap_pdf": (_I, [_VP, _VP, _I, _I, _I, _I, _VP, _VP, _VP]),
    "drc_interp_weights": (_I, [_VP, _I, _I, _I, _VP, ctypes.c_float, _VP, _VP, _VP]),
    "drc_augment": (_I, [_VP, _VP, _I, _I, _I, _VP, _VP, _VP, _VP, _VP]),
    "drc_unet_create": (_I, [ctypes.POINTER(_VP)]),
    "drc_unet_destroy": (None, [_VP]),
    "drc_unet_num_params": (_SZ, []),
    "drc_unet_set_params": (_I, [_VP, _VP, _VP]),
    "drc_unet_workspace_size": (_I, [_I, _I, _I, ctypes.POINTER(_SZ)]),
    "drc_unet_forward": (_I, [_VP, _VP, _VP, _I, _I, _I, _VP, _SZ, _VP]),
    "drc_unet_train_workspace_size": (_I, [_I, _I, _I, ctypes.POINTER(_SZ)]),
    "drc_unet_train_act_offsets": (_I, [_I, _I, _I, ctypes.POINTER(ctypes.c_int64)]),
    "drc_unet_train_step": (_I, [_VP, _VP, _VP, ctypes.c_int64, ctypes.POINTER(drc_adam_cfg), _VP, _VP, _VP, _VP,
                                 _VP, _I, _I, _I, _VP, _SZ, _VP]),
    "drc_cae_autotune": (_I, [_VP, _I, _I, _I, _VP, _VP, _SZ, ctypes.c_char_p, _VP]),
    "drc_cae_set_tile": (_I, [_VP, _I, _I, _I]),
    "drc_cae_wgrad_schedule": (_I, [_I, _I, _I, _I, _I, ctypes.POINTER(ctypes.c_int64)]),
    "drc_cae_profile": (_I, [_VP, _I]),
    "drc_cae_profile_read": (_I, [_VP, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
    "drc_status_string": (ctypes.c_char_p, [_I]),
    "drc_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Load libdrc_cae.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first "
                               "(python -c 'import __graft_entry__ as g; g.build()')")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status):
    if status != DRC_OK:
        raise DrcError(status, lib().drc_last_error().decode())


def _ptr(t):
    """Device pointer of a tensor (or None)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _nhw(x, c):
    if x.dim() != 4 or x.shape[3] != c:
        raise ValueError(f"expected NHWC tensor with {c} channels, got {tuple(x.shape)}")
    return int(x.shape[0]), int(x.shape[1]), int(x.shape[2])


def _nbytes(ws):
    return 0 if ws is None else ws.numel() * ws.element_size()


# ---------------------------------------------------------------- entry points
def drc_cae_default_desc(compute=DRC_F32):
    return lib().drc_cae_default_desc(compute)


def drc_cae_create(desc):
    h = _VP()
    _check(lib().drc_cae_create(ctypes.byref(desc), ctypes.byref(h)))
    return h.value


def drc_cae_destroy(h):
    lib().drc_cae_destroy(h)


def drc_cae_num_params(h):
    return int(lib().drc_cae_num_params(h))


def drc_cae_set_params(h, params, stream=None):
    _check(lib().drc_cae_set_params(h, _ptr(params), _stream(stream)))


def drc_cae_set_recompute(h, on):
    _check(lib().drc_cae_set_recompute(h, int(on)))


def drc_cae_set_fused(h, on):
    _check(lib().drc_cae_set_fused(h, int(on)))


def drc_cae_saved_size(h, n, H, W):
    b = _SZ()
    off = (ctypes.c_int64 * 5)()
    _check(lib().drc_cae_saved_size(h, n, H, W, ctypes.byref(b), off))
    return int(b.value), [int(v) for v in off]


def drc_cae_workspace_size(h, n, H, W, flags):
    b = _SZ()
    _check(lib().drc_cae_workspace_size(h, n, H, W, flags, ctypes.byref(b)))
    return int(b.value)


def drc_cae_forward(h, x, y, saved=None, ws=None, stream=None):
    n, H, W = _nhw(x, 7)
    _check(lib().drc_cae_forward(h, _ptr(x), _ptr(y), n, H, W, _ptr(saved), _ptr(ws), _nbytes(ws),
                                 _stream(stream)))


def drc_cae_backward(h, x, dy, saved, dparams, dx=None, ws=None, stream=None):
    n, H, W = _nhw(x, 7)
    _check(lib().drc_cae_backward(h, _ptr(x), _ptr(dy), _ptr(saved), _ptr(dparams), _ptr(dx), n, H, W,
                                  _ptr(ws), _nbytes(ws), _stream(stream)))


def drc_cae_step(h, params, m, v, t, adam, x, target, loss, dparams=None, ws=None, stream=None):
    n, H, W = _nhw(x, 7)
    _check(lib().drc_cae_step(h, _ptr(params), _ptr(m), _ptr(v), int(t), ctypes.byref(adam), _ptr(x),
                              _ptr(target), _ptr(loss), _ptr(dparams), n, H, W, _ptr(ws), _nbytes(ws),
                              _stream(stream)))


def drc_cae_step_aug(h, params, m, v, t, adam, x, target, roll, flip, loss, dparams=None, ws=None, stream=None):
    n, H, W = _nhw(x, 7)
    _check(lib().drc_cae_step_aug(h, _ptr(params), _ptr(m), _ptr(v), int(t), ctypes.byref(adam), _ptr(x),
                                  _ptr(target), _ptr(roll), _ptr(flip), _ptr(loss), _ptr(dparams), n, H, W,
                                  _ptr(ws), _nbytes(ws), _stream(stream)))


def drc_cae_static_scratch_bytes():
    return int(lib().drc_cae_static_scratch_bytes())


def drc_cae_forward_static(h, x, y, stream=None):
    n, H, W = _nhw(x, 7)
    _check(lib().drc_cae_forward_static(h, _ptr(x), _ptr(y), n, H, W, _stream(stream)))


def drc_cae_step_graph_create(h, params, m, v, adam, x, target, loss, dparams=None, ws=None, stream=None):
    """Record one training step as a graph on a non-null stream."""
    n, H, W = _nhw(x, 7)
    g = _VP()
    _check(lib().drc_cae_step_graph_create(h, _ptr(params), _ptr(m), _ptr(v), ctypes.byref(adam), _ptr(x),
                                           _ptr(target), _ptr(loss), _ptr(dparams), n, H, W, _ptr(ws), _nbytes(ws),
                                           _stream(stream), ctypes.byref(g)))
    return g.value


def drc_cae_step_graph_launch(g, t):
    _check(lib().drc_cae_step_graph_launch(g, int(t)))


def drc_cae_step_graph_captures(g):
    c = ctypes.c_int64()
    _check(lib().drc_cae_step_graph_captures(g, ctypes.byref(c)))
    return int(c.value)


def drc_cae_step_graph_destroy(g):
    lib().drc_cae_step_graph_destroy(g)


def drc_cae_calibrate_fp8(h, x, ws=None, stream=None):
    n, H, W = _nhw(x, 7)
    _check(lib().drc_cae_calibrate_fp8(h, _ptr(x), n, H, W, _ptr(ws), _nbytes(ws), _stream(stream)))


def drc_cae_get_fp8_scales(h, stream=None):
    out = (ctypes.c_float * 10)()
    _check(lib().drc_cae_get_fp8_scales(h, out, _stream(stream)))
    return [float(v) for v in out]


def drc_cae_plan_create(h, maps, tune_cache=None):
    """maps: sequence of (h, w, x_off, y_off)."""
    arr = (drc_map_desc * len(maps))(*[drc_map_desc(int(a), int(b), int(c), int(d)) for a, b, c, d in maps])
    p = _VP()
    _check(lib().drc_cae_plan_create(h, arr, len(maps), None if tune_cache is None else
                                     tune_cache.encode(), ctypes.byref(p)))
    return p.value


def drc_cae_plan_workspace_size(p):
    b = _SZ()
    _check(lib().drc_cae_plan_workspace_size(p, ctypes.byref(b)))
    return int(b.value)


def drc_cae_plan_launch(p, x_packed, y_packed, ws=None, stream=None):
    _check(lib().drc_cae_plan_launch(p, _ptr(x_packed), _ptr(y_packed), _ptr(ws), _nbytes(ws),
                                     _stream(stream)))


def drc_cae_plan_destroy(p):
    lib().drc_cae_plan_destroy(p)


def drc_cae_plan_captures(p):
    c = ctypes.c_int64()
    _check(lib().drc_cae_plan_captures(p, ctypes.byref(c)))
    return int(c.value)


def drc_envmap_build(y, cdf_u, cdf_v, total, stream=None):
    """y [n, H, W, 3] -> cdf_u [n, H, W], cdf_v [n, H], total [n]."""
    n, H, W = _nhw(y, 3)
    _check(lib().drc_envmap_build(_ptr(y), n, H, W, _ptr(cdf_u), _ptr(cdf_v), _ptr(total), _stream(stream)))


def drc_envmap_sample(cdf_u, cdf_v, xi, dirs, pdf, pix, stream=None):
    """xi [n, S, 2] -> dirs [n, S, 3], pdf [n, S], pix [n, S] (int32)."""
    n, H, W = (int(v) for v in cdf_u.shape)
    S = int(xi.shape[1])
    _check(lib().drc_envmap_sample(_ptr(cdf_u), _ptr(cdf_v), n, H, W, S, _ptr(xi), _ptr(dirs), _ptr(pdf),
                                   _ptr(pix), _stream(stream)))


def drc_envmap_pdf(cdf_u, cdf_v, dirs, pdf, stream=None):
    """dirs [n, S, 3] -> pdf [n, S]."""
    n, H, W = (int(v) for v in cdf_u.shape)
    S = int(dirs.shape[1])
    _check(lib().drc_envmap_pdf(_ptr(cdf_u), _ptr(cdf_v), n, H, W, S, _ptr(dirs), _ptr(pdf), _stream(stream)))


def drc_interp_weights(normals, r, cache_normals, eps, idx, prob, stream=None):
    """normals [Hi, Wi, 3], cache_normals [Gy, Gx, 3] -> idx [Hi, Wi, 4] int32, prob [Hi, Wi, 4]."""
    if normals.dim() != 3 or normals.shape[2] != 3:
        raise ValueError(f"expected [Hi, Wi, 3] normals, got {tuple(normals.shape)}")
    Hi, Wi = int(normals.shape[0]), int(normals.shape[1])
    _check(lib().drc_interp_weights(_ptr(normals), Hi, Wi, int(r), _ptr(cache_normals), float(eps), _ptr(idx),
                                    _ptr(prob), _stream(stream)))


def drc_augment(x, t, roll, flip, x_out, t_out=None, stream=None):
    """x [n, H, W, 7] (and t [n, H, W, 3] or None), roll / flip int32 [n] -> x_out (t_out)."""
    n, H, W = _nhw(x, 7)
    _check(lib().drc_augment(_ptr(x), _ptr(t), n, H, W, _ptr(roll), _ptr(flip), _ptr(x_out), _ptr(t_out),
                             _stream(stream)))


def drc_unet_create():
    u = _VP()
    _check(lib().drc_unet_create(ctypes.byref(u)))
    return u.value


def drc_unet_destroy(u):
    lib().drc_unet_destroy(u)


def drc_unet_num_params():
    return int(lib().drc_unet_num_params())


def drc_unet_set_params(u, params, stream=None):
    _check(lib().drc_unet_set_params(u, _ptr(params), _stream(stream)))


def drc_unet_workspace_size(n, H, W):
    b = _SZ()
    _check(lib().drc_unet_workspace_size(n, H, W, ctypes.byref(b)))
    return int(b.value)


def drc_unet_forward(u, x, y, ws, stream=None):
    n, H, W = _nhw(x, 7)
    _check(lib().drc_unet_forward(u, _ptr(x), _ptr(y), n, H, W, _ptr(ws), _nbytes(ws), _stream(stream)))


def drc_cae_autotune(h, x, ws, tune_cache, stream=None):
    n, H, W = _nhw(x, 7)
    _check(lib().drc_cae_autotune(h, n, H, W, _ptr(x), _ptr(ws), _nbytes(ws), tune_cache.encode(),
                                  _stream(stream)))


def drc_cae_set_tile(h, layer, H, npw):
    _check(lib().drc_cae_set_tile(h, layer, H, npw))


def drc_cae_wgrad_schedule(compute, layer, n, H, W):
    """(kernel, rows per strip, strips (or pixels) per chunk, chunks) of a
    layer's weight gradient; host only."""
    info = (ctypes.c_int64 * 4)()
    _check(lib().drc_cae_wgrad_schedule(int(compute), int(layer), int(n), int(H), int(W), info))
    return tuple(int(v) for v in info)


def drc_cae_profile(h, enable):
    _check(lib().drc_cae_profile(h, int(enable)))


def drc_cae_profile_read(h):
    """(ms[24], calls[24]) per timing slot; waits for the recorded events."""
    ms = (ctypes.c_double * 24)()
    calls = (ctypes.c_int64 * 24)()
    _check(lib().drc_cae_profile_read(h, ms, calls))
    return list(ms), list(calls)


def drc_status_string(s):
    return lib().drc_status_string(s).decode()


def drc_last_error():
    return lib().drc_last_error().decode()


def drc_unet_train_workspace_size(n, H, W):
    sz = _SZ()
    _check(lib().drc_unet_train_workspace_size(n, H, W, ctypes.byref(sz)))
    return sz.value


def drc_unet_train_step(params, m, v, t, adam, x, target, loss, dparams=None, y=None, ws=None, stream=None):
    n, H, W = _nhw(x, 7)
    _check(lib().drc_unet_train_step(_ptr(params), _ptr(m), _ptr(v), int(t), ctypes.byref(adam), _ptr(x),
                                     _ptr(target), _ptr(loss), _ptr(dparams), _ptr(y), n, H, W, _ptr(ws),
                                     _nbytes(ws), _stream(stream)))


def drc_unet_train_act_offsets(n, H, W):
    off = (ctypes.c_int64 * 14)()
    _check(lib().drc_unet_train_act_offsets(n, H, W, off))
    return list(off)

"""PyTorch-facing wrapper: a handle object that owns its workspace tensors,
and a torch.autograd.Function whose forward and backward are the library's
drc_cae_forward / drc_cae_backward. PyTorch supplies memory and streams only.
"""
from __future__ import annotations

import torch

from . import binding as B


def _aligned_bytes(nbytes: int, device) -> torch.Tensor:
    """A uint8 device buffer of nbytes whose data pointer is 256-byte aligned."""
    buf = torch.empty(max(nbytes, 1) + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf[off:off + max(nbytes, 1)]


class CAE:
    """One autoencoder handle (compute dtype 'f32', 'bf16' or 'fp8'; circular:
    the width wraps around, circular azimuth padding)."""

    def __init__(self, compute: str = "bf16", params: torch.Tensor | None = None, device="cuda",
                 final_relu: bool = False, recompute: bool = False, circular: bool = False):
        self.device = torch.device(device)
        self.compute = compute
        desc = B.drc_cae_default_desc(B.DTYPES[compute])
        desc.final_relu = int(final_relu)
        desc.pad_w = B.DRC_PAD_CIRCULAR if circular else B.DRC_PAD_ZERO
        with torch.cuda.device(self.device):
            self.h = B.drc_cae_create(desc)
        self.num_params = B.drc_cae_num_params(self.h)
        B.drc_cae_set_recompute(self.h, int(recompute))
        self._ws = {}
        self.params = None
        if params is not None:
            self.set_params(params)

    def __del__(self):
        h = getattr(self, "h", None)
        destroy = getattr(B, "drc_cae_destroy", None)
        if h and callable(destroy):  # the binding may be torn down first at interpreter exit
            destroy(h)
            self.h = None

    def set_params(self, params: torch.Tensor):
        assert params.dtype == torch.float32 and params.numel() == self.num_params
        self.params = params.contiguous()
        B.drc_cae_set_params(self.h, self.params)
        # what the packs were made from: storage and its in-place version
        self._packed = (self.params.data_ptr(), self.params._version)

    def ensure_packed(self, params: torch.Tensor):
        """Check that the handle's packs hold the current values of params:
        repack after an in-place update of the packed tensor (its version
        counter moved); a different tensor is an error, since the packs
        would silently hold other weights."""
        if self.params is None or params.data_ptr() != self._packed[0]:
            raise ValueError("params is not the tensor this handle was packed from: call cae.set_params(params)")
        if params._version != self._packed[1]:
            self.set_params(params.detach())

    def set_recompute(self, on: bool):
        B.drc_cae_set_recompute(self.h, int(on))

    def set_fused(self, on: bool):
        """BF16 forward (and training recompute) of 32x32 / 64x64 maps in one kernel (default) or layer by layer."""
        B.drc_cae_set_fused(self.h, int(on))
        self._ws.clear()

    def workspace(self, n, H, W, flags):
        key = (n, H, W, flags)
        if key not in self._ws:
            self._ws[key] = _aligned_bytes(B.drc_cae_workspace_size(self.h, n, H, W, flags), self.device)
        return self._ws[key]

    def saved_buffer(self, n, H, W):
        nbytes, offsets = B.drc_cae_saved_size(self.h, n, H, W)
        return _aligned_bytes(nbytes, self.device), offsets

    def forward(self, x: torch.Tensor, y: torch.Tensor | None = None, saved=None):
        n, H, W, _ = x.shape
        if y is None:
            y = torch.empty((n, H, W, 3), dtype=torch.float32, device=x.device)
        ws = self.workspace(n, H, W, B.DRC_WS_FORWARD)
        B.drc_cae_forward(self.h, x, y, saved, ws)
        return y

    __call__ = forward

    def backward(self, x, dy, saved, dparams=None, want_dx=False):
        n, H, W, _ = x.shape
        if dparams is None:
            dparams = torch.empty(self.num_params, dtype=torch.float32, device=x.device)
        dx = torch.empty_like(x) if want_dx else None
        ws = self.workspace(n, H, W, B.DRC_WS_BACKWARD)
        B.drc_cae_backward(self.h, x, dy, saved, dparams, dx, ws)
        return dparams, dx

    def calibrate_fp8(self, x):
        n, H, W, _ = x.shape
        ws = self.workspace(n, H, W, B.DRC_WS_CALIBRATE)
        B.drc_cae_calibrate_fp8(self.h, x, ws)


def augment(x: torch.Tensor, t: torch.Tensor | None, roll: torch.Tensor, flip: torch.Tensor):
    """Rotated / mirrored copies of training maps (drc_augment): map m turned
    by roll[m] columns about the normal and mirrored where flip[m] != 0."""
    xo = torch.empty_like(x)
    to = None if t is None else torch.empty_like(t)
    B.drc_augment(x.contiguous(), None if t is None else t.contiguous(), roll.to(torch.int32).contiguous(),
                  flip.to(torch.int32).contiguous(), xo, to)
    return xo, to


class Trainer:
    """Adam training on the device: one drc_cae_step per call."""

    def __init__(self, cae: CAE, params: torch.Tensor, lr=6e-5, betas=(0.9, 0.999), eps=1e-8):
        self.cae = cae
        self.params = params
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.t = 0
        self.adam = B.drc_adam_cfg(lr, betas[0], betas[1], eps)
        self.loss = torch.zeros(1, dtype=torch.float32, device=params.device)
        cae.set_params(params)

    def step(self, x, target, dparams=None, roll=None, flip=None):
        """One step; with roll and flip (int32 [n] device tensors) on the
        maps augmented by them, read through the loaders (drc_cae_step_aug)."""
        n, H, W, _ = x.shape
        ws = self.cae.workspace(n, H, W, B.DRC_WS_STEP)
        self.t += 1
        if roll is None:
            B.drc_cae_step(self.cae.h, self.params, self.m, self.v, self.t, self.adam, x, target, self.loss,
                           dparams, ws)
        else:
            B.drc_cae_step_aug(self.cae.h, self.params, self.m, self.v, self.t, self.adam, x, target, roll, flip,
                               self.loss, dparams, ws)
        return self.loss


class GraphTrainer(Trainer):
    """Trainer whose step is recorded once as a HIP graph on its own stream
    (drc_cae_step_graph_*) and replayed; the batch tensors are fixed at the
    first step (fill them in place for the next batch)."""

    def __init__(self, cae: CAE, params: torch.Tensor, **kw):
        super().__init__(cae, params, **kw)
        self._own = torch.cuda.Stream(device=params.device)
        self.g = None
        self._key = None

    def _stream(self):
        """The current stream if it can be captured (not the null stream),
        else the trainer's own stream (joined to the current one per step)."""
        cur = torch.cuda.current_stream(self.params.device)
        return (cur, False) if cur.cuda_stream != 0 else (self._own, True)

    def step(self, x, target, dparams=None):
        n, H, W, _ = x.shape
        stream, join = self._stream()
        key = (x.data_ptr(), target.data_ptr(), None if dparams is None else dparams.data_ptr(), n, H, W,
               stream.cuda_stream)
        cur = torch.cuda.current_stream(self.params.device)
        if self.g is None or key != self._key:
            self.close()
            ws = self.cae.workspace(n, H, W, B.DRC_WS_STEP)
            if join:
                stream.wait_stream(cur)
            self.g = B.drc_cae_step_graph_create(self.cae.h, self.params, self.m, self.v, self.adam, x, target,
                                                 self.loss, dparams, ws, stream=stream)
            self._key = key
        self.t += 1
        if join:
            stream.wait_stream(cur)
        B.drc_cae_step_graph_launch(self.g, self.t)
        if join:
            cur.wait_stream(stream)
        return self.loss

    def close(self):
        if self.g is not None:
            B.drc_cae_step_graph_destroy(self.g)
            self.g = None

    def __del__(self):
        self.close()


class CAEFunction(torch.autograd.Function):
    """y = CAE(x; params) with the library's forward and backward kernels.

    params must be the tensor the handle was packed from (cae.set_params);
    an in-place update of it since then (e.g. an optimizer step) is repacked
    before the forward, and any other tensor is rejected.
    """

    @staticmethod
    def forward(ctx, x, params, cae: CAE):
        cae.ensure_packed(params)
        x = x.contiguous()
        n, H, W, _ = x.shape
        saved, _ = cae.saved_buffer(n, H, W)
        y = cae.forward(x, saved=saved)
        ctx.cae = cae
        ctx.saved = saved
        ctx.save_for_backward(x)
        return y

    @staticmethod
    def backward(ctx, dy):
        (x,) = ctx.saved_tensors
        dparams, dx = ctx.cae.backward(x, dy.contiguous(), ctx.saved, want_dx=ctx.needs_input_grad[0])
        return dx, dparams, None

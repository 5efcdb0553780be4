"""drc_cae_forward_static: the forward pass that allocates nothing, its
intermediate activations in the library's per-device scratch array (needs
gfx950). Its outputs must equal drc_cae_forward's with a workspace, bit for
bit (same kernels, K order and rounding), on two calls in a row, the second
with a smaller batch, so that the second call runs over what the first left
in the shared array."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1910_02480_amd import binding as B
from paper_1910_02480_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def params():
    return torch.from_numpy(synth.init_params(0)).to(DEV)


def _reference(cae, x):
    y = torch.empty((*x.shape[:3], 3), device=DEV)
    cae.forward(x, y)
    return y


@pytest.mark.parametrize("compute,fused", [("f32", True), ("bf16", False), ("bf16", True), ("fp8", True)])
def test_forward_static_matches_forward(params, compute, fused):
    from paper_1910_02480_amd.cae import CAE
    cae = CAE(compute, params, device=DEV)
    cae.set_fused(fused)
    if compute == "fp8":
        cae.calibrate_fp8(torch.from_numpy(synth.radiance_maps(8, 64, 64, seed=3)).to(DEV))
    cap = B.drc_cae_static_scratch_bytes()
    assert cap == 64 << 20
    # a larger batch, then a smaller one of another size, over the same scratch
    for n, H in ((48, 64), (5, 32)):
        need = B.drc_cae_workspace_size(cae.h, n, H, H, B.DRC_WS_FORWARD)
        assert need <= cap
        x = torch.from_numpy(synth.radiance_maps(n, H, H, seed=20 + n)).to(DEV)
        y = torch.full((n, H, H, 3), float("nan"), device=DEV)
        B.drc_cae_forward_static(cae.h, x, y)
        ref = _reference(cae, x)
        torch.cuda.synchronize()
        print(f"{compute} fused={fused} n={n} {H}x{H}: scratch {need} of {cap} bytes", flush=True)
        assert torch.isfinite(y).all()
        np.testing.assert_array_equal(y.cpu().numpy(), ref.cpu().numpy())


def test_forward_static_rejects_oversized_batch(params):
    """A batch whose layer-path activations exceed the array is refused on
    the host with DRC_ERR_WORKSPACE; the output keeps its contents."""
    from paper_1910_02480_amd.cae import CAE
    cae = CAE("f32", params, device=DEV)
    n, H = 16, 256
    need = B.drc_cae_workspace_size(cae.h, n, H, H, B.DRC_WS_FORWARD)
    assert need > B.drc_cae_static_scratch_bytes()
    x = torch.zeros((n, H, H, 7), device=DEV)
    y = torch.full((n, H, H, 3), -7.0, device=DEV)
    with pytest.raises(B.DrcError) as e:
        B.drc_cae_forward_static(cae.h, x, y)
    assert e.value.status == 4 and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert torch.all(y == -7.0)
    L = B.lib()
    assert L.drc_cae_forward_static(None, None, None, 1, 8, 8, None) == 1
    assert L.drc_cae_forward_static(cae.h, x.data_ptr(), y.data_ptr(), 1, 12, 8, None) == 2
    assert L.drc_cae_forward_static(cae.h, x.data_ptr() + 4, y.data_ptr(), 1, 8, 8, None) == 1

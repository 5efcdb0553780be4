"""C-ABI contract checks that run without a GPU: the library loads, exports
every function the header declares, and rejects bad arguments on the host
before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "drc_cae.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(drc_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def B():
    from paper_1910_02480_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.fail("libdrc_cae.so is not built (run __graft_entry__.build())")
    binding.lib()
    return binding


def test_exports_every_declared_symbol(B):
    names = _declared()
    assert len(names) >= 20
    L = ctypes.CDLL(B.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # the binding exposes the same names
    assert not [n for n in names if not hasattr(B, n)]


def test_status_strings(B):
    for k, name in B.STATUS_NAMES.items():
        assert B.drc_status_string(k) == name


def test_default_desc(B):
    d = B.drc_cae_default_desc(B.DRC_BF16)
    assert (d.in_ch, d.out_ch, list(d.widths), d.compute, d.final_relu, d.pad_w) == \
        (7, 3, [32, 64, 128], 1, 0, B.DRC_PAD_ZERO)


def _expect(B, status, fn, *args):
    with pytest.raises(B.DrcError) as e:
        fn(*args)
    assert e.value.status == status, str(e.value)


def test_create_rejects_bad_descriptions(B):
    d = B.drc_cae_default_desc(B.DRC_F32)
    d.widths[2] = 256
    _expect(B, 3, B.drc_cae_create, d)
    d = B.drc_cae_default_desc(B.DRC_F32)
    d.in_ch = 6
    _expect(B, 3, B.drc_cae_create, d)
    d = B.drc_cae_default_desc(9)
    _expect(B, 1, B.drc_cae_create, d)
    d = B.drc_cae_default_desc(B.DRC_F32)
    d.final_relu = 2
    _expect(B, 1, B.drc_cae_create, d)
    d = B.drc_cae_default_desc(B.DRC_F32)
    d.pad_w = 2
    _expect(B, 1, B.drc_cae_create, d)
    L = B.lib()
    assert L.drc_cae_create(None, None) == 1
    h = ctypes.c_void_p()
    assert L.drc_cae_create(None, ctypes.byref(h)) == 1 and h.value is None


def test_null_handle_rejected(B):
    L = B.lib()
    sz = ctypes.c_size_t()
    assert L.drc_cae_workspace_size(None, 1, 8, 8, 1, ctypes.byref(sz)) == 1
    assert L.drc_cae_saved_size(None, 1, 8, 8, ctypes.byref(sz), None) == 1
    assert L.drc_cae_forward(None, None, None, 1, 8, 8, None, None, 0, None) == 1
    assert L.drc_cae_backward(None, None, None, None, None, None, 1, 8, 8, None, 0, None) == 1
    assert L.drc_cae_set_params(None, None, None) == 1
    assert L.drc_cae_set_recompute(None, 1) == 1
    assert L.drc_cae_num_params(None) == 0
    L.drc_cae_destroy(None)
    assert "NULL" in B.drc_last_error()


def test_no_device_reports_hip_error(B):
    """Without a GPU the create call fails with DRC_ERR_HIP instead of crashing."""
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present")
    _expect(B, 5, B.drc_cae_create, B.drc_cae_default_desc(B.DRC_BF16))


def test_product_path_never_imports_oracle():
    """The HIP path and its binding share no code with the oracle."""
    pkg = os.path.join(ROOT, "paper_1910_02480_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in txt.lower() or f == "synth.py", f


def test_envmap_rejects_bad_shapes_and_pointers(B):
    L = B.lib()
    # shapes are checked first, then pointers; nothing reaches the device
    assert L.drc_envmap_build(None, 1, 0, 8, None, None, None, None) == 2
    assert L.drc_envmap_build(None, 1, 8, 1025, None, None, None, None) == 2
    assert L.drc_envmap_build(None, 1, 4097, 8, None, None, None, None) == 2
    assert L.drc_envmap_build(None, -1, 8, 8, None, None, None, None) == 2
    assert L.drc_envmap_build(None, 1, 8, 8, None, None, None, None) == 1
    assert L.drc_envmap_build(2, 1, 8, 8, 4, 4, 4, None) == 1          # misaligned d_y
    assert L.drc_envmap_build(None, 0, 8, 8, None, None, None, None) == 0  # empty batch
    assert L.drc_envmap_sample(None, None, 1, 8, 8, -1, None, None, None, None, None) == 2
    assert L.drc_envmap_sample(None, None, 1, 8, 8, 4, None, None, None, None, None) == 1
    assert L.drc_envmap_sample(None, None, 1, 8, 8, 0, None, None, None, None, None) == 0
    assert L.drc_envmap_pdf(None, None, 1, 0, 8, 4, None, None, None) == 2
    assert L.drc_envmap_pdf(None, None, 1, 8, 8, 4, None, None, None) == 1
    assert "envmap_pdf" in B.drc_last_error()


def test_interp_rejects_bad_arguments(B):
    L = B.lib()
    f = ctypes.c_float
    assert L.drc_interp_weights(None, 0, 8, 4, None, f(0.0), None, None, None) == 2
    assert L.drc_interp_weights(None, 8, 8, 0, None, f(0.0), None, None, None) == 2
    assert L.drc_interp_weights(None, 8, 8, 4, None, f(-1.0), None, None, None) == 1
    assert L.drc_interp_weights(None, 8, 8, 4, None, f(float("nan")), None, None, None) == 1
    assert L.drc_interp_weights(None, 8, 8, 4, None, f(1e-3), None, None, None) == 1
    assert L.drc_interp_weights(16, 8, 8, 4, 16, f(1e-3), 8, 16, None) == 1   # d_idx not 16-byte aligned
    assert L.drc_interp_weights(2, 8, 8, 4, 16, f(1e-3), 16, 16, None) == 1   # d_normals not 4-byte aligned


def test_augment_rejects_bad_arguments(B):
    L = B.lib()
    assert L.drc_augment(None, None, 1, 0, 8, None, None, None, None, None) == 2
    assert L.drc_augment(None, None, -1, 8, 8, None, None, None, None, None) == 2
    assert L.drc_augment(None, None, 0, 8, 8, None, None, None, None, None) == 0     # empty batch
    assert L.drc_augment(None, None, 1, 8, 8, None, None, None, None, None) == 1
    assert L.drc_augment(16, None, 1, 8, 8, 16, 16, 16, None, None) == 1            # output overlaps input
    assert L.drc_augment(16, None, 1, 8, 8, 16, 16, 4096, 64, None) == 1            # target out without target
    assert L.drc_augment(16, 64, 1, 8, 8, 16, 16, 4096, None, None) == 1            # target without target out


def test_unet_host_checks(B):
    L = B.lib()
    sz = ctypes.c_size_t()
    assert L.drc_unet_workspace_size(1, 12, 16, ctypes.byref(sz)) == 2
    assert L.drc_unet_workspace_size(0, 32, 32, ctypes.byref(sz)) == 2
    assert L.drc_unet_workspace_size(1, 32, 32, None) == 1
    assert L.drc_unet_forward(None, None, None, 1, 32, 32, None, 0, None) == 1
    assert L.drc_unet_set_params(None, None, None) == 1
    assert L.drc_unet_create(None) == 1
    from oracle import unet as U
    assert B.drc_unet_num_params() == U.num_params()


def test_wgrad_schedule_host_only(B):
    """The weight-gradient schedule is computed on the host: the parity tests'
    small batches run one strip per chunk, the benchmark's training batch
    (256 x 64x64) at least two in every BF16 layer."""
    for l in range(6):
        kind, R, spc, chunks = B.drc_cae_wgrad_schedule(B.DRC_BF16, l, 256, 64, 64)
        assert kind == 2 and R >= 4 and spc >= 2 and chunks >= 128, (l, kind, R, spc, chunks)
        kind, R, spc, chunks = B.drc_cae_wgrad_schedule(B.DRC_BF16, l, 4, 64, 64)
        assert kind == 2 and spc == 1, (l, spc)
        kind, R, per, chunks = B.drc_cae_wgrad_schedule(B.DRC_F32, l, 256, 64, 64)
        assert kind == 0 and per >= 64 and chunks >= 1
    _expect(B, 3, B.drc_cae_wgrad_schedule, B.DRC_FP8_E4M3, 0, 4, 64, 64)
    _expect(B, 1, B.drc_cae_wgrad_schedule, B.DRC_BF16, 6, 4, 64, 64)
    _expect(B, 2, B.drc_cae_wgrad_schedule, B.DRC_BF16, 0, 0, 64, 64)
    _expect(B, 2, B.drc_cae_wgrad_schedule, B.DRC_BF16, 0, 4, 60, 64)
    L = B.lib()
    assert L.drc_cae_wgrad_schedule(1, 0, 4, 64, 64, None) == 1

"""Mixed-resolution frames (one persistent, graph-captured pass over maps of
several sizes) and the tile autotuner (needs gfx950).

A map's output must not depend on the frame it sits in: the plan's result
for every map is compared bitwise with a uniform forward of that map's
resolution class, on every replay of the captured graph (with other eager
work between replays), and a sample is checked against the FP64 oracle.
"""
import numpy as np
import pytest
import torch

from paper_1910_02480_amd import binding as B
from paper_1910_02480_amd import synth
from tests.helpers import max_rel_per_map

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def params():
    return synth.init_params(0)


def _frame(sizes):
    """Packed frame of maps with the given (h, w) sizes."""
    pix = np.array([h * w for h, w in sizes], dtype=np.int64)
    xo = np.concatenate([[0], np.cumsum(pix * 7)[:-1]])
    yo = np.concatenate([[0], np.cumsum(pix * 3)[:-1]])
    x = np.empty(int(pix.sum()) * 7, dtype=np.float32)
    for m, (h, w) in enumerate(sizes):
        x[xo[m]:xo[m] + h * w * 7] = synth.radiance_map(m, h, w).reshape(-1)
    return x, xo, yo, int(pix.sum()) * 3


@pytest.mark.parametrize("compute,gate", [("bf16", 1e-2), ("f32", 1e-5)])
def test_plan_mixed_frame(oracle, params, compute, gate):
    from paper_1910_02480_amd.cae import CAE
    res = synth.mixed_resolutions(60)
    sizes = [(int(r), int(r)) for r in res] + [(24, 40), (24, 40), (24, 40)]
    x, xo, yo, ny = _frame(sizes)
    cae = CAE(compute, torch.from_numpy(params).to(DEV), device=DEV)
    maps = [(h, w, int(xo[m]), int(yo[m])) for m, (h, w) in enumerate(sizes)]
    plan = B.drc_cae_plan_create(cae.h, maps)
    try:
        ws = torch.empty(B.drc_cae_plan_workspace_size(plan) + 256, dtype=torch.uint8, device=DEV)
        ws = ws[(-ws.data_ptr()) % 256:]
        xd = torch.from_numpy(x).to(DEV)
        # reference: uniform forward of each map on its own
        ref = {}
        for m, (h, w) in enumerate(sizes):
            xm = xd[xo[m]:xo[m] + h * w * 7].view(1, h, w, 7)
            ref[m] = cae.forward(xm).cpu().numpy().reshape(-1)
        outs = []
        stream = torch.cuda.Stream(device=DEV)  # a capturable (non-null) stream
        yd = torch.empty((ny,), device=DEV)     # one output buffer: reps 2 and 3 replay the graph
        torch.cuda.synchronize()
        for rep in range(3):
            with torch.cuda.stream(stream):
                yd.fill_(float("nan"))
                B.drc_cae_plan_launch(plan, xd, yd, ws)      # captured once, then replayed
                junk = torch.randn(1 << 20, device=DEV).sum()  # eager work between replays
            torch.cuda.synchronize()
            y = yd.cpu().numpy()
            for m, (h, w) in enumerate(sizes):
                np.testing.assert_array_equal(y[yo[m]:yo[m] + h * w * 3], ref[m], err_msg=f"rep {rep} map {m}")
            outs.append(y)
            del junk
        assert B.drc_cae_plan_captures(plan) == 1
        # null stream: direct launches, same result
        yd = torch.zeros((ny,), device=DEV)
        B.drc_cae_plan_launch(plan, xd, yd, ws, stream=0)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(yd.cpu().numpy(), outs[0])
    finally:
        B.drc_cae_plan_destroy(plan)
    # oracle on one map of each size
    seen = {}
    for m, s in enumerate(sizes):
        seen.setdefault(s, m)
    for (h, w), m in seen.items():
        r = oracle.forward(params, synth.radiance_map(m, h, w)[None])["y"]
        g = outs[0][yo[m]:yo[m] + h * w * 3].reshape(1, h, w, 3)
        assert max_rel_per_map(g, r).max() <= gate, (h, w)


def test_plan_validation(params):
    from paper_1910_02480_amd.cae import CAE
    cae = CAE("bf16", torch.from_numpy(params).to(DEV), device=DEV)
    with pytest.raises(B.DrcError) as e:
        B.drc_cae_plan_create(cae.h, [])
    assert e.value.status == 2
    with pytest.raises(B.DrcError) as e:
        B.drc_cae_plan_create(cae.h, [(30, 32, 0, 0)])
    assert e.value.status == 2
    with pytest.raises(B.DrcError) as e:
        B.drc_cae_plan_create(cae.h, [(8 * (k + 1), 8, 0, 0) for k in range(5)])
    assert e.value.status == 3
    plan = B.drc_cae_plan_create(cae.h, [(32, 32, 0, 0)])
    try:
        need = B.drc_cae_plan_workspace_size(plan)
        ws = torch.empty(need, dtype=torch.uint8, device=DEV)
        x = torch.zeros(32 * 32 * 7, device=DEV)
        y = torch.zeros(32 * 32 * 3, device=DEV)
        with pytest.raises(B.DrcError) as e:
            B.drc_cae_plan_launch(plan, x, y, ws[: need - 256] if need > 256 else ws[:0])
        assert e.value.status in (1, 4)
    finally:
        B.drc_cae_plan_destroy(plan)


def test_autotune_keeps_results_bitwise(tmp_path, params):
    """Tile shapes change the schedule only: outputs stay bitwise equal."""
    from paper_1910_02480_amd.cae import CAE
    cae = CAE("bf16", torch.from_numpy(params).to(DEV), device=DEV)
    x = torch.from_numpy(synth.radiance_maps(64, 64, 64)).to(DEV)
    y0 = cae.forward(x).cpu().numpy()
    cache = str(tmp_path / "tune.jsonl")
    n, H, W = 64, 64, 64
    ws = cae.workspace(n, H, W, B.DRC_WS_AUTOTUNE)
    B.drc_cae_autotune(cae.h, x, ws, cache)
    lines = open(cache).read().strip().split("\n")
    assert len(lines) == 6 and all('"layer"' in ln and '"npw"' in ln for ln in lines)
    y1 = cae.forward(x).cpu().numpy()
    np.testing.assert_array_equal(y0, y1)
    # a plan reads the cache and agrees too
    maps = [(64, 64, k * 64 * 64 * 7, k * 64 * 64 * 3) for k in range(n)]
    plan = B.drc_cae_plan_create(cae.h, maps, cache)
    try:
        w2 = torch.empty(B.drc_cae_plan_workspace_size(plan), dtype=torch.uint8, device=DEV)
        yd = torch.empty(n * H * W * 3, device=DEV)
        B.drc_cae_plan_launch(plan, x.reshape(-1), yd, w2)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(yd.cpu().numpy(), y0.reshape(-1))
    finally:
        B.drc_cae_plan_destroy(plan)


@pytest.mark.parametrize("compute", ["bf16", "fp8"])
def test_layer_e1_staged_matches_gather(params, compute):
    """E1 of the layer path (BF16, FP8) stages the float32 input rows in LDS
    when every map starts on a 16-byte boundary and gathers it per lane
    otherwise; both give bitwise-equal outputs (same operands, K order and
    rounding). Frames with the maps packed, and with every map shifted by a
    few floats, are compared map by map (32x32, 64x64, 128x128 through the
    layer kernels, and a size the staged kernel does not take)."""
    from paper_1910_02480_amd.cae import CAE
    sizes = [(128, 128), (32, 32), (64, 64), (128, 128), (40, 40), (32, 32)]
    x, xo, yo, ny = _frame(sizes)
    shift = np.array([1 + m % 3 for m in range(len(sizes))])           # 1..3 floats: not 16-byte aligned
    xo_u = xo + np.cumsum(shift)
    xu = np.zeros(len(x) + int(shift.sum()), dtype=np.float32)
    for m, (h, w) in enumerate(sizes):
        xu[xo_u[m]:xo_u[m] + h * w * 7] = x[xo[m]:xo[m] + h * w * 7]
    cae = CAE(compute, torch.from_numpy(params).to(DEV), device=DEV)
    cae.set_fused(False)
    if compute == "fp8":
        cae.calibrate_fp8(torch.from_numpy(synth.radiance_maps(4, 64, 64, seed=3)).to(DEV))
    ys = []
    for xx, offs in ((x, xo), (xu, xo_u)):
        maps = [(h, w, int(offs[m]), int(yo[m])) for m, (h, w) in enumerate(sizes)]
        plan = B.drc_cae_plan_create(cae.h, maps)
        try:
            ws = torch.empty(B.drc_cae_plan_workspace_size(plan) + 256, dtype=torch.uint8, device=DEV)
            ws = ws[(-ws.data_ptr()) % 256:]
            yd = torch.full((ny,), float("nan"), device=DEV)
            B.drc_cae_plan_launch(plan, torch.from_numpy(xx).to(DEV), yd, ws, stream=0)
            torch.cuda.synchronize()
            ys.append(yd.cpu().numpy())
        finally:
            B.drc_cae_plan_destroy(plan)
    assert np.all(np.isfinite(ys[0]))
    for m, (h, w) in enumerate(sizes):
        np.testing.assert_array_equal(ys[0][yo[m]:yo[m] + h * w * 3], ys[1][yo[m]:yo[m] + h * w * 3],
                                      err_msg=f"map {m} ({h}x{w})")


def test_plan_recaptures_after_handle_changes(params):
    """A plan's graph bakes in kernel arguments of the handle (FP8 scales, the
    fused or layer route, tile shapes). After set_params with doubled weights
    and a new FP8 calibration, or a switch of the route, the next launch on
    the same buffers records the graph again and equals an eager forward."""
    from paper_1910_02480_amd.cae import CAE
    sizes = [(32, 32)] * 3 + [(64, 64)] * 2 + [(128, 128)]
    x, xo, yo, ny = _frame(sizes)
    maps = [(h, w, int(xo[m]), int(yo[m])) for m, (h, w) in enumerate(sizes)]
    xd = torch.from_numpy(x).to(DEV)
    calib = torch.from_numpy(synth.radiance_maps(8, 64, 64, seed=3)).to(DEV)
    stream = torch.cuda.Stream(device=DEV)
    for compute in ("fp8", "bf16"):
        cae = CAE(compute, torch.from_numpy(params).to(DEV), device=DEV)
        if compute == "fp8":
            cae.calibrate_fp8(calib)
        plan = B.drc_cae_plan_create(cae.h, maps)
        try:
            ws = torch.empty(B.drc_cae_plan_workspace_size(plan) + 256, dtype=torch.uint8, device=DEV)
            ws = ws[(-ws.data_ptr()) % 256:]
            yd = torch.empty((ny,), device=DEV)

            def launch_and_compare(tag):
                with torch.cuda.stream(stream):
                    yd.fill_(float("nan"))
                    B.drc_cae_plan_launch(plan, xd, yd, ws)
                torch.cuda.synchronize()
                y = yd.cpu().numpy()
                for m, (h, w) in enumerate(sizes):
                    xm = xd[xo[m]:xo[m] + h * w * 7].view(1, h, w, 7)
                    ref = cae.forward(xm).cpu().numpy().reshape(-1)
                    np.testing.assert_array_equal(y[yo[m]:yo[m] + h * w * 3], ref, err_msg=f"{tag} map {m}")
                return y

            y0 = launch_and_compare(f"{compute} first")
            launch_and_compare(f"{compute} replay")
            assert B.drc_cae_plan_captures(plan) == 1
            cae.set_params(torch.from_numpy(2.0 * params).to(DEV))
            if compute == "fp8":
                cae.calibrate_fp8(calib)
            y1 = launch_and_compare(f"{compute} new weights")
            assert not np.array_equal(y0, y1)
            if compute == "bf16":
                cae.set_fused(False)
                y2 = launch_and_compare("bf16 layer route")
                np.testing.assert_array_equal(y1, y2)  # both routes agree bit for bit
            assert B.drc_cae_plan_captures(plan) == (3 if compute == "bf16" else 2)
        finally:
            B.drc_cae_plan_destroy(plan)

"""The training step recorded as a HIP graph and replayed
(drc_cae_step_graph_*), needs gfx950: replayed steps equal eager
drc_cae_step calls bit for bit (parameters, Adam moments, loss), with the
step count changing every replay and eager work between replays."""
import numpy as np
import pytest
import torch

from paper_1910_02480_amd import binding as B
from paper_1910_02480_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.mark.parametrize("compute,H,recompute", [("bf16", 64, True), ("bf16", 32, False), ("f32", 32, True)])
def test_step_graph_replays_equal_eager_steps(compute, H, recompute):
    from paper_1910_02480_amd.cae import CAE, GraphTrainer, Trainer
    n = 16
    x, t = synth.training_batch(n, H)
    x, t = torch.from_numpy(x).to(DEV), torch.from_numpy(t).to(DEV)
    p0 = torch.from_numpy(synth.init_params(0)).to(DEV)
    eager = Trainer(CAE(compute, device=DEV, recompute=recompute), p0.clone(), lr=1e-3)
    graph = GraphTrainer(CAE(compute, device=DEV, recompute=recompute), p0.clone(), lr=1e-3)
    ge, gg = torch.empty_like(p0), torch.empty_like(p0)
    try:
        for step in range(1, 4):
            le = float(eager.step(x, t, dparams=ge))
            lg = float(graph.step(x, t, dparams=gg))
            junk = torch.randn(1 << 20, device=DEV).sum()  # eager work between replays
            torch.cuda.synchronize()
            print(f"{compute} {H}x{H} step {step}: loss {le:.6f} / {lg:.6f}", flush=True)
            assert le == lg, step
            np.testing.assert_array_equal(ge.cpu().numpy(), gg.cpu().numpy(), err_msg=f"gradient, step {step}")
            for name in ("params", "m", "v"):
                np.testing.assert_array_equal(getattr(eager, name).cpu().numpy(),
                                              getattr(graph, name).cpu().numpy(), err_msg=f"{name}, step {step}")
            del junk
        assert B.drc_cae_step_graph_captures(graph.g) == 1
        # a handle change (route switch) records the step again; results stay equal
        graph.cae.set_fused(not (compute == "bf16"))
        eager.cae.set_fused(not (compute == "bf16"))
        le = float(eager.step(x, t, dparams=ge))
        lg = float(graph.step(x, t, dparams=gg))
        torch.cuda.synchronize()
        assert le == lg
        np.testing.assert_array_equal(eager.params.cpu().numpy(), graph.params.cpu().numpy())
        assert B.drc_cae_step_graph_captures(graph.g) == 2
    finally:
        graph.close()


def test_step_graph_rejects_bad_arguments():
    from paper_1910_02480_amd.cae import CAE
    import ctypes
    L = B.lib()
    cae = CAE("bf16", device=DEV)
    p = torch.from_numpy(synth.init_params(0)).to(DEV)
    adam = B.drc_adam_cfg(6e-5, 0.9, 0.999, 1e-8)
    g = ctypes.c_void_p()
    x = torch.zeros((2, 32, 32, 7), device=DEV)
    ws = cae.workspace(2, 32, 32, B.DRC_WS_STEP)
    s = torch.cuda.Stream(device=DEV)
    args = lambda stream: (cae.h, p.data_ptr(), p.data_ptr(), p.data_ptr(), ctypes.byref(adam), x.data_ptr(),  # noqa: E731
                           x.data_ptr(), p.data_ptr(), None, 2, 32, 32, ws.data_ptr(), ws.numel(), stream,
                           ctypes.byref(g))
    assert L.drc_cae_step_graph_create(*args(None)) == 1          # the null stream cannot be captured
    a = list(args(s.cuda_stream))
    a[10] = 30
    assert L.drc_cae_step_graph_create(*a) == 2                    # H not a multiple of 8
    assert L.drc_cae_step_graph_create(*args(s.cuda_stream)[:-1], None) == 1
    assert L.drc_cae_step_graph_launch(None, 1) == 1

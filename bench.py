#!/usr/bin/env python3
"""Throughput of the radiance-cache autoencoder hot path on one MI355X.

One timed step = one forward pass of the autoencoder over a batch of 4096
cache-point maps of 64x64 (7 channels in, 3 out) in BF16 on MFMA, inputs
already resident in HBM. The JSON line also carries the other legs of the
metric (FP32 forward, FP8 forward, forward+backward, the training step with
Adam), the roofline position of the dominant kernel measured live with HIP
events, and the FP64 oracle timed on the host cores.

Progress goes to stderr; stdout gets exactly one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
import time

METRIC = "maps/s CAE fwd & fwd+bwd, 64x64 maps; BF16 vs FP32 at rel-err<=1e-2"
PEAK_HBM_GBS = 8000.0
PEAK_TFLOPS = {"f32": 157.3, "bf16": 2500.0, "fp8": 5000.0}
LAYERS = (("E1", False, 7, 32), ("E2", False, 32, 64), ("E3", False, 64, 128),
          ("D3", True, 128, 64), ("D2", True, 128, 32), ("D1", True, 64, 3))
ESIZE = {"f32": 4, "bf16": 2, "fp8": 1}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def layer_io(l, H):
    din = (1, 2, 4, 8, 4, 2)[l]
    dout = (2, 4, 8, 4, 2, 1)[l]
    return H // din, H // dout


def layer_cost(l, n, H, compute):
    """Algorithmic FLOPs and HBM bytes of one forward launch of layer l.

    FLOPs are nominal: 2 * Cout * Cin * 9 per output pixel of a convolution
    and per input pixel of a transposed convolution. Bytes: the layer input
    (float32 x for E1, else the stored activations), its output (float32 y
    for D1), and the packed weights once.
    """
    name, tconv, cin, cout = LAYERS[l]
    hin, hout = layer_io(l, H)
    pin, pout = n * hin * hin, n * hout * hout
    flops = 2.0 * cout * cin * 9 * (pin if tconv else pout)
    es = ESIZE[compute]
    bytes_in = pin * cin * (4 if l == 0 else es)
    bytes_out = pout * cout * (4 if l == 5 else es)
    bytes_w = cout * 9 * cin * es
    return flops, bytes_in + bytes_out + bytes_w


FUSED_SLOT = 21  # timing slot of the whole-network kernel


def fused_cost(n, H):
    """Algorithmic FLOPs and HBM bytes of one whole-network forward launch:
    all six layers' nominal FLOPs; bytes = float32 x in (7 ch), float32 y
    out (3 ch) and the BF16 weight packs once (activations stay on chip)."""
    flops = sum(layer_cost(l, n, H, "bf16")[0] for l in range(6))
    w = sum(cout * 9 * cin * 2 for _, _, cin, cout in LAYERS)
    return flops, n * H * H * (7 + 3) * 4 + w


def gen_maps(n, H, chunk=512):
    import numpy as np
    import torch
    from paper_1910_02480_amd import synth
    x = torch.empty((n, H, H, 7), dtype=torch.float32)
    for s in range(0, n, chunk):
        k = min(chunk, n - s)
        x[s:s + k] = torch.from_numpy(synth.radiance_maps(k, H, H, start=s))
    return x


SETTLE_S = 0.3  # set from --settle-ms


def settle(fn):
    """Run the workload for SETTLE_S seconds before its warmup steps: the GPU
    clock ramps up over the first ~20 ms of sustained load, and the timed
    steps should see the steady state."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < SETTLE_S:
        for _ in range(4):
            fn()
        torch.cuda.synchronize()


def timed(fn, steps, warmup, do_settle=True):
    import torch
    if do_settle:
        settle(fn)
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def event_timed(fn, steps, warmup):
    """Seconds per call from HIP events recorded on the current stream (the
    stream the library launches on) around `steps` back-to-back calls."""
    import torch
    settle(fn)
    for _ in range(warmup):
        fn()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(steps):
        fn()
    b.record()
    b.synchronize()
    return a.elapsed_time(b) * 1e-3 / steps


def envmap_leg(B, y, steps, warmup, samples=64):
    """Sampling tables of the forward's predicted maps (drc_envmap_build),
    then `samples` directions per map and their densities. HBM-bound: the
    build reads y (12 B per pixel) and writes the CDFs (4 B per pixel, 4 B
    per row, 4 B per map); a sample reads 8 B of uniforms and writes 20 B, a
    density evaluation reads 12 B and writes 4 B (table reads hit the caches)."""
    import torch
    n, H, W, _ = y.shape
    dev = y.device
    cu = torch.empty((n, H, W), device=dev)
    cv = torch.empty((n, H), device=dev)
    tot = torch.empty((n,), device=dev)
    tb = event_timed(lambda: B.drc_envmap_build(y, cu, cv, tot), steps, warmup)
    gen = torch.Generator(device=dev)
    gen.manual_seed(7)
    xi = torch.rand((n, samples, 2), generator=gen, device=dev)
    d = torch.empty((n, samples, 3), device=dev)
    p = torch.empty((n, samples), device=dev)
    pix = torch.empty((n, samples), dtype=torch.int32, device=dev)
    ts = event_timed(lambda: B.drc_envmap_sample(cu, cv, xi, d, p, pix), steps, warmup)
    p2 = torch.empty_like(p)
    tp = event_timed(lambda: B.drc_envmap_pdf(cu, cv, d, p2), steps, warmup)
    bb = n * (H * W * 16 + 4 * H + 4)
    bs = n * samples * 28
    bp = n * samples * 16
    return {"maps": n, "H": H, "W": W, "samples_per_map": samples,
            "build_ms": tb * 1e3, "build_maps_per_s": n / tb, "build_GB/s": bb / tb / 1e9,
            "build_hbm_frac": bb / tb / 1e9 / PEAK_HBM_GBS, "build_alg_bytes": bb,
            "sample_ms": ts * 1e3, "samples_per_s": n * samples / ts, "sample_GB/s": bs / ts / 1e9,
            "pdf_ms": tp * 1e3, "pdf_evals_per_s": n * samples / tp, "pdf_GB/s": bp / tp / 1e9}


def interp_leg(B, dev, steps, warmup, Hi=1080, Wi=1920, r=16, eps=1e-4):
    """Cache-point interpolation weights of one Hi x Wi frame with a grid of
    spacing r (drc_interp_weights). HBM-bound: 12 B of normal in and 32 B
    of indices and probabilities out per pixel (cache normals hit the caches)."""
    import torch
    from paper_1910_02480_amd import synth
    n = torch.from_numpy(synth.gbuffer_normals(Hi, Wi)).to(dev)
    cn = n[::r, ::r].contiguous()
    idx = torch.empty((Hi, Wi, 4), dtype=torch.int32, device=dev)
    prob = torch.empty((Hi, Wi, 4), device=dev)
    t = event_timed(lambda: B.drc_interp_weights(n, r, cn, eps, idx, prob), steps, warmup)
    by = Hi * Wi * 44 + cn.numel() * 4
    return {"image": [Hi, Wi], "r": r, "cache_points": int(cn.shape[0] * cn.shape[1]), "ms": t * 1e3,
            "pixels_per_s": Hi * Wi / t, "GB/s": by / t / 1e9, "hbm_frac": by / t / 1e9 / PEAK_HBM_GBS,
            "alg_bytes": by}


def unet_train_leg(B, dev, steps, warmup, n=32, H=32):
    """The paper's own network, one FP32 training step (batch statistics,
    L1 loss, backward, Adam) on n maps of H x H: the paper's batch (32) and
    map size. FLOPs nominal: 3x the forward's (forward, data and weight
    gradients)."""
    import torch
    from paper_1910_02480_amd import synth
    div = (1, 1, 2, 2, 4, 4, 8, 8, 4, 4, 2, 2, 1, 1, 1)
    flops = 3 * sum(2.0 * co * ci * (1 if name == "out" else 9) * n * (H // d) ** 2
                    for (name, ci, co, _), d in zip(synth.UNET_LAYERS, div))
    p = torch.from_numpy(synth.unet_flat(synth.unet_params(0))).to(dev)
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    xs, ts = synth.training_batch(n, H)
    x, t = torch.from_numpy(xs).to(dev), torch.from_numpy(ts).to(dev)
    ws = torch.empty(B.drc_unet_train_workspace_size(n, H, H) + 256, dtype=torch.uint8, device=dev)
    ws = ws[(-ws.data_ptr()) % 256:]
    loss = torch.zeros(1, device=dev)
    adam = B.drc_adam_cfg(6e-5, 0.9, 0.999, 1e-8)
    cnt = [0]

    def step():
        cnt[0] += 1
        B.drc_unet_train_step(p, m, v, cnt[0], adam, x, t, loss, None, None, ws)
    tm = event_timed(step, steps, warmup)
    return {"maps": n, "H": H, "precision": "f32", "ms": tm * 1e3, "maps_per_s": n / tm,
            "TFLOP/s": flops / tm / 1e12, "mfma_frac_flop_based": flops / tm / (PEAK_TFLOPS["f32"] * 1e12),
            "loss_after": float(loss)}


def unet_leg(B, dev, steps, warmup, n=4096, H=32):
    """The paper's own network (inference, BF16 activations) over n maps of
    H x H, the paper's map size. FLOPs are nominal: 2 * cout * cin * taps per
    output pixel of every convolution."""
    import torch
    from paper_1910_02480_amd import synth
    div = (1, 1, 2, 2, 4, 4, 8, 8, 4, 4, 2, 2, 1, 1, 1)  # resolution divisor per layer
    flops = sum(2.0 * co * ci * (1 if name == "out" else 9) * n * (H // d) ** 2
                for (name, ci, co, _), d in zip(synth.UNET_LAYERS, div))
    u = B.drc_unet_create()
    try:
        B.drc_unet_set_params(u, torch.from_numpy(synth.unet_flat(synth.unet_params(0))).to(dev))
        x = gen_maps(n, H).to(dev)
        y = torch.empty((n, H, H, 3), device=dev)
        ws = torch.empty(B.drc_unet_workspace_size(n, H, H) + 256, dtype=torch.uint8, device=dev)
        ws = ws[(-ws.data_ptr()) % 256:]
        t = event_timed(lambda: B.drc_unet_forward(u, x, y, ws), steps, warmup)
    finally:
        B.drc_unet_destroy(u)
    return {"maps": n, "H": H, "ms": t * 1e3, "maps_per_s": n / t, "gflop_per_map": flops / n / 1e9,
            "TFLOP/s": flops / t / 1e12, "mfma_frac_flop_based": flops / t / (PEAK_TFLOPS["bf16"] * 1e12)}


def read_profile(B, h):
    return B.drc_cae_profile_read(h)


def host_cpu():
    """CPU model name, current clock (MHz) and logical CPUs of this host."""
    model, mhz = "unknown", None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name") and model == "unknown":
                model = line.split(":", 1)[1].strip()
            if line.startswith("cpu MHz") and mhz is None:
                mhz = float(line.split(":", 1)[1])
    except OSError:
        pass
    return {"model": model, "mhz": mhz, "logical_cpus": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0))}


_SINGLE_CORE = """
import sys, time
sys.path.insert(0, {root!r})
from oracle import oracle as O
from paper_1910_02480_amd import synth
p = synth.init_params(0)
x = synth.radiance_maps({n}, {H}, {H})
O.forward(p, x[:1])
t0 = time.perf_counter()
O.forward(p, x)
print({n} / (time.perf_counter() - t0))
"""


def cpu_baseline(x_sample_fn, H, budget_s, len_x, train_maps):
    """FP64 oracle on the host, on bounded samples of the workloads: the
    forward over a prefix of the benchmark batch (about budget_s of work),
    the training step (forward, L1 loss and gradient, backward, Adam) over
    the training batch, and the forward on one core."""
    import subprocess
    import numpy as np
    from oracle import oracle as O
    from paper_1910_02480_amd import synth
    params = synth.init_params(0)
    O.build()
    x1 = x_sample_fn(1)
    t0 = time.perf_counter()
    O.forward(params, x1)
    t1 = time.perf_counter() - t0
    n = int(max(1, min(len_x, budget_s / max(t1, 1e-3))))
    xs = x_sample_fn(n)
    t0 = time.perf_counter()
    O.forward(params, xs)
    passes = 1
    # the whole batch may take less than the budget on many cores: repeat it
    while time.perf_counter() - t0 < 0.5 * budget_s and passes < 16:
        O.forward(params, xs)
        passes += 1
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or len(os.sched_getaffinity(0))
    out = {"value": n * passes / dt, "unit": "maps/s", "cores": threads, "kind": "oracle",
           "sample": f"FP64 oracle forward of maps 0..{n - 1} of the {H}x{H} workload, {passes} pass(es) "
                     f"({dt:.1f} s, {threads} OpenMP threads)", "host": host_cpu()}
    # training step of the training batch (the oracle's plain Adam in float64)
    xt, tg = synth.training_batch(train_maps, H)
    t0 = time.perf_counter()
    a = O.forward(params, xt)
    loss, dy = O.l1(a["y"], tg)
    g, _ = O.backward(params, xt, a, dy)
    O.adam(params, np.zeros_like(params), np.zeros_like(params), g, 1)
    ts = time.perf_counter() - t0
    out["train_step"] = {"maps": train_maps, "s_per_step": ts, "maps_per_s": train_maps / ts,
                         "sample": f"one FP64 oracle training step (forward, L1, backward, Adam) on the "
                                   f"{train_maps}-map {H}x{H} training batch, {threads} OpenMP threads"}
    # one core: a child process with one OpenMP thread
    n1 = max(1, min(64, int(round(2.0 / max(t1, 1e-3)))))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    root = os.path.dirname(os.path.abspath(__file__))
    r = subprocess.run([sys.executable, "-c", _SINGLE_CORE.format(root=root, n=n1, H=H)], env=env,
                       capture_output=True, text=True, timeout=600)
    if r.returncode == 0:
        out["single_core"] = {"maps_per_s": float(r.stdout.strip().splitlines()[-1]), "maps": n1,
                              "sample": f"FP64 oracle forward of maps 0..{n1 - 1}, OMP_NUM_THREADS=1"}
    return out


def accuracy(outputs, x_host, params_np, k):
    """C16 error metrics of each precision's outputs over maps 0..k-1 of the
    benchmark batch against the FP64 oracle: per map max_rel = max|y - r| /
    max|r| and mean_rel = sum|y - r| / sum|r|; reported as max, mean and
    p99 over the maps."""
    import numpy as np
    from oracle import oracle as O
    ref = O.forward(params_np, x_host[:k].numpy())["y"].reshape(k, -1)
    res = {"maps_checked": k, "subset": f"maps 0..{k - 1} of the benchmark batch"}
    for name, y in outputs.items():
        y = y[:k].reshape(k, -1).astype(np.float64)
        d = np.abs(y - ref)
        mx = d.max(1) / np.abs(ref).max(1)
        mn = d.sum(1) / np.abs(ref).sum(1)
        res[name] = {"max_rel_max": float(mx.max()), "max_rel_p99": float(np.percentile(mx, 99)),
                     "max_rel_mean": float(mx.mean()), "mean_rel_mean": float(mn.mean()),
                     "mean_rel_max": float(mn.max())}
    return res


def mixed_frame_leg(cae, tune_path, args):
    """6000 cache points (50 % 32x32, 35 % 64x64, 15 % 128x128, shuffled),
    BF16, one hipGraph-captured pass per frame; p50/p99 latency
    over replays. Tile shapes come from the autotuner, run per resolution."""
    import numpy as np
    import torch
    from paper_1910_02480_amd import binding as B
    from paper_1910_02480_amd import synth
    dev = cae.device
    res = synth.mixed_resolutions(args.frame_maps)
    log(f"mixed frame: generating {len(res)} maps")
    x, xo, yo = synth.mixed_frame(res)
    ny = int((res.astype(np.int64) ** 2).sum()) * 3
    for r in (32, 64, 128):
        k = {32: 512, 64: 256, 128: 64}[r]
        xt = torch.from_numpy(synth.radiance_maps(k, r, r, seed=5)).to(dev)
        B.drc_cae_autotune(cae.h, xt, cae.workspace(k, r, r, B.DRC_WS_AUTOTUNE), tune_path)
        del xt
    maps = [(int(r), int(r), int(xo[m]), int(yo[m])) for m, r in enumerate(res)]
    plan = B.drc_cae_plan_create(cae.h, maps, tune_path)
    try:
        nb = B.drc_cae_plan_workspace_size(plan)
        wsb = torch.empty(nb + 256, dtype=torch.uint8, device=dev)
        ws = wsb[(-wsb.data_ptr()) % 256:]
        xd = torch.from_numpy(x).to(dev)
        yd = torch.empty(ny, device=dev)
        stream = torch.cuda.Stream(device=dev)
        torch.cuda.synchronize()
        reps = args.frame_reps
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        with torch.cuda.stream(stream):
            settle(lambda: B.drc_cae_plan_launch(plan, xd, yd, ws))
            for _ in range(10):
                B.drc_cae_plan_launch(plan, xd, yd, ws)
            for e0, e1 in ev:
                e0.record(stream)
                B.drc_cae_plan_launch(plan, xd, yd, ws)
                e1.record(stream)
        torch.cuda.synchronize()
        lat = np.array([e0.elapsed_time(e1) for e0, e1 in ev])
        p50, p99 = float(np.percentile(lat, 50)), float(np.percentile(lat, 99))
        flops = sum(13392.0 * int(r) * int(r) for r in res)
        log(f"mixed frame ({len(res)} maps): p50 {p50:.3f} ms, p99 {p99:.3f} ms, {len(res) / p50 * 1e3:,.0f} maps/s")
        return {"maps": len(res), "p50_ms": p50, "p99_ms": p99, "maps_per_s": len(res) / p50 * 1e3,
                "replays": reps, "gflop_per_frame": flops / 1e9,
                "mfma_frac_flop_based": flops / (p50 * 1e-3) / (PEAK_TFLOPS["bf16"] * 1e12)}
    finally:
        B.drc_cae_plan_destroy(plan)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--maps", type=int, default=4096)
    ap.add_argument("--res", type=int, default=64)
    ap.add_argument("--train-maps", type=int, default=256)
    ap.add_argument("--main-only", action="store_true", help="time only the headline leg")
    ap.add_argument("--with-envmap", action="store_true",
                    help="with --main-only: also time the sampling tables of the forward's output")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-calib", action="store_true",
                    help="first run a plain 256 MiB device copy (reference for HBM byte counters)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--settle-ms", type=float, default=300.0,
                    help="run each leg's workload this long before its warmup steps (clock ramp-up)")
    ap.add_argument("--frame-maps", type=int, default=6000)
    ap.add_argument("--frame-reps", type=int, default=200)
    ap.add_argument("--frame-only", action="store_true",
                    help="time only the mixed frame (for a kernel trace of it); prints that leg, not the bench line")
    args = ap.parse_args()

    global SETTLE_S
    SETTLE_S = max(0.0, args.settle_ms) * 1e-3
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the autoencoder path is built and measured on one "
              "MI355X; multi-GPU sharding is design only (see the design notes).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1910_02480_amd import binding as B
    from paper_1910_02480_amd import synth
    from paper_1910_02480_amd.cae import CAE, Trainer

    dev = torch.device("cuda:0")
    if args.frame_only:
        params = torch.from_numpy(synth.init_params(0)).to(dev)
        cae = CAE("bf16", params, device=dev)
        tune_path = os.path.join(tempfile.gettempdir(), f"drc_tune_{os.getpid()}.jsonl")
        print(json.dumps({"bf16_mixed_frame": mixed_frame_leg(cae, tune_path, args)}), flush=True)
        return
    n, H = args.maps, args.res
    log(f"generating {n} maps of {H}x{H}")
    x_host = gen_maps(n, H)
    x = x_host.to(dev)
    params = torch.from_numpy(synth.init_params(0)).to(dev)
    y = torch.empty((n, H, H, 3), dtype=torch.float32, device=dev)
    legs = {}

    if args.copy_calib:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)  # 256 MiB
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 2.0, out=dst)  # one elementwise kernel: reads 256 MiB, writes 256 MiB
        torch.cuda.synchronize()
        del src, dst
    # ---------------- headline: BF16 forward, profiled live
    cae = CAE("bf16", params, device=dev)
    tune_path = os.path.join(tempfile.gettempdir(), f"drc_tune_{os.getpid()}.jsonl")
    fused_headline = H in (32, 64)  # BF16 maps of these sizes run the whole-network kernel
    if not args.no_autotune and not fused_headline:
        log("autotuning tile shapes for the headline batch")
        B.drc_cae_autotune(cae.h, x, cae.workspace(n, H, H, B.DRC_WS_AUTOTUNE), tune_path)
    ws = cae.workspace(n, H, H, B.DRC_WS_FORWARD)
    fwd = lambda: B.drc_cae_forward(cae.h, x, y, None, ws)
    settle(fwd)
    for _ in range(args.warmup):
        fwd()
    torch.cuda.synchronize()
    B.drc_cae_profile(cae.h, 1)
    read_profile(B, cae.h)
    if fused_headline:
        # one launch per forward: one profiled call shows that it is the
        # whole-network kernel alone; the timed steps then run without
        # per-launch events (they cost ~1.7 % of a 0.43 ms step), and two
        # HIP events on the launch stream around the timed region give the
        # kernel's average duration (gaps between launches included)
        fwd()
        ms_1, calls_1 = read_profile(B, cae.h)
        B.drc_cae_profile(cae.h, 0)
        if calls_1[FUSED_SLOT] != 1 or sum(calls_1) != 1:
            raise RuntimeError(f"bf16 forward of {n}x{H}x{H}: expected one whole-network launch, got {calls_1}")
        log(f"timing bf16 forward: {args.steps} steps")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record()
        for _ in range(args.steps):
            fwd()
        e1.record()
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / args.steps
        ms_l = [0.0] * len(ms_1)
        calls_l = [0] * len(calls_1)
        ms_l[FUSED_SLOT] = e0.elapsed_time(e1)
        calls_l[FUSED_SLOT] = args.steps
    else:
        log(f"timing bf16 forward: {args.steps} steps")
        t = timed(fwd, args.steps, 0, do_settle=False)
        ms_l, calls_l = read_profile(B, cae.h)
        B.drc_cae_profile(cae.h, 0)
    ACC_MAPS = min(512, n)  # maps checked against the oracle
    y_bf16 = y[:ACC_MAPS].cpu().numpy()
    value = n / t
    kernels = []
    tot_ms = max(sum(ms_l[:6]) + ms_l[FUSED_SLOT], 1e-30)
    for l in range(6):
        if calls_l[l] == 0:
            continue
        avg = ms_l[l] / calls_l[l] * 1e-3
        fl, by = layer_cost(l, n, H, "bf16")
        kernels.append({"kernel": f"forward {LAYERS[l][0]}", "avg_ms": avg * 1e3, "share": ms_l[l] / tot_ms,
                        "GB/s": by / avg / 1e9, "TFLOP/s": fl / avg / 1e12,
                        "alg_bytes": by, "alg_flops": fl})
    if calls_l[FUSED_SLOT]:
        avg = ms_l[FUSED_SLOT] / calls_l[FUSED_SLOT] * 1e-3
        fl, by = fused_cost(n, H)
        kernels.append({"kernel": "forward fused", "avg_ms": avg * 1e3, "share": ms_l[FUSED_SLOT] / tot_ms,
                        "GB/s": by / avg / 1e9, "TFLOP/s": fl / avg / 1e12,
                        "alg_bytes": by, "alg_flops": fl})
    dom = max(kernels, key=lambda k: k["avg_ms"] * 1.0)
    ai = dom["alg_flops"] / dom["alg_bytes"]
    ridge = PEAK_TFLOPS["bf16"] * 1e12 / (PEAK_HBM_GBS * 1e9)
    if ai < ridge:
        roof = {"bound": "hbm", "achieved": dom["GB/s"], "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": dom["GB/s"] / PEAK_HBM_GBS}
    else:
        roof = {"bound": "mfma", "achieved": dom["TFLOP/s"], "peak": PEAK_TFLOPS["bf16"],
                "unit": "TFLOP/s", "frac": dom["TFLOP/s"] / PEAK_TFLOPS["bf16"]}
    # HBM bytes per launch from the committed counter runs, if the kernels are unchanged since
    from paper_1910_02480_amd import prof_summary
    tr = prof_summary.read_traffic(os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                                                f"cae_forward_bf16_{n}x{H}x{H}_traffic.md"))
    traffic = None
    if tr and dom["kernel"] in tr["kernels"]:
        traffic = tr["kernels"][dom["kernel"]]["bytes_per_launch"]
    # rocprof MFMA-busy fraction (padding lanes counted) and LDS bank-conflict
    # share of the same kernel, from the committed SQ counter runs while fresh
    sq = prof_summary.read_counters(os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                                                 f"cae_forward_bf16_{n}x{H}x{H}_counters.md"))
    sqk = sq["kernels"].get(dom["kernel"], {}) if sq else {}
    roof.update({"mfma_busy_rocprof": sqk.get("mfma_busy"), "lds_bank_conflict_share": sqk.get("lds_conflict")})
    roof.update({"kernel": dom["kernel"], "traffic": traffic, "traffic_unit": "bytes per launch",
                 "avg_ms": dom["avg_ms"],
                 "alg_bytes_per_launch": dom["alg_bytes"], "alg_flops_per_launch": dom["alg_flops"]})
    total_flops = sum(layer_cost(l, n, H, "bf16")[0] for l in range(6))
    legs["bf16_fwd"] = {"maps_per_s": value, "ms": t * 1e3,
                        "mfma_frac_flop_based": total_flops / t / (PEAK_TFLOPS["bf16"] * 1e12)}
    log(f"bf16 forward: {value:,.0f} maps/s ({t * 1e3:.3f} ms / {n} maps)")

    if not args.main_only or args.with_envmap:
        # ---------------- the step after the forward: sampling tables of the predicted maps
        legs["envmap_of_bf16_fwd_output"] = em = envmap_leg(B, y, args.steps, args.warmup)
        if tr and "envmap build" in tr["kernels"]:
            em["build_traffic_bytes"] = tr["kernels"]["envmap build"]["bytes_per_launch"]
        log(f"envmap build: {em['build_maps_per_s']:,.0f} maps/s ({em['build_ms']:.4f} ms, "
            f"{em['build_GB/s']:.0f} GB/s); sample {em['samples_per_s'] / 1e9:.2f} G/s; "
            f"pdf {em['pdf_evals_per_s'] / 1e9:.2f} G/s")
        legs["interp_weights_1080p"] = iw = interp_leg(B, dev, args.steps, args.warmup)
        log(f"interpolation weights, 1920x1080, r=16: {iw['ms']:.4f} ms ({iw['GB/s']:.0f} GB/s)")
    if not args.main_only:
        # ---------------- the same BF16 forward, one kernel per layer (activations through HBM)
        cae.set_fused(False)
        if not args.no_autotune and fused_headline:
            log("autotuning tile shapes of the layer kernels")
            B.drc_cae_autotune(cae.h, x, cae.workspace(n, H, H, B.DRC_WS_AUTOTUNE), tune_path)
        tl = timed(fwd, args.steps, args.warmup)
        legs["bf16_fwd_layer_by_layer"] = {"maps_per_s": n / tl, "ms": tl * 1e3,
                                           "mfma_frac_flop_based": total_flops / tl / (PEAK_TFLOPS["bf16"] * 1e12)}
        log(f"bf16 forward, layer by layer: {n / tl:,.0f} maps/s")
        cae.set_fused(True)
        # ---------------- FP32 and FP8 forward
        for comp in ("f32", "fp8"):
            c = CAE(comp, params, device=dev)
            if comp == "fp8":
                c.calibrate_fp8(x[:256])
            w = c.workspace(n, H, H, B.DRC_WS_FORWARD)
            tt = timed(lambda: B.drc_cae_forward(c.h, x, y, None, w), args.steps, args.warmup)
            legs[f"{comp}_fwd"] = {"maps_per_s": n / tt, "ms": tt * 1e3,
                                   "mfma_frac_flop_based": total_flops / tt / (PEAK_TFLOPS[comp] * 1e12)}
            if comp == "f32":
                y_f32 = y[:ACC_MAPS].cpu().numpy()
            if comp == "fp8":
                y_fp8 = y[:ACC_MAPS].cpu().numpy()
            log(f"{comp} forward: {n / tt:,.0f} maps/s")
            del c, w
        # ---------------- forward + backward (activations saved, no optimizer)
        for comp in ("bf16", "f32"):
            c = CAE(comp, params, device=dev)
            saved, _ = c.saved_buffer(n, H, H)
            dy = torch.randn((n, H, H, 3), device=dev) * 1e-6
            dp = torch.empty_like(params)
            wf = c.workspace(n, H, H, B.DRC_WS_FORWARD)
            wb = c.workspace(n, H, H, B.DRC_WS_BACKWARD)

            def fb():
                B.drc_cae_forward(c.h, x, y, saved, wf)
                B.drc_cae_backward(c.h, x, dy, saved, dp, None, wb)
            tt = timed(fb, max(3, args.steps // 2), 2)
            legs[f"{comp}_fwd_bwd"] = {"maps_per_s": n / tt, "ms": tt * 1e3}
            # one more pass with the timing hook on: where the backward time goes
            B.drc_cae_profile(c.h, 1)
            B.drc_cae_profile_read(c.h)
            fb()
            ms_s, calls_s = B.drc_cae_profile_read(c.h)
            B.drc_cae_profile(c.h, 0)
            names = [f"fwd {LAYERS[l][0]}" for l in range(6)] + [f"dgrad {LAYERS[l][0]}" for l in range(6)] + \
                    [f"wgrad {LAYERS[l][0]}" for l in range(6)] + ["gradient sums", "loss", "adam", "fused forward",
                                                                   "fused data gradients"]
            legs[f"{comp}_fwd_bwd"]["breakdown_ms"] = {names[k]: round(ms_s[k], 4) for k in range(23)
                                                       if calls_s[k]}
            log(f"{comp} forward+backward: {n / tt:,.0f} maps/s")
            del c, saved, dy, wf, wb
        # ---------------- training step (fwd + L1 + bwd + Adam + repack), recompute on
        nt = args.train_maps
        xt, tg = synth.training_batch(nt, H)
        xt, tg = torch.from_numpy(xt).to(dev), torch.from_numpy(tg).to(dev)
        for comp in ("bf16", "f32"):
            p = params.clone()
            tr = Trainer(CAE(comp, device=dev, recompute=True), p)
            tt = timed(lambda: tr.step(xt, tg), args.steps, args.warmup)
            legs[f"{comp}_train_step"] = {"maps_per_s": nt / tt, "ms": tt * 1e3, "batch": nt,
                                          "recompute": True}
            B.drc_cae_profile(tr.cae.h, 1)
            B.drc_cae_profile_read(tr.cae.h)
            tr.step(xt, tg)
            ms_s, calls_s = B.drc_cae_profile_read(tr.cae.h)
            B.drc_cae_profile(tr.cae.h, 0)
            names = [f"fwd {LAYERS[l][0]}" for l in range(6)] + [f"dgrad {LAYERS[l][0]}" for l in range(6)] + \
                    [f"wgrad {LAYERS[l][0]}" for l in range(6)] + ["gradient sums", "loss", "adam+repack",
                                                                   "fused forward / recompute",
                                                                   "fused data gradients"]
            legs[f"{comp}_train_step"]["breakdown_ms"] = {names[k]: round(ms_s[k], 4) for k in range(23)
                                                          if calls_s[k]}
            log(f"{comp} train step (batch {nt}): {nt / tt:,.0f} maps/s, {tt * 1e3:.3f} ms")
            # the same step recorded once as a HIP graph and replayed
            from paper_1910_02480_amd.cae import GraphTrainer
            gtr = GraphTrainer(CAE(comp, device=dev, recompute=True), params.clone())
            with torch.cuda.stream(torch.cuda.Stream(device=dev)):  # capture and replay on this stream
                tg_ = timed(lambda: gtr.step(xt, tg), args.steps, args.warmup)
            gtr.close()
            legs[f"{comp}_train_step"]["graph_ms"] = tg_ * 1e3
            legs[f"{comp}_train_step"]["graph_maps_per_s"] = nt / tg_
            log(f"{comp} train step as a replayed graph: {tg_ * 1e3:.3f} ms")
            if comp == "bf16":
                # augmentation of the step's batch (rotations and mirrors), before the step
                gen = torch.Generator(device=dev)
                gen.manual_seed(9)
                roll = torch.randint(0, H, (nt,), generator=gen, device=dev, dtype=torch.int32)
                flip = torch.randint(0, 2, (nt,), generator=gen, device=dev, dtype=torch.int32)
                xa, ta = torch.empty_like(xt), torch.empty_like(tg)
                tau = event_timed(lambda: B.drc_augment(xt, tg, roll, flip, xa, ta), args.steps, args.warmup)
                ab = 2 * nt * H * H * (7 + 3) * 4
                legs["bf16_augment"] = {"batch": nt, "ms": tau * 1e3, "GB/s": ab / tau / 1e9,
                                        "hbm_frac": ab / tau / 1e9 / PEAK_HBM_GBS, "alg_bytes": ab,
                                        "share_of_step": tau / tt}
                log(f"augmentation of the batch: {tau * 1e3:.4f} ms ({ab / tau / 1e9:.0f} GB/s)")
        # ---------------- the paper's own network (inference), 4096 maps of 32x32
        legs["unet_bf16_fwd_4096x32x32"] = un = unet_leg(B, dev, max(3, args.steps // 4), 2)
        log(f"paper's U-Net forward, 4096 maps of 32x32: {un['maps_per_s']:,.0f} maps/s "
            f"({un['ms']:.3f} ms, {un['TFLOP/s']:.0f} TFLOP/s)")
        legs["unet_f32_train_step_32x32x32"] = ut = unet_train_leg(B, dev, max(3, args.steps // 4), 2)
        log(f"paper's U-Net training step, 32 maps of 32x32 (FP32): {ut['ms']:.3f} ms "
            f"({ut['TFLOP/s']:.1f} TFLOP/s)")
        # ---------------- mixed-resolution frame: one graph replay per frame
        legs["bf16_mixed_frame"] = mixed_frame_leg(cae, tune_path, args)
        legs["speedup_bf16_vs_f32"] = {
            "fwd": legs["bf16_fwd"]["maps_per_s"] / legs["f32_fwd"]["maps_per_s"],
            "fwd_bwd": legs["bf16_fwd_bwd"]["maps_per_s"] / legs["f32_fwd_bwd"]["maps_per_s"],
            "train_step": legs["bf16_train_step"]["maps_per_s"] / legs["f32_train_step"]["maps_per_s"]}

    out = {"metric": METRIC, "value": value, "unit": "maps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": t * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
           "config": {"workload": f"cae_forward_{n}x{H}x{H}", "maps": n, "H": H, "W": H,
                      "in_ch": 7, "out_ch": 3, "widths": [32, 64, 128], "parallelism": "single-gpu"},
           "roofline": roof, "kernels": kernels, "legs": legs}

    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host")
        cb = cpu_baseline(lambda k: x_host[:k].numpy(), H, args.cpu_seconds, n, args.train_maps)
        out["cpu_baseline"] = cb
        outs = {"bf16": y_bf16}
        if not args.main_only:
            outs.update({"f32": y_f32, "fp8": y_fp8})
        acc = accuracy(outs, x_host, synth.init_params(0), ACC_MAPS)
        out["accuracy_vs_fp64_oracle"] = acc
        log(f"oracle: {cb['value']:.2f} maps/s on {cb['cores']} threads; accuracy "
            + ", ".join(f"{k} max_rel {v['max_rel_max']:.2e} mean_rel {v['mean_rel_mean']:.2e}"
                        for k, v in acc.items() if isinstance(v, dict)))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

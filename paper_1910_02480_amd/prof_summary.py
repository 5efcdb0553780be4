"""Short text summaries of rocprofv3 output for the library's kernels.

    python -m paper_1910_02480_amd.prof_summary stats <run_kernel_stats.csv> --cmd "..." --out X.md
    python -m paper_1910_02480_amd.prof_summary traffic <fetch counter csv> <write counter csv> \
        --cmd "..." --out X.md
    python -m paper_1910_02480_amd.prof_summary counters <pass1 csv> <pass2 csv> --agent <agent csv> \
        --cmd "..." --cmd "..." --out X.md
    python -m paper_1910_02480_amd.prof_summary timeline <run_kernel_trace.csv> --labels a,b --last 50 \
        --cmd "..." --out X.md

`stats` turns a `--kernel-trace --stats` kernel table into a markdown table
with the layer each kernel instantiation serves. `traffic` turns two `--pmc`
runs (FETCH_SIZE, then WRITE_SIZE; both in KiB per dispatch) into HBM bytes
per launch, scaled by what the same counters read for a plain elementwise
copy of known size run in the same process (torch.mul over 256 MiB): the
scale factors are (true bytes) / (counted bytes) of that copy. The traffic
file carries a hash of the kernel sources it was measured with, so that a
reader can tell when the kernels have changed since.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 256 << 20  # one read and one write stream of this size

# (regex on the demangled name, label); first match wins. A first group,
# when present, is the precision template argument (0 FP32, 1 BF16, 2 FP8).
# Some layer-kernel instantiations serve two layers (same channel counts).
_LABELS = (
    (r"conv_layer_kernel<(\d), \d+, 8, 8, 32,", "forward E1"),
    (r"conv_layer_kernel<(\d), \d+, 32, 32, 64,", "forward E2"),
    (r"conv_layer_kernel<(\d), \d+, 64, 64, 128,", "forward E3 / data gradient D3"),
    (r"conv_layer_kernel<(\d), \d+, 32, 32, 128,", "data gradient D2"),
    (r"conv_layer_kernel<(\d), \d+, 4, 4, 64,", "data gradient D1"),
    (r"tconv_pairs_kernel<(\d), 128, 128, 64,", "forward D3 / data gradient E3"),
    (r"tconv_pairs_kernel<(\d), 128, 64, 32,", "forward D2"),
    (r"tconv_pairs_kernel<(\d), 64, 64, 32,", "data gradient E2"),
    (r"tconv_merged_kernel<(\d), 64, 32, 3,", "forward D1"),
    (r"cae_fused_forward_kernel<\d+, \d+, false, false>", "forward fused"),
    (r"cae_fused_forward_kernel<\d+, \d+, false, true>", "forward fused (augmented input)"),
    (r"cae_fused_fp8_kernel", "FP8 forward fused"),
    (r"cae_fused_forward_kernel<\d+, \d+, true, false>", "recompute fused"),
    (r"pack_weights_kernel|pack_all_kernel", "weight pack"),
    (r"envmap_build_kernel", "envmap build"),
    (r"envmap_sample_kernel", "envmap sample"),
    (r"envmap_pdf_kernel", "envmap pdf"),
    (r"interp_weights_kernel", "interp weights"),
    (r"augment_kernel", "augmentation"),
    (r"unet_conv_kernel<\d+, \d+, 9>", "U-Net 3x3 convolution"),
    (r"unet_conv_lds_kernel<\d+>", "U-Net 3x3 convolution (LDS-tiled)"),
    (r"e1_band_kernel<(\d)>", "forward E1 (band-staged)"),
    (r"d1_band_kernel<(\d)>", "forward D1 (band-staged)"),
    (r"unet_conv_kernel<\d+, \d+, 1>", "U-Net 1x1 output convolution"),
    (r"unet_upcat_kernel", "U-Net upsample + concat"),
    (r"unet_pool_kernel", "U-Net max-pool"),
    (r"unet_cast_kernel", "U-Net input cast"),
    (r"unet_pack_kernel", "U-Net weight pack"),
    (r"ut_conv_kernel", "U-Net training convolution (FP32)"),
    (r"ut_reduce_kernel|ut_finish_kernel", "U-Net training batch-norm reductions"),
    (r"ut_bn_act_kernel|ut_bn_bwd_kernel", "U-Net training batch norm + LeakyReLU"),
    (r"ut_pool", "U-Net training max-pool"),
    (r"ut_upcat", "U-Net training upsample + concat"),
    (r"ut_out", "U-Net training output layer"),
    (r"ut_flip_kernel|ut_pad_|ut_fill_kernel", "U-Net training copies"),
    (r"cae_fused_tail_kernel", "128x128 E1-D2 fused (banded)"),
    (r"(?<!w)grad_final_kernel", "gradient sums (weights, biases, loss)"),
    (r"cae_fused_dgrad_kernel", "fused data gradients"),
    (r"wgrad_tr_kernel", "weight gradient (BF16, transpose reads)"),
    (r"wgrad_bf16_kernel", "weight gradient (BF16)"),
    (r"wgrad_kernel", "weight gradient (FP32)"),
    (r"wgrad_final_kernel", "weight-gradient reduction"),
    (r"bias_final_kernel|colsum_", "bias gradients"),
    (r"adam_kernel", "Adam"),
    (r"l1_", "L1 loss"),
    (r"elementwise.*Mul|Mul.*elementwise", "copy (torch.mul, 256 MiB)"),
)
_PREC = {"0": "FP32", "1": "BF16", "2": "FP8"}


def label(name: str) -> str | None:
    for pat, lab in _LABELS:
        m = re.search(pat, name)
        if m:
            return f"{_PREC.get(m.group(1), '?')} {lab}" if m.groups() else lab
    return None


# The HIP sources each labelled kernel is built from: a change to any of
# them makes that kernel's stored counters stale. Other labels depend on
# every source.
_KERNEL_SOURCES = {
    "forward fused": ("fused_fwd.hip", "common.h", "conv_layer.h", "internal.h"),
    "FP8 forward fused": ("fused_fp8.hip", "common.h", "conv_layer.h", "internal.h"),
    "envmap build": ("envmap.hip", "internal.h"),
    "envmap sample": ("envmap.hip", "internal.h"),
    "envmap pdf": ("envmap.hip", "internal.h"),
    "interp weights": ("interp.hip", "internal.h"),
}


def source_hash(lab: str | None = None) -> str:
    """Hash of the HIP sources and the public header a kernel (label) or the
    whole library (None) is built from."""
    h = hashlib.sha256()
    csrc = os.path.join(_HERE, "csrc")
    names = _KERNEL_SOURCES.get(lab) if lab else None
    if names is None:
        names = [f for f in sorted(os.listdir(csrc)) if f.endswith((".hip", ".h"))]
    files = [os.path.join(csrc, f) for f in sorted(names)]
    files.append(os.path.join(_HERE, "..", "include", "drc_cae.h"))
    for p in files:
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _short(name: str, n: int = 90) -> str:
    name = name.replace("(anonymous namespace)::", "")
    return name if len(name) <= n else name[: n - 3] + "..."


def stats(csv_path: str, cmd: str, title: str, top: int = 16) -> str:
    rows = list(csv.DictReader(open(csv_path)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows) or 1.0
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = [f"# {title}", "", "Command (run from /tmp with TMPDIR=/tmp; $R = repository root):", "",
           f"    {cmd}", "", f"Source hash of the kernels: `{source_hash()}`", "",
           "| Kernel | Serves | Calls | Avg (us) | Total (ms) | Share |", "|---|---|--:|--:|--:|--:|"]
    for r in rows[:top]:
        lab = label(r["Name"]) or ""
        out.append(f"| `{_short(r['Name'])}` | {lab} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['TotalDurationNs']) / 1e6:.3f} | {100 * float(r['TotalDurationNs']) / tot:.1f} % |")
    return "\n".join(out) + "\n"


def _per_dispatch(csv_path: str, counter: str):
    """Mean counter value per dispatch of every labelled kernel instantiation."""
    acc = collections.defaultdict(list)
    for r in csv.DictReader(open(csv_path)):
        if r["Counter_Name"] != counter:
            continue
        lab = label(r["Kernel_Name"])
        if lab:
            acc[(lab, r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return {k: (sum(v) / len(v), len(v)) for k, v in acc.items()}


def traffic(fetch_csv: str, write_csv: str, cmd_fetch: str, cmd_write: str, title: str) -> str:
    f = _per_dispatch(fetch_csv, "FETCH_SIZE")
    w = _per_dispatch(write_csv, "WRITE_SIZE")
    copy = "copy (torch.mul, 256 MiB)"
    fc = [v[0] for (lab, _), v in f.items() if lab == copy]
    wc = [v[0] for (lab, _), v in w.items() if lab == copy]
    if not fc or not wc:
        raise SystemExit("the copy kernel is missing from the counter files (run with --copy-calib)")
    kf = COPY_BYTES / (fc[0] * 1024.0)
    kw = COPY_BYTES / (wc[0] * 1024.0)
    rows = []
    kernels = {}
    for key in sorted(set(f) & set(w)):
        lab, name = key
        if lab == copy:
            continue
        fk, nf = f[key]
        wk, nw = w[key]
        d = {"name": name, "fetch_kib": fk, "write_kib": wk, "dispatches": min(nf, nw),
             "bytes_per_launch": fk * 1024.0 * kf + wk * 1024.0 * kw, "source_hash": source_hash(lab)}
        rows.append((lab, d))
        # a label's figure: its most dispatched instantiation (the one the timed loop runs)
        if lab not in kernels or d["dispatches"] > kernels[lab]["dispatches"]:
            kernels[lab] = d
    doc = {"source_hash": source_hash(), "fetch_scale": kf, "write_scale": kw,
           "copy_fetch_kib": fc[0], "copy_write_kib": wc[0], "kernels": kernels}
    out = [f"# {title}", "", "Commands (run from /tmp with TMPDIR=/tmp; $R = repository root):", "",
           f"    {cmd_fetch}", f"    {cmd_write}", "",
           f"Calibration: the 256 MiB elementwise copy reads {fc[0]:.0f} KiB (FETCH_SIZE) and writes "
           f"{wc[0]:.0f} KiB (WRITE_SIZE) per dispatch, so counted FETCH is scaled by {kf:.3f} and "
           f"WRITE by {kw:.3f}. Source hash of the kernels: `{doc['source_hash']}`.", "",
           "| Kernel | Serves | Dispatches | FETCH (KiB) | WRITE (KiB) | HBM bytes per launch (scaled) |",
           "|---|---|--:|--:|--:|--:|"]
    for lab, d in rows:
        out.append(f"| `{_short(d['name'])}` | {lab} | {d['dispatches']} | {d['fetch_kib']:.0f} | "
                   f"{d['write_kib']:.0f} | {d['bytes_per_launch'] / 1e6:.1f} MB |")
    out += ["", "Machine-readable copy (per layer: its most dispatched instantiation):", "", "```json",
            json.dumps(doc, indent=1), "```", ""]
    return "\n".join(out)


def _agent(info_csv: str):
    """(XCDs, SIMDs, CUs) of the GPU from rocprofv3's agent table."""
    for r in csv.DictReader(open(info_csv)):
        if r.get("Agent_Type") == "GPU":
            return int(r["Num_Xcc"]), int(r["Simd_Count"]), int(r["Cu_Count"])
    raise SystemExit(f"no GPU agent in {info_csv}")


def counters(csv_paths, info_csv: str, cmds, title: str) -> str:
    """SQ counters per dispatch of each labelled kernel (one or more --pmc
    passes), and the derived figures:
      mfma_busy   = sum over SIMDs of SQ_VALU_MFMA_BUSY_CYCLES / (cycles x SIMDs),
                    cycles = GRBM_GUI_ACTIVE / XCDs (the counter sums the XCDs);
      mfma_flops  = SQ_INSTS_VALU_MFMA_MOPS_BF16 x 512 (FLOPs the MFMAs executed,
                    padding lanes included);
      lds_conflict = SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE (share of the
                    LDS's active cycles stalled by bank conflicts)."""
    nx, simds, cus = _agent(info_csv)
    vals = collections.defaultdict(dict)
    names = {}
    for path in csv_paths:
        acc = collections.defaultdict(list)
        for r in csv.DictReader(open(path)):
            lab = label(r["Kernel_Name"])
            if lab:
                acc[(lab, r["Counter_Name"])].append(float(r["Counter_Value"]))
                names.setdefault(lab, collections.Counter())[r["Kernel_Name"]] += 1
        for (lab, c), v in acc.items():
            vals[lab][c] = sum(v) / len(v)
    kernels = {}
    for lab, v in vals.items():
        d = {"name": names[lab].most_common(1)[0][0], "counters": v, "source_hash": source_hash(lab)}
        for grbm in ("GRBM_GUI_ACTIVE",):
            if grbm in v:
                cyc = v[grbm] / nx
                d["cycles"] = cyc
                if "SQ_VALU_MFMA_BUSY_CYCLES" in v:
                    d["mfma_busy"] = v["SQ_VALU_MFMA_BUSY_CYCLES"] / (cyc * simds)
        if "SQ_INSTS_VALU_MFMA_MOPS_BF16" in v:
            d["mfma_flops"] = v["SQ_INSTS_VALU_MFMA_MOPS_BF16"] * 512.0
        if "SQ_LDS_IDX_ACTIVE" in v and "SQ_LDS_BANK_CONFLICT" in v and v["SQ_LDS_IDX_ACTIVE"] > 0:
            d["lds_conflict"] = v["SQ_LDS_BANK_CONFLICT"] / v["SQ_LDS_IDX_ACTIVE"]
        kernels[lab] = d
    doc = {"source_hash": source_hash(), "xcds": nx, "simds": simds, "cus": cus, "kernels": kernels}
    out = [f"# {title}", "", "Commands (run from /tmp with TMPDIR=/tmp; $R = repository root):", ""]
    out += [f"    {c}" for c in cmds]
    out += ["", f"GPU: {cus} CUs, {simds} SIMDs, {nx} XCDs. Values are per dispatch (mean over the dispatches "
                "of the kernel). mfma_busy = SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / XCDs x SIMDs); "
                "lds_conflict = SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE. "
                f"Source hash of the kernels: `{doc['source_hash']}`.", ""]
    allc = sorted({c for d in kernels.values() for c in d["counters"]})
    out.append("| Kernel | Serves | " + " | ".join(allc) + " | mfma_busy | lds_conflict |")
    out.append("|---|---|" + "--:|" * (len(allc) + 2))
    for lab, d in sorted(kernels.items()):
        cells = [f"{d['counters'][c]:.4g}" if c in d["counters"] else "" for c in allc]
        mb = f"{100 * d['mfma_busy']:.1f} %" if "mfma_busy" in d else ""
        lc = f"{100 * d['lds_conflict']:.1f} %" if "lds_conflict" in d else ""
        out.append(f"| `{_short(d['name'], 60)}` | {lab} | " + " | ".join(cells) + f" | {mb} | {lc} |")
    out += ["", "Machine-readable copy:", "", "```json", json.dumps(doc, indent=1), "```", ""]
    return "\n".join(out)


def read_counters(md_path: str):
    """The json block of a counter summary without its stale kernels (or None)."""
    return read_traffic(md_path)


def read_traffic(md_path: str):
    """The json block of a traffic summary without its stale kernels, or None
    when absent or when every kernel is stale."""
    try:
        text = open(md_path).read()
    except OSError:
        return None
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    if not m:
        return None
    doc = json.loads(m.group(1))
    # keep the kernels whose sources are unchanged since the counters were taken
    doc["kernels"] = {lab: d for lab, d in doc.get("kernels", {}).items()
                      if d.get("source_hash", doc.get("source_hash")) == source_hash(lab)}
    return doc if doc["kernels"] else None


def timeline(trace_csv: str, cmd: str, title: str, labels: list[str], last: int) -> str:
    """Launch timeline of a repeated pass (a frame replayed many times) from
    a `--kernel-trace` CSV: the last `last` dispatches of each kernel label
    are taken as the last `last` passes, one dispatch per label per pass;
    for each label the median start (relative to the pass's first start) and
    duration, and the median span of a pass."""
    ev = collections.defaultdict(list)
    names = {}
    with open(trace_csv, newline="") as fh:
        for r in csv.DictReader(fh):
            lab = label(r["Kernel_Name"])
            m = re.search(r"cae_fused_forward_kernel<(\d+), (\d+)", r["Kernel_Name"])
            if lab and m:  # the whole-network kernel of each map size
                lab = f"{lab} {m.group(1)}x{m.group(2)}"
            if lab in labels:
                ev[lab].append((int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
                names[lab] = r["Kernel_Name"]
    missing = [lab for lab in labels if len(ev[lab]) < last]
    if missing:
        raise SystemExit(f"timeline: fewer than {last} dispatches of {missing}")
    for lab in labels:
        ev[lab].sort()
    spans, start, dur = [], collections.defaultdict(list), collections.defaultdict(list)
    for i in range(1, last + 1):
        pas = {lab: ev[lab][-i] for lab in labels}
        t0 = min(v[0] for v in pas.values())
        spans.append((max(v[1] for v in pas.values()) - t0) / 1e3)
        for lab, (b, e) in pas.items():
            start[lab].append((b - t0) / 1e3)
            dur[lab].append((e - b) / 1e3)

    def med(v):
        v = sorted(v)
        return v[len(v) // 2] if len(v) % 2 else 0.5 * (v[len(v) // 2 - 1] + v[len(v) // 2])

    out = [f"# {title}", "", "Command (run from /tmp with TMPDIR=/tmp; $R = repository root):", "", f"    {cmd}", "",
           f"Source hash of the kernels: `{source_hash()}`", "",
           f"Last {last} passes; medians over them (us). Span of a pass: {med(spans):.1f} us "
           f"(min {min(spans):.1f}).", "", "| Kernel | Serves | Start | Duration | End |", "|---|---|--:|--:|--:|"]
    for lab in sorted(labels, key=lambda x: med(start[x])):
        out.append(f"| `{_short(names[lab])}` | {lab} | {med(start[lab]):.1f} | {med(dur[lab]):.1f} | "
                   f"{med(start[lab]) + med(dur[lab]):.1f} |")
    return "\n".join(out) + "\n"


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd_name", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--cmd", required=True)
    s.add_argument("--title", default="Kernel trace")
    s.add_argument("--top", type=int, default=16)
    s.add_argument("--out", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("fetch_csv")
    t.add_argument("write_csv")
    t.add_argument("--cmd-fetch", required=True)
    t.add_argument("--cmd-write", required=True)
    t.add_argument("--title", default="HBM traffic")
    t.add_argument("--out", required=True)
    c = sub.add_parser("counters")
    c.add_argument("csv", nargs="+", help="counter_collection.csv of each --pmc pass")
    c.add_argument("--agent", required=True, help="agent_info.csv of one of the passes")
    c.add_argument("--cmd", action="append", required=True, help="the command of each pass")
    c.add_argument("--title", default="SQ counters")
    c.add_argument("--out", required=True)
    tl = sub.add_parser("timeline")
    tl.add_argument("csv", help="run_kernel_trace.csv of a --kernel-trace run")
    tl.add_argument("--labels", required=True, help="comma-separated kernel labels of one pass")
    tl.add_argument("--last", type=int, default=50)
    tl.add_argument("--cmd", required=True)
    tl.add_argument("--title", default="Launch timeline")
    tl.add_argument("--out", required=True)
    a = ap.parse_args()
    if a.cmd_name == "timeline":
        text = timeline(a.csv, a.cmd, a.title, a.labels.split(","), a.last)
    elif a.cmd_name == "stats":
        text = stats(a.csv, a.cmd, a.title, a.top)
    elif a.cmd_name == "counters":
        text = counters(a.csv, a.agent, a.cmd, a.title)
    else:
        text = traffic(a.fetch_csv, a.write_csv, a.cmd_fetch, a.cmd_write, a.title)
    with open(a.out, "w") as fh:
        fh.write(text)
    print(text)


if __name__ == "__main__":
    main()

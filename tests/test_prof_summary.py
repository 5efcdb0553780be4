"""Host logic of the profile summaries: stored counters are used only for
kernels whose sources are unchanged since the counters were taken."""
import json

from paper_1910_02480_amd import prof_summary as P


def _doc(kernels, path):
    text = "# t\n\n```json\n" + json.dumps({"source_hash": "x", "kernels": kernels}) + "\n```\n"
    path.write_text(text)
    return str(path)


def test_fresh_kernels_kept_stale_dropped(tmp_path):
    k = {"forward fused": {"bytes_per_launch": 1.0, "source_hash": P.source_hash("forward fused")},
         "envmap build": {"bytes_per_launch": 2.0, "source_hash": "0000000000000000"}}
    d = P.read_traffic(_doc(k, tmp_path / "a.md"))
    assert list(d["kernels"]) == ["forward fused"]


def test_all_stale_or_missing_gives_none(tmp_path):
    k = {"forward fused": {"bytes_per_launch": 1.0, "source_hash": "0000000000000000"}}
    assert P.read_traffic(_doc(k, tmp_path / "b.md")) is None
    assert P.read_traffic(str(tmp_path / "missing.md")) is None


def test_per_kernel_hash_covers_only_its_sources():
    # the fused forward's hash is not the library's, and each is stable
    assert P.source_hash("forward fused") != P.source_hash()
    assert P.source_hash("forward fused") == P.source_hash("forward fused")
    assert P.source_hash("some layer kernel") == P.source_hash()


def test_committed_traffic_summary_parses():
    import os
    path = os.path.join(os.path.dirname(__file__), "..", "profiles", "cae_forward_bf16_4096x64x64_traffic.md")
    text = open(path).read()
    assert "```json" in text and "FETCH_SIZE" in text

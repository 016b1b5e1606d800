"""Host-side logic of bench.py (no GPU): the byte model behind every roofline
entry, the lookup of counter summaries in profiles/, and the refusal of more
than one GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_algorithmic_bytes_of_a_pass():
    # 2D 512^2 x 64 complex64: the 3-component field read and written once
    assert bench.algorithmic_bytes("xpass", (2, (512, 512), 64), 8) == 2 * 3 * 8 * 512 * 512 * 64 == 805306368
    assert bench.algorithmic_bytes("zpass", (3, (256, 256, 256), 8), 8) == 6442450944
    assert bench.algorithmic_bytes("spectrum", (2, (512, 512), 64), 8) is None
    assert bench.pass_bytes([(2, (512, 512), 0.5, 64)], "c64") == 805306368
    assert bench.pass_bytes([(1, (4096,), 0.5, 250)], "c128") == 2 * 3 * 16 * 4096 * 250
    groups = [(1, (4096,), 0.5, 128), (2, (256, 256), 0.5, 32), (2, (512, 512), 0.5, 16), (2, (1024, 1024), 0.5, 4)]
    assert bench.pass_bytes(groups, "c64") == 48 * 11010048


def test_whole_step_entry_counts_one_pass_per_axis():
    # 1e10 site-steps/s of a 2D grid move 96 B per site-step: 960 GB/s
    e = bench.whole_step_entry(1e10, [(2, (512, 512), 0.5, 64)], "c64")
    assert e["bytes_per_site_step"] == 96.0
    assert e["achieved"] == pytest.approx(960.0)
    assert e["frac"] == pytest.approx(960.0 / bench.HBM_PEAK_GBPS)
    e3 = bench.whole_step_entry(1e10, [(3, (256, 256, 256), 0.5, 8)], "c128")
    assert e3["bytes_per_site_step"] == 288.0


def test_variant_lookup_keys():
    tuned = {"gfx950/c64/0/512": 1, "gfx950/c64/1/512": 2, "gfx950/c64/1/256": 0}
    assert bench.variant_of("xpass", [(2, (512, 512), 0.5, 64)], tuned) == 1
    assert bench.variant_of("ypass", [(2, (512, 512), 0.5, 64)], tuned) == 2
    assert bench.variant_of("zpass", [(3, (256, 256, 256), 0.5, 8)], tuned) == 0
    assert bench.variant_of("zpass", [(2, (512, 512), 0.5, 64)], tuned) is None
    assert bench.variant_of("xpass", [(2, (512, 512), 0.5, 64)], None) is None


def test_committed_summaries_parse():
    """Every traffic and VALU summary in profiles/ carries one machine-readable
    line per pass kind and variant, with a source hash of the form bench.py
    compares against."""
    for workload, name in bench.TRAFFIC_FILES.items():
        rec = bench.summary_lines(os.path.join(ROOT, "profiles", name), "traffic")
        kinds = {k for k, _ in rec}
        assert {"xpass", "ypass"} <= kinds, (workload, rec)
        if workload.startswith("3d"):
            assert "zpass" in kinds
        for (kind, variant), r in rec.items():
            assert variant in (0, 1, 2)
            assert r["workload"] == workload
            assert len(r["source"]) == 16
            assert float(r["bytes"]) > 0
    rec = bench.summary_lines(os.path.join(ROOT, "profiles", "valu_xpass_ypass_2d512_s64.md"), "valu")
    assert {k for k, _ in rec} == {"xpass", "ypass"}
    assert all(float(r["instr"]) > 0 for r in rec.values())


def test_traffic_lookup_follows_variant_and_source_hash(tmp_path, monkeypatch):
    current = bench.kernel_source_hash()
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "t.md").write_text(
        "traffic: kind=xpass variant=1 workload=w bytes=123 source=%s\n"
        "traffic: kind=xpass variant=0 workload=w bytes=456 source=0000000000000000\n" % current)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: current)
    monkeypatch.setitem(bench.TRAFFIC_FILES, "w", "t.md")
    assert bench.measured_traffic("xpass", "w", 1) == 123.0
    assert bench.measured_traffic("xpass", "w", 0) is None  # counted on other kernel sources
    assert bench.measured_traffic("ypass", "w", 1) is None  # no such line
    assert bench.measured_traffic("xpass", "other", 1) is None  # no such summary


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr

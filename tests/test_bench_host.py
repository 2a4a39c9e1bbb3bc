"""Host-side logic of bench.py: the one-GPU refusal, the algorithmic byte
counts it divides by, and the rule that ties a committed counter summary to
the kernel source it measured."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_splat_bytes_are_the_stage_sums():
    # per active Gaussian and view: projection reads 236 B and writes 52,
    # scan 24, screen-space gradient 40, projection backward reads 236 + 40
    # and writes 236
    assert bench.SPLAT_BYTES["per_gaussian"] == 236 + 52 + 24 + 40 + (236 + 40) + 236
    # per pair: emission 12, sort read + write 24, ranges 8, forward and
    # backward record gathers 40 each
    assert bench.SPLAT_BYTES["per_pair"] == 12 + 24 + 8 + 40 + 40
    # per pixel: forward output 24, backward input 36
    assert bench.SPLAT_BYTES["per_pixel"] == 24 + 36
    R = 59  # SH degree 3: 11 geometry rows + 48 colour rows
    assert bench.stage_bytes("adam", 1, 0, 0, R) == 1664
    assert bench.stage_bytes("compact", 1, 0, 0, R) == 476
    assert bench.stage_bytes("tile_sort", 0, 1, 0, R) == 32
    assert bench.stage_bytes("raster_bwd", 1, 1, 1, R) == 0.0  # a VALU-bound stage


def test_counter_summary_is_used_only_for_its_kernel_and_source(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("kernel source v1\n")
    (tmp_path / "profiles").mkdir()
    t = {"bytes_per_launch": 1.5e9, "source": "k.hip", "kernel_regex": "k_raster_bwd<16, 16, 4>",
         "source_sha256": bench.source_digest(str(src))}
    (tmp_path / "profiles" / "traffic_raster_bwd_w.json").write_text(json.dumps(t))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("w", "raster_bwd", "k_raster_bwd<16, 16, 4>") == 1.5e9
    assert bench.measured_traffic("w", "raster_bwd", "k_raster_bwd<8, 8, 1>") is None
    assert bench.measured_traffic("other", "raster_bwd") is None
    src.write_text("kernel source v2\n")  # the kernel changed since the counters
    assert bench.measured_traffic("w", "raster_bwd", "k_raster_bwd<16, 16, 4>") is None


def test_committed_counter_summaries_name_their_command_and_source():
    for name in os.listdir(os.path.join(ROOT, "profiles")):
        if name.startswith("traffic_") and name.endswith(".json"):
            with open(os.path.join(ROOT, "profiles", name)) as f:
                t = json.load(f)
            assert t["command"].startswith("rocprofv3 --pmc FETCH_SIZE"), name
            assert os.path.exists(os.path.join(ROOT, t["source"])), name
            assert t["bytes_per_launch"] == (t["FETCH_SIZE"]["bytes_per_launch"]
                                             + t["WRITE_SIZE"]["bytes_per_launch"]), name

"""Host logic of bench.py (no GPU): the single-GPU guard, the kernel source
hash that decides whether the committed counter summary still describes the
sweep kernel (its source and the headers it includes), and the traffic
figures taken from that summary only on a match."""
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

SOURCES = ("paper_1607_02214_amd/csrc/ppmlr_sweep.hpp", "paper_1607_02214_amd/csrc/ppmlr_mlp.hpp",
           "paper_1607_02214_amd/csrc/ppmlr_char.hpp")


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 3
    assert "exactly one GPU" in r.stderr
    assert r.stdout.strip() == ""                     # no bench line


@pytest.fixture
def source_copy(tmp_path, monkeypatch):
    for rel in SOURCES:
        dst = tmp_path / rel
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(ROOT, rel), dst)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    return tmp_path


def test_source_hash_ignores_comments_and_whitespace_but_not_code(source_copy):
    h0 = bench.kernel_source_hash()
    p = source_copy / SOURCES[0]
    src = p.read_text()
    p.write_text("// a new comment line\n/* and a block\n   comment */\n" + src.replace("\n", "\n\n", 3))
    assert bench.kernel_source_hash() == h0
    p.write_text(src.replace("constexpr int kCflSlots = 64;", "constexpr int kCflSlots = 32;"))
    assert "kCflSlots = 32" in p.read_text()
    assert bench.kernel_source_hash() != h0


def test_traffic_summary_used_only_for_the_source_it_was_taken_from(source_copy, tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "PROFILES", str(prof))
    assert bench.load_traffic("f32") == (None, None)           # no summary
    h = bench.kernel_source_hash()
    rec = {"source_hash": h, "bytes_per_launch": {"2": 1.0}}
    (prof / "traffic_sweep_inflow_dipole_f32.json").write_text(json.dumps(rec))
    d, hh = bench.load_traffic("f32")
    assert hh == h and d["bytes_per_launch"] == {"2": 1.0}
    rec["source_hash"] = "0" * 16                                # taken from other sources
    (prof / "traffic_sweep_inflow_dipole_f32.json").write_text(json.dumps(rec))
    assert bench.load_traffic("f32") == (None, "0" * 16)


def test_counter_record_matches_the_launched_tile_shape():
    prof = {"tiles": [5, 8, 8], "segments": [3, 4, 4], "segment_order": [1, 1, 2], "bytes_per_launch": {"2": 1.0},
            "alternates": [{"tiles": [5, 4, 4], "segments": [3, 4, 4], "segment_order": [1, 2, 2],
                            "bytes_per_launch": {"2": 2.0}}]}
    assert bench.shape_record(prof, 2, (8, 4, 2))["bytes_per_launch"]["2"] == 1.0
    assert bench.shape_record(prof, 2, (4, 4, 2))["bytes_per_launch"]["2"] == 2.0
    assert bench.shape_record(prof, 2, (4, 4, 1)) is None          # other tile order
    assert bench.shape_record(prof, 1, (8, 4, 2)) is None          # y was taken with order 1 or 2, not this
    assert bench.shape_record(None, 2, (8, 4, 2)) is None

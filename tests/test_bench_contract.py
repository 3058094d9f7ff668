"""bench.py's output contract, on the CPU: the multi-GPU refusal, the
roofline fields, and the traffic lookup keyed by launch shape and kernel
sources."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def _fake_run(ms=1.25, launch=(32, 8, 16)):
    return dict(nodes=512 * 256 * 128, ms=ms,
                launch=dict(bx=launch[0], by=launch[1], bz=launch[2], persistent=0))


def test_roofline_fields_and_arithmetic(monkeypatch):
    import bench
    monkeypatch.setattr(bench, "measured_traffic", lambda p, l, b=None: None)
    r = bench.roofline("fp32", _fake_run())
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in r
    n = 512 * 256 * 128
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["achieved"] == pytest.approx(352 * n / 1.25e-3 / 1e9, rel=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0, rel=1e-3)
    assert r["traffic"] is None and r["bytes_min_per_node"] == 416
    r16 = bench.roofline("fp16s", _fake_run())
    assert r16["bytes_alg_per_node"] == 200 and r16["bytes_min_per_node"] == 264


def test_traffic_lookup_needs_matching_sources(tmp_path, monkeypatch):
    import bench
    from paper_1411_2181_amd.build import source_hash
    entry = {"k_step": {"bytes": 2, "bytes_per_node": 500.0}}
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    for h, want in (("0" * 16, None), (source_hash(), entry)):
        (prof / "traffic_mv512.json").write_text(json.dumps(
            {"fp32": {"source_hash": h, "launches": {"32x8x16": entry}}}))
        assert bench.measured_traffic("fp32", _fake_run()["launch"]) == want
    # a shape that was not measured, a precision that was not, another lattice
    assert bench.measured_traffic("fp32", dict(bx=64, by=4, bz=8, persistent=0)) is None
    assert bench.measured_traffic("fp16s", _fake_run()["launch"]) is None
    assert bench.measured_traffic("fp32", _fake_run()["launch"], (64, 256, 128)) is None
    r = bench.roofline("fp32", _fake_run())
    assert r["traffic"] == 2 and r["traffic_per_node"] == 500.0

"""CPU: the host logic of bench.py's roofline line -- which kernel family it reports, how the achieved rate and
the bound follow from the per-family totals, and that a measured-traffic record is used only while the sources
it names are unchanged."""

import hashlib
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def fam(ms, launches, byts, flops):
    return {"ms": ms, "launches": launches, "bytes": byts, "flops": flops}


def test_roofline_takes_the_family_with_most_time_and_its_bound():
    # gram: 2 launches of 6.45e9 flops and 3.2e8 bytes (20 flop/byte, above the FP64 ridge of 78.6/8 ~ 9.8)
    stats = {"gram": fam(0.3, 2, 6.4e8, 1.29e10), "block_update": fam(0.2, 2, 9.6e8, 1.29e10),
             "spmm": fam(0.1, 5, 5e8, 1e8), "small_dense": fam(0.5, 9, 0.0, 0.0)}
    r = bench.roofline(stats, steps=1)
    assert r["kernel"] == "gram"  # the one-workgroup family has no algorithmic work and is passed over
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s" and r["peak"] == 78.6
    assert r["achieved"] == pytest.approx(1.29e10 / 2 / (0.15e-3) / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / 78.6)
    assert r["avg_launch_ms"] == pytest.approx(0.15) and r["launches_per_step"] == 2


def test_roofline_below_the_ridge_is_hbm_bound():
    stats = {"schur_epi": fam(0.4, 4, 4e9, 1e9)}  # 0.25 flop/byte
    r = bench.roofline(stats, steps=2)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == bench.HBM_PEAK_GBS
    assert r["achieved"] == pytest.approx(1e9 / 0.1e-3 / 1e9)
    assert r["launches_per_step"] == 2


def test_roofline_of_the_band_cholesky_sums_both_families():
    stats = {"chol_update": fam(3.0, 50, 1e8, 6e10), "chol_panel": fam(1.0, 50, 1e7, 2e10)}
    r = bench.roofline(stats, steps=1)
    assert r["kernel"] == "chol_update+chol_panel" and r["bound"] == "mfma"
    assert r["achieved"] == pytest.approx(8e10 / 4e-3 / 1e12)


def test_measured_traffic_only_while_its_sources_are_unchanged(tmp_path, monkeypatch):
    src = tmp_path / "kernel.hip"
    src.write_text("// kernel source\n")
    rec = {"kernel": "gram", "workload": "w", "traffic_bytes_per_launch": 1.5e8,
           "sources": {"kernel.hip": hashlib.sha256(src.read_bytes()).hexdigest()}}
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic_gram_w.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "profiles" / "traffic_{}_{}.json"))
    monkeypatch.setattr(bench.os.path, "abspath", lambda p: str(tmp_path / "bench.py") if p == bench.__file__
                        else os.path.realpath(p))
    assert bench.measured_traffic("gram", "w") == 1.5e8
    assert bench.measured_traffic("gram", "other") is None  # no record for this workload
    src.write_text("// kernel source, changed\n")
    assert bench.measured_traffic("gram", "w") is None


def test_committed_traffic_records_name_existing_sources():
    prof = os.path.join(ROOT, "profiles")
    names = [n for n in os.listdir(prof) if n.startswith("traffic_") and n.endswith(".json")]
    assert names
    for n in names:
        with open(os.path.join(prof, n)) as f:
            rec = json.load(f)
        assert rec["traffic_bytes_per_launch"] > 0
        assert rec["sources"], n
        for rel in rec["sources"]:
            assert os.path.exists(os.path.join(ROOT, rel)), (n, rel)

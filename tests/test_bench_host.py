"""Host-side checks of bench.py's reporting (no GPU): the roofline arithmetic
and the one-GPU contract."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _stats():
    # a build of 1,000 tile pairs with 2e6 candidate pairs and 16 Stage IV pivots
    return {
        "ms_vgrng": 2.0, "vgrng_ops": 2.0 * 100_000 * 1000 * 256,
        "ms_pairs": 10.0, "candidate_pairs": 2e6, "stage4_pivots": 16,
        "pair_method_distances": 2e6 + 1000 * 128 * 16 + 600 * 4096,
        "pair_tile_entries": 1000 * (4096 + 128 * 16) + 600 * 4096,
        "ms_lune": 5.0, "lune_tests": 1e9,
        "ms_pair_masks": 1.0, "tile_pairs": 1000,
        "ms_partner": 0.5, "partner_tests": 1e8, "partner_kills": 5e5,
    }


def test_roofline_fractions_follow_from_the_counts():
    st = _stats()
    d = 16
    ks = bench.kernel_rooflines(st, d, 1)
    v = ks["k_vgrng_tiles"]
    assert v["bound"] == "alu" and v["achieved"] == pytest.approx(2 * st["vgrng_ops"] / 2e-3 / 1e12)
    p = ks["k_pairs_tiled"]
    # float64 tiles: 2 d flops per method distance against the FP64 MFMA peak
    flops = st["pair_method_distances"] * 2 * d
    valu = 2 * st["candidate_pairs"] * 16
    assert flops / 78.6e12 > valu / 39.3216e12
    assert p["bound"] == "mfma" and p["unit"] == "TFLOP/s" and p["peak"] == 78.6
    assert p["achieved"] == pytest.approx(flops / 1e-2 / 1e12)
    assert p["valu"]["achieved"] == pytest.approx(valu / 1e-2 / 1e12)
    assert p["dense_tile_tflop_s"] == pytest.approx(st["pair_tile_entries"] * 2 * 16 / 1e-2 / 1e12)
    lu = ks["k_lune_guided"]
    assert lu["bound"] == "alu" and lu["achieved"] == pytest.approx(1e9 * 4 * d / 5e-3 / 1e12)
    pw = ks["k_partner_witness"]   # one squared distance (3 d flops) per partner test
    assert pw["bound"] == "alu" and pw["achieved"] == pytest.approx(1e8 * 3 * d / 0.5e-3 / 1e12)
    assert pw["kills"] == 5e5
    mk = ks["k_pair_masks"]
    assert mk["achieved"] == pytest.approx(1120 * 1000 / 1e-3 / 1e9)
    for r in ks.values():
        assert r["frac"] == pytest.approx(r["achieved"] / r["peak"])
    # the line's roofline object is the longest kernel's entry
    r = bench.roofline(st, d, 1, "none")
    assert r["kernel"] == "k_pairs_tiled" and r["traffic"] is None


def test_bf16_tiles_leave_the_pair_kernel_bound_by_its_valu_work():
    st = _stats()
    p = bench.kernel_rooflines(st, 32, 2)["k_pairs_bf16"]
    assert p["bound"] == "alu" and p["unit"] == "Tops/s"
    assert p["achieved"] == pytest.approx(2 * st["candidate_pairs"] * 16 / 1e-2 / 1e12)
    # three split products per 32-wide K block against the bf16 peak
    assert p["mfma"]["peak"] == 2500.0
    assert p["mfma"]["dense_tile_tflop_s"] == pytest.approx(st["pair_tile_entries"] * 2 * 32 * 3 / 1e-2 / 1e12)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_traffic_record_applies_only_to_its_sources_and_workload(tmp_path, monkeypatch):
    rec = {"k_pairs_tiled": {"workload": "w", "source_sha256": "a" * 64, "fetch_bytes": 1.0, "write_bytes": 2.0}}
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_hash", lambda k: "a" * 64)
    assert bench.measured_traffic("k_pairs_tiled", "w") == pytest.approx(3.0)
    assert bench.measured_traffic("k_pairs_tiled", "other workload") is None
    assert bench.measured_traffic("k_lune_guided", "w") is None
    monkeypatch.setattr(bench, "source_hash", lambda k: "b" * 64)   # kernel changed since
    assert bench.measured_traffic("k_pairs_tiled", "w") is None

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
    # a build of 1,000 tile pairs, 600 of them reaching Stage V, dp = 16
    dp, tp, tpv, K = 16, 1000, 600, 16
    return {
        "ms_vgrng": 2.0, "vgrng_ops": 2.0 * 100_000 * 1000 * 256,
        "ms_pairs": 10.0, "pairs_flops": 2.0 * dp * ((64 * 64 + 2 * 64 * 16) * tp + 2 * 64 * 64 * tpv),
        "stage4_ops": 2.0 * 64 * 64 * K * tp,
        "ms_lune": 5.0, "lune_bytes": 1e9 * (4 * dp + 4),
        "ms_pair_masks": 1.0, "tile_pairs": tp,
    }


def test_roofline_fractions_follow_from_the_counts():
    st = _stats()
    ks = bench.kernel_rooflines(st)
    v = ks["k_vgrng_tiles"]
    assert v["bound"] == "alu" and v["achieved"] == pytest.approx(2 * st["vgrng_ops"] / 2e-3 / 1e12)
    p = ks["k_pairs_tiled"]
    assert p["bound"] == "mfma" and p["unit"] == "TFLOP/s" and p["peak"] == 78.6
    assert p["achieved"] == pytest.approx(st["pairs_flops"] / 1e-2 / 1e12)
    lu = ks["k_lune_guided"]
    assert lu["achieved"] == pytest.approx(st["lune_bytes"] / 5e-3 / 1e9)
    mk = ks["k_pair_masks"]
    assert mk["achieved"] == pytest.approx(1120 * 1000 / 1e-3 / 1e9)
    for r in ks.values():
        assert r["frac"] == pytest.approx(r["achieved"] / r["peak"])
    # the line's roofline object is the longest kernel's entry
    r = bench.roofline(st, "none")
    assert r["kernel"] == "k_pairs_tiled" and r["traffic"] is None


def test_stage4_bound_wins_when_its_time_at_peak_is_longer():
    st = _stats()
    st["stage4_ops"] = st["pairs_flops"] * 10.0
    p = bench.kernel_rooflines(st)["k_pairs_tiled"]
    assert p["bound"] == "alu" and p["unit"] == "Tops/s"


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

"""Host logic of bench.py (no GPU): the refusal of more than one GPU, the
roofline and sweep-level arithmetic, the matching of recorded counter
traffic, and the CPU baseline record."""
import json
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _variant(prec="fp32_r12", n_lat=4, or_us=45.0, ms=7.4):
    # a 32^4 batch: 32 overrelaxation phases per lattice and sweep, V/2 links each
    V = 32 ** 4
    or_launches = 32 * n_lat
    or_bytes = or_launches * (V // 2) * bench.PHASE_RECORDS * bench.LINK_BYTES[prec]
    return {"prec": prec, "n_lat": n_lat, "or_bytes_total": or_bytes, "or_launches": or_launches,
            "or_kernel_us": or_us, "streaming_or_kernel_us": 4 * or_us * 1.2,
            "bytes_per_step": 40 * n_lat * (V // 2) * bench.PHASE_RECORDS * bench.LINK_BYTES[prec],
            "ms_per_step": ms, "step_ms_median": ms * 1.01,
            "launch": {"block": 256, "xcd_remap": 1, "ty": 8, "tz": 8, "tt": 8}}


def test_roofline_is_algorithmic_bytes_over_the_launch_time():
    v = _variant()
    r = bench.roofline(v)
    per_launch = 524288 * 9 * 48  # 226.5 MB: V/2 links x 9 records x 48 B
    assert r["algorithmic_bytes_per_launch"] == per_launch
    assert r["achieved"] == pytest.approx(per_launch / 45e-6 / 1e9, rel=1e-4)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0, abs=1e-4)
    assert r["bound"] == "hbm" and r["peak"] == 8000.0 and r["unit"] == "GB/s"
    # the streaming figure covers the four lattices of one launch
    s = r["streaming"]
    assert s["algorithmic_bytes_per_launch"] == 4 * per_launch
    assert s["achieved"] == pytest.approx(4 * per_launch / (4 * 45e-6 * 1.2) / 1e9, rel=1e-4)
    # a single lattice has no grouping note and no streaming figure
    r1 = bench.roofline(_variant(n_lat=1))
    assert "streaming" not in r1 and "note" not in r1


def test_sweep_level_fraction():
    v = _variant()
    s = bench.sweep_level(v)
    assert s["algorithmic_bytes_per_step"] == 36238786560  # 40 phases x 226.5 MB x 4 lattices
    assert s["frac"] == pytest.approx(36238786560 / 7.4e-3 / 8e12, abs=1e-4)
    assert s["one_sweep_per_call"]["frac_at_median"] == pytest.approx(36238786560 / (7.4e-3 * 1.01) / 8e12,
                                                                       abs=1e-4)


def test_recorded_traffic_matches_only_its_own_workload():
    v = _variant()
    with open(os.path.join(ROOT, bench.TRAFFIC_SUMMARY)) as fh:
        recs = [json.loads(line.split(":", 1)[1]) for line in fh if line.startswith("traffic-record:")]
    assert recs, "the phase-kernel summary holds no traffic records"
    # every record states its scaling and source hash
    for rec in recs:
        assert rec["hbm_bytes_per_launch"] == pytest.approx(
            1024 * (rec["fetch_kib"] * rec["fetch_factor"] + rec["write_kib"] * rec["write_factor"]), rel=1e-3)
        assert len(rec["sources_sha256"]) == 64
    # a launch shape, precision or lattice count without a record gives None
    assert bench.recorded_traffic(dict(v, launch={"block": 64, "xcd_remap": 0, "ty": 2, "tz": 2, "tt": 2}), 32) is None
    assert bench.recorded_traffic(dict(v, prec="fp64"), 32) is None
    assert bench.recorded_traffic(dict(v, n_lat=3), 32) is None
    assert bench.recorded_traffic(v, 24) is None


def test_cpu_baseline_record():
    c = bench.cpu_baseline([4, 4, 4, 4], 1, n_sweeps=1)
    assert c["kind"] == "oracle" and c["cores"] == 1 and c["unit"] == "link updates/s"
    assert c["value"] > 0 and "4^4" in c["sample"]

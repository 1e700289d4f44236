"""Host logic of bench.py (no GPU): the roofline peaks of each staging, the
refusal of more than one GPU, and the traffic figure's tie to the kernel
sources its counters were taken with."""
import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_peaks_from_unit_counts(bench):
    # 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz of 32-bit VALU lane operations
    lane_ops = 256 * 4 * 16 * 2.4e9 / 1e12
    assert bench.CMP_PEAK_TOPS == pytest.approx(lane_ops)
    # SWAR codes: 5 operations per two column steps, 4 (bytes) or 2 (16-bit) rows per operation
    assert bench.BYTE_PEAK_TOPS == pytest.approx(lane_ops * 4 / 2.5)
    assert bench.HALF_PEAK_TOPS == pytest.approx(lane_ops * 2 / 2.5)


@pytest.mark.parametrize("staging,peak_name,unit", [
    (3, "BYTE_PEAK_TOPS", "T row-checks/s"),
    (4, "HALF_PEAK_TOPS", "T row-checks/s"),
    (2, "CMP_PEAK_TOPS", "T compare lane-ops/s"),
    (0, "CMP_PEAK_TOPS", "T compare lane-ops/s"),
    (None, "CMP_PEAK_TOPS", "T compare lane-ops/s"),
])
def test_alu_roofline(bench, staging, peak_name, unit):
    steps, k_ms = 3_000_000, 0.1
    r = bench.alu_roofline(steps, k_ms, staging)
    achieved = steps * 64 / (k_ms * 1e-3) / 1e12
    assert r["bound"] == "alu" and r["unit"] == unit
    assert r["achieved"] == pytest.approx(achieved)
    assert r["peak"] == getattr(bench, peak_name)
    assert r["frac"] == pytest.approx(achieved / r["peak"])


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_traffic_only_for_matching_kernel_sources(bench, tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    csrc = tmp_path / "paper_1807_09932_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in bench.KERNEL_SOURCES:
        (csrc / f).write_text("// " + f + "\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    sha = bench.kernel_sources_sha()
    path = prof / "k_eval_methylation_436444x64_traffic.json"
    assert bench.traffic_from_profile(1) is None  # no summary
    path.write_text(json.dumps({"kernel_sources_sha": sha, "hbm_bytes_per_launch": 1234.0,
                                "launch_shape": [8, 16, 200, 3]}))
    assert bench.traffic_from_profile(1) == 1234.0
    assert bench.traffic_from_profile(1, shape=(8, 16, 200, 3)) == 1234.0
    assert bench.traffic_from_profile(1, shape=(16, 16, 200, 3)) is None  # another launch shape
    path.write_text(json.dumps({"kernel_sources_sha": sha, "hbm_bytes_per_launch": 1234.0,
                                "launch_shape": [8, 16, 200, 3],
                                "other_shapes": [{"launch_shape": [16, 16, 200, 3],
                                                  "hbm_bytes_per_launch": 999.0}]}))
    assert bench.traffic_from_profile(1, shape=(16, 16, 200, 3)) == 999.0
    assert bench.traffic_from_profile(1, shape=(4, 16, 200, 3)) is None
    (csrc / bench.KERNEL_SOURCES[0]).write_text("// changed\n")
    assert bench.traffic_from_profile(1) is None  # the kernel changed since


def test_pair_window_pairs_counts_distinct_window_pairs():
    import numpy as np
    import bench
    from paper_1807_09932_amd import gen
    inds = [[1, 2, 3], [3, 3, 1], [5], [1, 2, 1, 2], [4, 4, 4],
            [0, 1, 2, 3, 4, 5, 6, 7, 8, 9],   # past the window: (7, 8), (8, 9) not read per chunk
            [6, 6, 7, 7, 6], [2, 99]]          # inner repeats; an invalid column: pair (0, 0)
    offs, cols = gen.csr([np.asarray(i, np.int32) for i in inds])
    want = {(1, 2), (2, 3), (3, 1), (5, 5), (2, 1), (4, 4),
            (0, 1), (1, 2), (2, 3), (3, 4), (4, 5), (5, 6), (6, 7), (7, 6), (0, 0)}
    assert bench.pair_window_pairs(offs, cols, 10) == len(want)

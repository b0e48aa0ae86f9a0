"""Host-side checks of bench.py (no GPU): the one-GPU contract, the
algorithmic byte model of the CG kernel and the roofline record built from
per-kernel timings."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_cg_bytes_follow_the_documented_terms():
    # n rows, T tets, nnz CSR entries (diagonal included), FP32 and FP64:
    # B_pcg = (W + 4) nnz + 4 (n + 1) + 35 W n per CG iteration
    info = {"n_verts": 100, "n_tets": 300, "nnz": 1500, "n_query_verts": 40}
    for W in (4, 8):
        assert bench.pcg_bytes_per_iteration(info, W) == (W + 4) * 1500 + 4 * 101 + 35 * W * 100
    n, T, off, W = 100, 300, 1400, 4
    ex = bench.pcg_extra_bytes(info, W)
    assert ex["gather"] == 4 * T * 4 * W + n * (4 + 6 * W)
    assert ex["final_update"] == n * (9 * W + 24)
    assert ex["warm_start"] == n * (13 * W) + off * (4 + W) + n * 9 * W + n * 30 * W + off * W


def test_roofline_record_from_kernel_timings():
    info = {"n_verts": 100, "n_tets": 300, "nnz": 1500, "n_query_verts": 40}
    prof = {"pcg": (2.0, 4), "tet_query": (0.5, 4), "ray_cast": (0.1, 4)}  # ms total, launches
    r = bench.roofline_of(prof, info, 4, 40, traffic_key="no-such-workload")
    per_launch = 10 * bench.pcg_bytes_per_iteration(info, 4)           # 40 CG iterations over 4 launches
    assert r["kernel"] == "pcg" and r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["avg_launch_us"] == pytest.approx(500.0)
    assert r["algorithmic_bytes_per_launch"] == per_launch
    assert r["achieved"] == pytest.approx(per_launch / 500e-6 / 1e9, rel=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / bench.PEAK_HBM_GBS, abs=1e-5)  # rounded to 5 places
    assert r["traffic"] is None  # counters exist only for the measured workloads


def test_roofline_traffic_only_for_the_measured_workload_and_grid():
    info = {"n_verts": 100, "n_tets": 300, "nnz": 1500, "n_query_verts": 40}
    prof = {"pcg": (2.0, 4)}
    (wl, grid), per_cg = next(iter(bench.PMC_TRAFFIC_PER_CG_ITERATION.items()))
    r = bench.roofline_of(prof, info, 4, 40, traffic_key=(wl, grid))
    assert r["traffic"] == int(per_cg * 10)  # 10 CG iterations per launch
    assert bench.roofline_of(prof, info, 4, 40, traffic_key=(wl, grid + 1))["traffic"] is None


def test_physical_core_count_is_within_the_allowed_cpus():
    cores, allowed = bench.physical_cores()
    assert 1 <= cores <= allowed == len(os.sched_getaffinity(0))

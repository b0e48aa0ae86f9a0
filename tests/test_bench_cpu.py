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
    # n rows, T tets, nnz ELL entries (diagonal included), S query vertices,
    # FP32; 3 launches doing 30 CG iterations in all
    info = {"n_verts": 100, "n_tets": 300, "nnz": 1500, "n_query_verts": 40}
    W, n, T, off, S = 4, 100, 300, 1400, 40
    kb = bench.kernel_bytes(info, W, {"pcg": 3}, 30)
    gather = 4 * T * 4 * W + n * (4 + 6 * W)                    # phase 0
    per_it = n * (24 * W + 17 * W) + off * (4 + W)              # per CG iteration
    startup = n * 81 * W + off * (8 + 3 * W)
    finish = n * (7 * W + 24) + 36 * S
    assert kb["gather"] == gather
    assert kb["pcg"] == pytest.approx(gather + 10 * per_it + startup + finish, rel=0, abs=1e-6)
    assert kb["hash_insert"] == 60 * S


def test_roofline_record_from_kernel_timings():
    info = {"n_verts": 100, "n_tets": 300, "nnz": 1500, "n_query_verts": 40}
    prof = {"pcg": (2.0, 4), "tet_query": (0.5, 4), "ray_cast": (0.1, 4)}  # ms total, launches
    r = bench.roofline_of(prof, info, 4, 40, workload="no-such-workload")
    kb = bench.kernel_bytes(info, 4, {k: v[1] for k, v in prof.items()}, 40)["pcg"]
    assert r["kernel"] == "pcg" and r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["avg_launch_us"] == pytest.approx(500.0)
    assert r["achieved"] == pytest.approx(kb / 500e-6 / 1e9, rel=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / bench.PEAK_HBM_GBS, abs=1e-5)  # rounded to 5 places
    assert r["traffic"] is None  # counters exist only for the measured workloads
    assert bench.roofline_of(prof, info, 4, 40, workload="finger")["traffic"] == bench.PMC_TRAFFIC[("finger", "pcg")]

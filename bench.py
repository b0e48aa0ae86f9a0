"""Benchmark: tet-iterations per second of the collision-aware local/global
solve to the 1e-6 residual on one GPU.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload finger]

A step is one complete solve of the workload from its rest shape (all
iterations until r_k <= 1e-6 with an unchanged active set).  Inputs are
resident on the device before the timed region.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def kernel_bytes(info, W, n_launch, pcg_iters):
    """Algorithmic bytes per launch of each kernel: the data the method must
    move, each array element counted once per launch (W = 4 or 8 bytes per
    real, int32 indices, collision positions in double).

      pcg        per CG iteration: per row the CG state (r, w, s: 3 vectors of
                 4 reals) read and written, p and the correction read and
                 written, the Jacobi diagonal; per off-diagonal entry its column
                 and value.  Plus the two start-up passes and the end-of-iteration
                 update (u read/written, correction read, collision positions
                 written).
      local      per tet connectivity 16, tag 4, residual slot index 16, residual
                 columns written 4 x 4W; per vertex rest position 24 and
                 displacement 3W read once.
      gather     per incidence one residual column 4W; per vertex the
                 incidence range 4, right-hand side 4W and two diagonals 2W.
      tet_query  per tet connectivity 16; per vertex its collision position 24.
      hash_insert per query vertex its id 4, position 24, entry written 32.
    """
    n, T, nnz = info["n_verts"], info["n_tets"], info["nnz"]
    S = info["n_query_verts"]
    off = nnz - n
    out = {}
    m = pcg_iters / max(n_launch.get("pcg", 1), 1)
    per_it = n * (12 * W * 2 + 8 * W + 8 * W + W) + off * (4 + W)
    startup = n * (17 * W) + off * (4 + 2 * W) + n * (9 * W) + off * (4 + W)
    finish = n * (3 * W + 4 * W + 24) + 4 * info["hash_buckets"]
    out["pcg"] = m * per_it + startup + finish
    out["local"] = T * (36 + 16 * W) + n * (24 + 3 * W)
    out["gather"] = 4 * T * 4 * W + n * (4 + 6 * W)
    out["tet_query"] = 16 * T + 24 * n
    out["hash_insert"] = S * 60
    return out


def run_cpu_baseline(wl, budget_s=15.0):
    import torch
    import oracle
    from oracle import solver as so
    prob = oracle.Problem.from_workload(wl)
    x = prob.X0.copy()
    prev = None
    fac = so._Factor()
    t0 = time.perf_counter()
    it = 0
    while True:
        x, prev, _, _ = so.step(prob, x, wl.alpha, prev, fac)
        it += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": prob.T * it / dt, "unit": "tet-iterations/s", "cores": int(torch.get_num_threads()),
            "kind": "oracle",
            "sample": f"first {it} local/global iterations of the {prob.T}-tet finger from rest "
                      f"(FP64 oracle: brute-force collision, sparse direct global step), {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="finger")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the sharding plan is described in DESIGN.md).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2203_02054_amd import geosim as G
    from paper_2203_02054_amd import meshgen as mg

    wl = mg.make(a.workload)
    gp = G.Problem.from_workload(wl, precision=wl.precision)
    W = wl.precision
    x0 = gp.tensor(wl.rest_xyz)
    alpha = gp.tensor(wl.alpha)
    x = x0.clone()
    stream = gp.stream

    def step():
        x.copy_(x0)
        gp.reset_contacts()
        _, st = gp.solve(alpha, x)
        return st

    print(f"# warmup {a.warmup} solves of {wl.name} ({wl.n_tets} tets)", file=sys.stderr, flush=True)
    for _ in range(a.warmup):
        st = step()
    torch.cuda.synchronize()
    gp.profile(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stats = []
    t_host = time.perf_counter()
    e0.record(stream)
    for i in range(a.steps):
        stats.append(step())
        print(f"# step {i}: {stats[-1]}", file=sys.stderr, flush=True)
    e1.record(stream)
    torch.cuda.synchronize()
    t_host = time.perf_counter() - t_host
    ms = e0.elapsed_time(e1)
    prof = gp.profile_read()
    gp.profile(False)

    iters = sum(s["iters"] for s in stats)
    pcg_iters = sum(s["pcg_iters_total"] for s in stats)
    value = wl.n_tets * iters / (ms / 1e3)
    n_launch = {k: v[1] for k, v in prof.items()}
    kb = kernel_bytes(gp.info, W, n_launch, pcg_iters)
    dom = max((k for k in prof if prof[k][1] > 0), key=lambda k: prof[k][0])
    avg_ms = prof[dom][0] / prof[dom][1]
    roof = None
    if dom in kb:
        achieved = kb[dom] / (avg_ms / 1e3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 5), "traffic": None, "kernel": dom,
                "avg_launch_us": round(1e3 * avg_ms, 3), "algorithmic_bytes_per_launch": int(kb[dom])}
    kernels = {k: {"total_ms": round(v[0], 3), "launches": v[1],
                   "avg_us": round(1e3 * v[0] / v[1], 3) if v[1] else None} for k, v in prof.items() if v[1]}
    out = {
        "metric": "tet-iterations/sec to 1e-6 residual (plain solve)",
        "value": round(value, 1),
        "unit": "tet-iterations/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms / a.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if W == 4 else "f64",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: {wl.n_tets} tets, {wl.n_verts} verts, {wl.n_chambers} chambers, "
                               f"self-collision {'on' if wl.self_collision else 'off'}, plain solve to 1e-6",
                   "tets": wl.n_tets, "outer_iters_per_step": iters / a.steps,
                   "pcg_iters_per_step": pcg_iters / a.steps, "contacts": stats[-1]["n_contacts"],
                   "residual": stats[-1]["residual"]},
        "roofline": roof,
        "kernels": kernels,
        "host_s": round(t_host, 3),
    }
    if not a.no_cpu_baseline:
        print("# cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = run_cpu_baseline(wl, a.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

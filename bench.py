"""Benchmark: tet-iterations per second of the collision-aware local/global
solve to the 1e-6 residual on one GPU, plain and batched, and adjoint
gradients per second.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload finger]

Headline (``value``): a step is one complete solve of the workload (default:
the 26,880-tet, 8-chamber finger) from its rest shape, all iterations until
r_k <= 1e-6 with an unchanged active set.  Inputs are resident on the device
before the timed region; the K steps are timed with HIP events on the
library's stream, without per-kernel events.  The same K steps are then run
again with per-kernel events for the kernel table and the roofline of the
dominant kernel.

Extra legs (same JSON line):
  batched  256 finger meshes of uneven size in one problem, solved once from
           rest (iterations capped); throughput sum_i T_i K_i / t and the
           speedup over solving a sample of the meshes one by one.
  adjoint  gs_adjoint on the converged finger for a fingertip loss: gradients
           per second, and the speedup over a finite-difference gradient by
           plain solves (2 solves per chamber).
  cpu_baseline  the FP64 oracle on the host cores for a bounded sample.
Prints one JSON line.
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

# HBM bytes per launch of the dominant kernel measured with rocprofv3 counters
# (FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000, factors from a 256 MiB copy);
# see profiles/*_hbm_traffic.md.  Only valid for the kernel build the counters
# were taken on: remove an entry when its kernel changes.
PMC_TRAFFIC = {("finger", "pcg"): 20769319, ("batched", "pcg"): 29054596115}


def kernel_bytes(info, W, n_launch, pcg_iters):
    """Algorithmic bytes per launch of each kernel: the data the method must
    move, each array element counted once per launch (W = 4 or 8 bytes per
    real, int32 indices, collision positions in double).

      pcg        phase 0, the right-hand-side gather (as `gather` below; the
                 contact update of the few active contact slots is not
                 counted).  Per CG iteration: per row the CG state (r, w, s: 3
                 vectors of 4 reals) read and written, p and the correction read
                 and written, the Jacobi diagonal; per off-diagonal entry its
                 column and value.  Plus the start-up (the warm start: the last three
                 corrections, right-hand side and diagonal read, their three
                 products written; the scaled ELL values written; then the
                 start, its residual and w_0 = A u_0 formed, the history moved
                 on) and the end-of-iteration update (u read/written,
                 correction read, collision positions written, each query
                 vertex's 32-byte hash entry and bucket count).
      local      per tet connectivity 16, tag 4, residual slot index 16, residual
                 columns written 4 x 4W; per vertex rest position 24 and
                 displacement 3W read once.
      gather     per incidence one residual column 4W; per vertex the
                 incidence range 4, right-hand side 4W and two diagonals 2W
                 (the CG kernel's phase 0; the adjoint's own gather kernel).
      tet_query  per tet connectivity 16; per vertex its collision position 24.
      hash_insert per query vertex its id 4, position 24, entry written 32.
    """
    n, T, nnz = info["n_verts"], info["n_tets"], info["nnz"]
    S = info["n_query_verts"]
    off = nnz - n
    out = {}
    m = pcg_iters / max(n_launch.get("pcg", 1), 1)
    per_it = n * (12 * W * 2 + 8 * W + 8 * W + W) + off * (4 + W)
    startup = n * (29 * W) + off * (4 + 2 * W) + n * (52 * W) + off * (4 + W)
    finish = n * (3 * W + 4 * W + 24) + S * 36
    out["gather"] = 4 * T * 4 * W + n * (4 + 6 * W)
    out["pcg"] = out["gather"] + m * per_it + startup + finish
    out["local"] = T * (36 + 16 * W) + n * (24 + 3 * W)
    out["tet_query"] = 16 * T + 24 * n
    out["hash_insert"] = S * 60
    return out


def roofline_of(prof, info, W, pcg_iters, workload=None):
    n_launch = {k: v[1] for k, v in prof.items()}
    kb = kernel_bytes(info, W, n_launch, pcg_iters)
    dom = max((k for k in prof if prof[k][1] > 0), key=lambda k: prof[k][0])
    avg_ms = prof[dom][0] / prof[dom][1]
    if dom not in kb:
        return None
    achieved = kb[dom] / (avg_ms / 1e3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 2), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 5), "traffic": PMC_TRAFFIC.get((workload, dom)), "kernel": dom,
            "avg_launch_us": round(1e3 * avg_ms, 3), "algorithmic_bytes_per_launch": int(kb[dom])}


def kernel_table(prof):
    return {k: {"total_ms": round(v[0], 3), "launches": v[1], "avg_us": round(1e3 * v[0] / v[1], 3) if v[1] else None}
            for k, v in prof.items() if v[1]}


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


def timed_on(stream, fn):
    """Run fn() between two HIP events recorded on `stream`; return (ms, result)."""
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    r = fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1), r


def run_batched(G, mg, n_mesh, max_iter, sample, autotune=True):
    import torch
    wls = mg.batched(n_mesh)
    Ts = np.array([w.n_tets for w in wls], dtype=np.int64)
    print(f"# batched: {n_mesh} meshes, {int(Ts.sum())} tets", file=sys.stderr, flush=True)
    gb = G.Problem.batch(wls, precision=4, self_collision=1, max_iter=max_iter)
    alpha = gb.tensor(np.concatenate([w.alpha for w in wls]))
    x0 = gb.tensor(gb._X)
    x = x0.clone()
    grid = gb.autotune(alpha, x, iters=8)[0] if autotune else gb.info["pcg_grid"]

    def solve():
        x.copy_(x0)
        gb.reset_contacts()
        return gb.solve(alpha, x)[1]

    solve()                                                   # warm-up
    torch.cuda.synchronize()
    ms, st = timed_on(gb.stream, solve)
    its = gb.mesh_iters().astype(np.int64)
    K = np.where(its > 0, its, st["iters"])                  # capped meshes ran every iteration
    value = float((Ts * K).sum() / (ms / 1e3))
    # kernel averages and the CG roofline from a profiled prefix of the same solve
    gb.set_params(max_iter=min(200, max_iter))
    gb.profile(True)
    x.copy_(x0)
    gb.reset_contacts()
    _, st_p = gb.solve(alpha, x)
    prof = gb.profile_read()
    gb.profile(False)
    roof = roofline_of(prof, gb.info, 4, st_p["pcg_iters_total"], "batched")
    # plain path on a sample of the meshes (every n_mesh/sample-th), one by one
    idx = list(range(0, n_mesh, max(1, n_mesh // sample)))[:sample]
    t_plain, work_plain = 0.0, 0
    for i in idx:
        w = wls[i]
        gp = G.Problem.from_workload(w, precision=4, max_iter=max_iter)
        a = gp.tensor(w.alpha)
        xx0 = gp.tensor(w.rest_xyz)
        xx = xx0.clone()

        def solve1():
            xx.copy_(xx0)
            gp.reset_contacts()
            return gp.solve(a, xx)[1]

        solve1()
        torch.cuda.synchronize()
        ms1, st1 = timed_on(gp.stream, solve1)
        t_plain += ms1 / 1e3
        work_plain += w.n_tets * st1["iters"]
        gp.close()
    rate_plain = work_plain / t_plain
    out = {"value": round(value, 1), "unit": "tet-iterations/s", "ms_per_step": round(ms, 3),
           "meshes": n_mesh, "tets": int(Ts.sum()), "chambers": int(sum(w.n_chambers for w in wls)),
           "max_iter": max_iter, "outer_iters": st["iters"], "pcg_iters": st["pcg_iters_total"], "pcg_grid": grid,
           "converged_meshes": int((its > 0).sum()),
           "plain_sample": {"meshes": len(idx), "value": round(rate_plain, 1), "unit": "tet-iterations/s"},
           "speedup_vs_plain": round(value / rate_plain, 3), "roofline": roof, "kernels": kernel_table(prof)}
    gb.close()
    return out


def run_adjoint(G, mg, wl, gp, x, alpha, t_solve_ms, n_iters, reps=3):
    """Adjoint of the converged solve left in gp (positions x)."""
    import torch
    verts, y = mg.finger_tip_targets(wl)
    xs = x.double().cpu().numpy()
    g = np.zeros((3, wl.n_verts))
    g[:, verts] = 2.0 * (xs[:, verts] - y.T)
    gt = gp.tensor(g)
    gp.set_params(adj_tol=1e-6, adj_aa_m=16)
    ga, st = gp.adjoint(gt)                                   # warm-up
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        ms, (ga, st) = timed_on(gp.stream, lambda: gp.adjoint(gt))
        times.append(ms)
    gp.profile(True)
    gp.adjoint(gt)
    prof = gp.profile_read()
    gp.profile(False)
    t = float(np.median(times))
    fd_ms = 2 * wl.n_chambers * t_solve_ms
    # unrolled variant over the solve's own iteration budget, from rest
    K = int(n_iters)
    gp.reset_contacts()
    gp.adjoint_unrolled(alpha, K, gt)                        # warm-up
    gp.reset_contacts()
    torch.cuda.synchronize()
    ms_u, (ga_u, _, _, st_u) = timed_on(gp.stream, lambda: gp.adjoint_unrolled(alpha, K, gt))
    return {"value": round(1e3 / t, 3), "unit": "gradients/s", "ms_per_gradient": round(t, 3),
            "params": wl.n_chambers, "adjoint_iters": st["iters"], "pcg_iters": st["pcg_iters_total"],
            "residual": st["residual"], "status": st["status"], "anderson_memory": 16,
            "loss": "sum of squared distances of 10 fingertip vertices to seeded targets",
            "forward_plus_adjoint_ms": round(t_solve_ms + t, 3),
            "fd_plain_ms": round(fd_ms, 3), "speedup_vs_fd": round(fd_ms / t, 2),
            "grad_norm": float(torch.linalg.norm(ga.double()).item()),
            "unrolled": {"value": round(1e3 / ms_u, 3), "unit": "gradients/s", "ms_per_gradient": round(ms_u, 3),
                         "K": K, "pcg_iters": st_u["pcg_iters_total"],
                         "note": "K iterations from rest, checkpoints every ceil(sqrt(K)), forward + reverse sweep"},
            "kernels": {k: v for k, v in kernel_table(prof).items() if k.startswith("adj_")}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="finger")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-meshes", type=int, default=256)
    ap.add_argument("--batched-max-iter", type=int, default=1000)
    ap.add_argument("--plain-sample", type=int, default=8)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default CG grid (counter runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 20 device-to-device copies of MIB MiB (reference traffic for HBM counters)")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(N > 1 is not supported).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2203_02054_amd import geosim as G
    from paper_2203_02054_amd import meshgen as mg

    if a.copy_calibration:
        n = a.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(20):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_per_copy": 4 * n, "copies": 20}), flush=True)
        return

    wl = mg.make(a.workload)
    gp = G.Problem.from_workload(wl, precision=wl.precision)
    W = wl.precision
    x0 = gp.tensor(wl.rest_xyz)
    alpha = gp.tensor(wl.alpha)
    x = x0.clone()
    stream = gp.stream
    grid = gp.info["pcg_grid"] if a.no_autotune else gp.autotune(alpha, x, iters=20)[0]

    def step():
        x.copy_(x0)
        gp.reset_contacts()
        _, st = gp.solve(alpha, x)
        return st

    print(f"# warmup {a.warmup} solves of {wl.name} ({wl.n_tets} tets)", file=sys.stderr, flush=True)
    for _ in range(a.warmup):
        st = step()
    torch.cuda.synchronize()
    stats = []

    def timed_steps():
        for i in range(a.steps):
            stats.append(step())
            print(f"# step {i}: {stats[-1]}", file=sys.stderr, flush=True)

    t_host = time.perf_counter()
    ms, _ = timed_on(stream, timed_steps)
    t_host = time.perf_counter() - t_host

    # the same steps again with per-kernel events (kernel table, roofline)
    gp.profile(True)
    pstats = []
    for _ in range(a.steps):
        x.copy_(x0)
        gp.reset_contacts()
        pstats.append(gp.solve(alpha, x)[1])
    torch.cuda.synchronize()
    prof = gp.profile_read()
    gp.profile(False)

    iters = sum(s["iters"] for s in stats)
    pcg_iters = sum(s["pcg_iters_total"] for s in stats)
    value = wl.n_tets * iters / (ms / 1e3)
    roof = roofline_of(prof, gp.info, W, sum(s["pcg_iters_total"] for s in pstats), wl.name)
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
                   "pcg_iters_per_step": pcg_iters / a.steps, "pcg_grid": grid, "contacts": stats[-1]["n_contacts"],
                   "residual": stats[-1]["residual"]},
        "roofline": roof,
        "kernels": kernel_table(prof),
        "host_s": round(t_host, 3),
    }
    if not a.no_adjoint:
        print("# adjoint", file=sys.stderr, flush=True)
        out["adjoint"] = run_adjoint(G, mg, wl, gp, x, alpha, ms / a.steps, iters / a.steps)
    gp.close()
    if not a.no_batched:
        out["batched"] = run_batched(G, mg, a.batched_meshes, a.batched_max_iter, a.plain_sample,
                                     autotune=not a.no_autotune)
    if not a.no_cpu_baseline:
        print("# cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = run_cpu_baseline(wl, a.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""Benchmark: tet-iterations per second of the collision-aware local/global
solve to the 1e-6 residual on one GPU, plain and batched, and adjoint
gradients per second.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload gripper]

Headline (``value``): a step is one complete solve of the workload (default:
the three-finger gripper, 378,666 tets, the largest single-GPU
configuration) from its rest shape, every outer iteration until r_k <= 1e-6
with an unchanged active set, with the workload's solver settings (for the
gripper the Anderson-accelerated iteration).  value = T * (outer iterations
of the K steps) / time.  Inputs are resident on the device before the timed
region; the K steps are timed with HIP events on the library's stream,
without per-kernel events.  One more solve is run with per-kernel events for
the kernel table and the roofline of the dominant kernel (the CG kernel).

Extra legs (same JSON line):
  coarse   the headline workload's first 200 outer iterations with the
           Jacobi and with the coarse-corrected CG (fixed count).
  membrane the four-chamber membrane rig solved to 1e-6.
  finger_sweep  the CG kernel's fraction of HBM peak against size: the
           finger at voxel sizes 2, 1.2, 0.8 and 0.6 mm (26,880 to 971,634
           tets), its first 30 outer iterations (fixed count).
  adjoint  gs_adjoint at the converged gripper for the fingertip loss (30
           tip vertices to seeded targets, gradient w.r.t. the 24 chamber
           ratios): gradients per second, and the speedup over a
           finite-difference gradient by plain solves (2 solves per chamber).
  batched  256 finger meshes of uneven size in one problem, solved once from
           rest (iterations capped): sum_i T_i K_i / t over the meshes that
           reached 1e-6 (the capped meshes' work is reported apart), and the
           speedup over solving a sample of the meshes one by one.
  stream_copy  device-to-device copies of 2 GiB: the streaming bandwidth
           this GPU reaches, beside the 8 TB/s peak of the roofline.
  cpu_baseline  the FP64 oracle on the host cores for a bounded sample of one
           gripper iteration, with all physical cores of this process's CPU
           share and with one thread.
Prints one JSON line.
"""
import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0

# HBM bytes per CG iteration of the dominant kernel measured with rocprofv3
# counters (FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000, factors from 256 MiB
# device copies; the launch's fixed parts spread over its CG iterations), keyed
# by workload and CG grid: a run on another grid reports no traffic, and an
# entry is removed when its kernel changes (profiles/*_hbm_traffic.md).
PMC_TRAFFIC_PER_CG_ITERATION = {
    ("gripper", 192): 24140421,    # k_pcg<float, 16, false, false, false, false, false>
    ("batched", 256): 558327374,   # k_pcg<float, 16, false, false, false, false, true>
}


def pcg_bytes_per_iteration(info, W):
    """Algorithmic bytes of one CG iteration: (W + 4) nnz + 4 (n + 1) + 35 W n
    (the CSR values and int32 columns, the row pointers, and the
    three-component vector streams of the SpMV (p in, q out), the update (x,
    r, p, q in; x, r out; the diagonal) and the p-update (r, diagonal, p in;
    p out))."""
    n, nnz = info["n_verts"], info["nnz"]
    return (W + 4) * nnz + 4 * (n + 1) + 35 * W * n


def pcg_extra_bytes(info, W):
    """Bytes the CG kernel moves once per launch besides its iterations, not
    part of B_pcg and reported apart: the right-hand-side gather (per
    incidence one residual column 4W; per vertex the incidence range 4, the
    right-hand side 4W and two diagonals 2W), the warm start (pass 1 reads
    the three history vectors, the right-hand side, the diagonal and the
    off-diagonal entries, and writes the three products; pass 2 reads the
    right-hand side and the products, writes the start, the history, the
    start's r, w, s and the scaled off-diagonal values), and the final update
    (correction and displacement read, displacement and FP64 collision
    positions written)."""
    n, T, off = info["n_verts"], info["n_tets"], info["nnz"] - info["n_verts"]
    gather = 4 * T * 4 * W + n * (4 + 6 * W)
    startup = (n * (9 * W + 3 * W + W) + off * (4 + W) + n * 9 * W
               + n * 12 * W + n * 18 * W + off * W)
    finish = n * (9 * W + 24)
    return {"gather": gather, "warm_start": startup, "final_update": finish}


def roofline_of(prof, info, W, pcg_iters, traffic_key=None):
    launches = prof["pcg"][1]
    avg_ms = prof["pcg"][0] / launches
    m = pcg_iters / launches
    per_launch = m * pcg_bytes_per_iteration(info, W)
    achieved = per_launch / (avg_ms / 1e3) / 1e9
    extra = pcg_extra_bytes(info, W)
    pmc = PMC_TRAFFIC_PER_CG_ITERATION.get(traffic_key)
    return {"bound": "hbm", "achieved": round(achieved, 3), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 5), "traffic": int(pmc * m) if pmc else None,
            "kernel": "pcg", "avg_launch_us": round(1e3 * avg_ms, 3), "launches": launches,
            "cg_iterations_per_launch": round(m, 3),
            "bytes_per_cg_iteration": int(pcg_bytes_per_iteration(info, W)),
            "algorithmic_bytes_per_launch": int(per_launch),
            "not_counted_bytes_per_launch": {k: int(v) for k, v in extra.items()},
            "with_those_frac": round((per_launch + sum(extra.values())) / (avg_ms / 1e3) / 1e9 / PEAK_HBM_GBS, 5)}


def kernel_table(prof):
    return {k: {"total_ms": round(v[0], 3), "launches": v[1], "avg_us": round(1e3 * v[0] / v[1], 3) if v[1] else None}
            for k, v in prof.items() if v[1]}


def physical_cores():
    """Physical cores among the CPUs this process may run on (lscpu's
    core/socket pairs), and the number of those CPUs."""
    allowed = sorted(os.sched_getaffinity(0))
    try:
        out = subprocess.run(["lscpu", "-p=CPU,CORE,SOCKET"], capture_output=True, text=True, check=True).stdout
        pairs = set()
        for line in out.splitlines():
            if line.startswith("#"):
                continue
            cpu, core, sock = (int(t) for t in line.split(",")[:3])
            if cpu in allowed:
                pairs.add((sock, core))
        return max(1, len(pairs)), len(allowed)
    except Exception:
        return max(1, len(allowed)), len(allowed)


def run_cpu_baseline(wl, query_fraction=0.02):
    """One local/global iteration of the FP64 oracle on the workload from
    rest, timed by phase: collision (brute force over a seeded sample of the
    query vertices, scaled to all of them), local step, global step (sparse
    factorisation and solve).  Run with all physical cores of this process's
    CPU share and with one thread."""
    import torch
    import oracle
    from oracle import collision as oc
    from oracle import local as ol
    from oracle import solver as so
    prob = oracle.Problem.from_workload(wl)
    x = prob.X0.copy()
    rng = np.random.default_rng(0)
    qs = np.sort(rng.choice(prob.query_verts, max(1, int(query_fraction * prob.query_verts.size)), replace=False))
    cores, allowed = physical_cores()
    legs = {}
    for threads in (cores, 1):
        torch.set_num_threads(threads)
        os.environ["OMP_NUM_THREADS"] = str(threads)
        t0 = time.perf_counter()
        oc.tet_candidates(prob, x, qs)
        t_col = (time.perf_counter() - t0) * prob.query_verts.size / qs.size
        t0 = time.perf_counter()
        Tt = ol.local_step(prob, x, wl.alpha)
        t_loc = time.perf_counter() - t0
        t0 = time.perf_counter()
        so.global_step(prob, Tt, oc.Contacts.empty(prob.query_verts.size, prob.n_slots), x, so._Factor())
        t_glob = time.perf_counter() - t0
        t_it = t_col + t_loc + t_glob
        legs[threads] = dict(t_it=t_it, collision_s=round(t_col, 3), local_s=round(t_loc, 3),
                             global_s=round(t_glob, 3))
    best = legs[cores]
    return {"value": round(prob.T / best["t_it"], 1), "unit": "tet-iterations/s", "cores": cores, "kind": "oracle",
            "sample": (f"one oracle iteration of the {prob.T}-tet {wl.name} from rest (FP64, NumPy/SciPy/PyTorch on "
                       f"the host): brute-force tet candidates for a seeded {query_fraction:.0%} of the "
                       f"{prob.query_verts.size} query vertices scaled to all, local step, sparse direct global "
                       f"step; {cores} physical cores of {allowed} allowed CPUs (torch threads; the brute "
                       f"force and SuperLU run on one)"),
            "per_phase_s": {k: v for k, v in best.items() if k != "t_it"},
            "one_thread": {"value": round(prob.T / legs[1]["t_it"], 1), "cores": 1,
                           "per_phase_s": {k: v for k, v in legs[1].items() if k != "t_it"}},
            "without_collision": round(prob.T / (best["local_s"] + best["global_s"]), 1)}


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
    conv = its > 0
    value = float((Ts[conv] * its[conv]).sum() / (ms / 1e3))
    capped_work = float(Ts[~conv].sum() * st["iters"])
    # kernel averages and the CG roofline from a profiled prefix of the same solve
    gb.set_params(max_iter=min(200, max_iter))
    gb.profile(True)
    x.copy_(x0)
    gb.reset_contacts()
    _, st_p = gb.solve(alpha, x)
    prof = gb.profile_read()
    gb.profile(False)
    roof = roofline_of(prof, gb.info, 4, st_p["pcg_iters_total"], ("batched", grid))
    # plain path on a sample of the meshes (every n_mesh/sample-th), one by one
    idx = list(range(0, n_mesh, max(1, n_mesh // sample)))[:sample]
    t_plain, work_plain = 0.0, 0
    for i in idx:
        w = wls[i]
        with G.Problem.from_workload(w, precision=4, max_iter=max_iter) as gp:
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
        if st1["status"] == G.OK:
            t_plain += ms1 / 1e3
            work_plain += w.n_tets * st1["iters"]
    rate_plain = work_plain / t_plain if t_plain > 0 else None
    # the same batch with the per-mesh CG (each mesh's own workgroups and CG
    # scalars), its workgroup budget autotuned the same way
    gb.set_params(max_iter=max_iter, pcg_per_mesh=1, pcg_blocks=0)
    budget_pm = gb.autotune(alpha, x, iters=8)[0] if autotune else None
    plan_pm = gb.cg_plan()
    solve()
    torch.cuda.synchronize()
    ms_pm, st_pm = timed_on(gb.stream, solve)
    its_pm = gb.mesh_iters().astype(np.int64)
    conv_pm = its_pm > 0
    value_pm = float((Ts[conv_pm] * its_pm[conv_pm]).sum() / (ms_pm / 1e3))
    per_mesh = {"value": round(value_pm, 1), "unit": "tet-iterations/s", "ms_per_step": round(ms_pm, 3),
                "outer_iters": st_pm["iters"], "pcg_iters": st_pm["pcg_iters_total"],
                "converged_meshes": int(conv_pm.sum()), "capped_meshes": int((~conv_pm).sum()),
                "capped_tet_iterations": float(Ts[~conv_pm].sum() * st_pm["iters"]),
                "aa_rejected": st_pm["aa_rejected"], "workgroups": int(plan_pm.sum()),
                "max_workgroups_per_mesh": int(plan_pm.max()),
                "note": "pcg_per_mesh=1: each mesh's CG on its own workgroups, a mesh's path is its path alone"}
    # the per-mesh CG with the longest-processing-time plan (large meshes
    # split, the smallest queued), on the default budget
    try:
        gb.set_params(max_iter=max_iter, pcg_per_mesh=2, pcg_blocks=0)
        plan_lpt = gb.cg_plan()
        solve()
        torch.cuda.synchronize()
        ms_l, st_l = timed_on(gb.stream, solve)
        its_l = gb.mesh_iters().astype(np.int64)
        conv_l = its_l > 0
        per_mesh["lpt_plan"] = {
            "value": round(float((Ts[conv_l] * its_l[conv_l]).sum() / (ms_l / 1e3)), 1), "unit": "tet-iterations/s",
            "ms_per_step": round(ms_l, 3), "outer_iters": st_l["iters"], "pcg_iters": st_l["pcg_iters_total"],
            "converged_meshes": int(conv_l.sum()), "capped_meshes": int((~conv_l).sum()),
            "workgroups": int(plan_lpt.sum()), "split_meshes": int((plan_lpt > 1).sum()),
            "max_workgroups_per_mesh": int(plan_lpt.max()),
            "note": "pcg_per_mesh=2: large meshes split over workgroups, the smallest queued; each mesh's path is "
                    "its path alone with as many workgroups"}
    except Exception as e:  # a supplementary figure: report, do not lose the line
        per_mesh["lpt_plan"] = {"error": f"{type(e).__name__}: {e}"}
    gb.set_params(pcg_per_mesh=0, pcg_blocks=grid)
    out = {"value": round(value, 1), "unit": "tet-iterations/s", "ms_per_step": round(ms, 3),
           "note": "converged meshes only: sum over meshes that reached 1e-6 of T_i x their iterations, over the "
                   "batch's time",
           "meshes": n_mesh, "tets": int(Ts.sum()), "chambers": int(sum(w.n_chambers for w in wls)),
           "max_iter": max_iter, "outer_iters": st["iters"], "pcg_iters": st["pcg_iters_total"], "pcg_grid": grid,
           "converged_meshes": int(conv.sum()), "capped_meshes": int((~conv).sum()),
           "capped_tet_iterations": capped_work, "aa_rejected": st["aa_rejected"],
           "plain_sample": {"meshes": len(idx), "value": round(rate_plain, 1) if rate_plain else None,
                            "unit": "tet-iterations/s",
                            "note": "each sampled mesh solved alone (same settings), converged ones counted"},
           "speedup_vs_alone": round(value / rate_plain, 3) if rate_plain else None,
           "per_mesh_cg": per_mesh,
           "roofline": roof, "kernels": kernel_table(prof)}
    gb.close()
    return out


def run_adjoint(G, mg, wl, gp, x, alpha, t_solve_ms, reps=3):
    """Implicit adjoint at the converged solve left in gp (positions x)."""
    import torch
    verts, y = mg.adjoint_targets(wl) if wl.name == "gripper" else mg.finger_tip_targets(wl)
    xs = x.double().cpu().numpy()
    g = np.zeros((3, wl.n_verts))
    g[:, verts] = 2.0 * (xs[:, verts] - y.T)
    gt = gp.tensor(g)
    ga, st = gp.adjoint(gt)                                   # warm-up
    torch.cuda.synchronize()
    print(f"# adjoint warm-up: {st}", file=sys.stderr, flush=True)
    times = []
    for _ in range(reps):
        ms, (ga, st) = timed_on(gp.stream, lambda: gp.adjoint(gt))
        times.append(ms)
        print(f"# adjoint: {ms:.1f} ms {st}", file=sys.stderr, flush=True)
    gp.profile(True)
    gp.adjoint(gt)
    prof = gp.profile_read()
    gp.profile(False)
    t = float(np.median(times))
    fd_ms = 2 * wl.n_chambers * t_solve_ms
    return {"value": round(1e3 / t, 3), "unit": "gradients/s", "ms_per_gradient": round(t, 3),
            "params": wl.n_chambers, "adjoint_iters": st["iters"], "pcg_iters": st["pcg_iters_total"],
            "residual": st["residual"], "status": st["status"], "anderson_memory": gp.params.adj_aa_m,
            "loss": f"sum of squared distances of {len(verts)} fingertip vertices to seeded targets",
            "forward_plus_adjoint_ms": round(t_solve_ms + t, 3),
            "fd_plain_ms": round(fd_ms, 3), "speedup_vs_fd": round(fd_ms / t, 2),
            "grad_norm": float(torch.linalg.norm(ga.double()).item()),
            "kernels": {k: v for k, v in kernel_table(prof).items() if k.startswith("adj_")}}


def run_coarse(G, wl, grid, iters):
    """The first `iters` outer iterations of the workload from rest on the
    headline's CG grid, with the Jacobi and with the coarse-corrected CG
    preconditioner (same solver settings otherwise): CG iterations and
    tet-iterations/s.  A fixed iteration count, not a converged solve (see the
    design notes on the gripper's path-fragile convergence)."""
    res = {"outer_iterations": iters, "pcg_grid": grid}
    for cz in (0, 1):
        with G.Problem.from_workload(wl, precision=wl.precision, pcg_blocks=grid, fixed_iters=iters,
                                     pcg_coarse=cz) as p:
            xa, aa = p.tensor(wl.rest_xyz), p.tensor(wl.alpha)
            p.solve(aa, xa.clone())
            p.reset_contacts()
            ms, (_, st) = timed_on(p.stream, lambda: p.solve(aa, xa.clone()))
        key = "coarse" if cz else "jacobi"
        res[key] = {"ms": round(ms, 3), "pcg_iters": st["pcg_iters_total"],
                    "value": round(wl.n_tets * st["iters"] / (ms / 1e3), 1), "unit": "tet-iterations/s",
                    "residual": st["residual"]}
    res["speedup"] = round(res["jacobi"]["ms"] / res["coarse"]["ms"], 3)
    return res


def run_finger_sweep(G, mg, hs=(2.0, 1.2, 0.8, 0.6), iters=30):
    """The CG kernel's roofline against problem size: the finger (8
    chambers, alpha 2.0, self-collision, default solver settings) at voxel
    sizes hs, its first `iters` outer iterations from rest on the autotuned
    CG grid.  Per size: the time per outer iteration, and the CG kernel's
    average launch time from per-kernel HIP events in a second run with its
    fraction of HBM peak by B_pcg.  A fixed iteration count, not a converged
    solve."""
    out = []
    for h in hs:
        w = mg.finger(h, 8, 2.0)
        with G.Problem.from_workload(w, precision=4, fixed_iters=iters) as p:
            a = p.tensor(w.alpha)
            x0 = p.tensor(w.rest_xyz)
            grid = p.autotune(a, x0.clone(), iters=min(iters, 8))[0]

            def run():
                p.reset_contacts()
                return p.solve(a, x0.clone())[1]

            run()
            ms, st = timed_on(p.stream, run)
            p.profile(True)
            st_p = run()
            prof = p.profile_read()
            p.profile(False)
            roof = roofline_of(prof, p.info, 4, st_p["pcg_iters_total"])
            out.append({"h_mm": h, "tets": w.n_tets, "verts": w.n_verts, "nnz": p.info["nnz"], "pcg_grid": grid,
                        "ms_per_outer_iteration": round(ms / st["iters"], 4),
                        "tet_iterations_per_s": round(w.n_tets * st["iters"] / (ms / 1e3), 1),
                        "cg_iterations_per_launch": roof["cg_iterations_per_launch"],
                        "cg_launch_us": roof["avg_launch_us"],
                        "us_per_cg_iteration": round(roof["avg_launch_us"] / roof["cg_iterations_per_launch"], 3),
                        "achieved_GBs": roof["achieved"], "frac": roof["frac"]})
    return {"outer_iterations": iters, "sizes": out}


def run_stream_copy(mib=2048, reps=10):
    """Device-to-device copies of `mib` MiB (torch's copy kernel): bytes read
    plus bytes written per second, the bandwidth a streaming kernel reaches on
    this GPU, beside the 8 TB/s peak the roofline fractions use."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    gbs = 2 * 4 * n / (ms / 1e3) / 1e9
    del src, dst
    return {"bytes_per_copy": 2 * 4 * n, "ms_per_copy": round(ms, 4), "GBs": round(gbs, 1),
            "frac_of_peak": round(gbs / PEAK_HBM_GBS, 4), "note": "read + write bytes of a device copy"}


def run_membrane(G, mg):
    """The membrane rig (40,446 tets: four chamber units under a sheet) solved
    from rest to 1e-6: tet-iterations/s, as the headline."""
    wl = mg.make("membrane")
    with G.Problem.from_workload(wl, precision=wl.precision) as p:
        xa, aa = p.tensor(wl.rest_xyz), p.tensor(wl.alpha)
        p.solve(aa, xa.clone())
        p.reset_contacts()
        ms, (_, st) = timed_on(p.stream, lambda: p.solve(aa, xa.clone()))
    return {"tets": wl.n_tets, "ms": round(ms, 3), "iters": st["iters"], "pcg_iters": st["pcg_iters_total"],
            "converged": st["status"] == G.OK, "residual": st["residual"], "contacts": st["n_contacts"],
            "value": round(wl.n_tets * st["iters"] / (ms / 1e3), 1), "unit": "tet-iterations/s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="gripper")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-meshes", type=int, default=256)
    ap.add_argument("--batched-max-iter", type=int, default=1000)
    ap.add_argument("--plain-sample", type=int, default=8)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-legs", action="store_true", help="skip the coarse-correction, membrane and finger size-sweep legs")
    ap.add_argument("--coarse-iters", type=int, default=200)
    ap.add_argument("--adjoint-max-iter", type=int, default=600)
    ap.add_argument("--no-autotune", action="store_true", help="keep the default CG grid (counter runs)")
    ap.add_argument("--pcg-blocks", type=int, default=0, help="CG grid for the headline solve (no autotune)")
    ap.add_argument("--max-iter", type=int, default=0,
                    help="cap the headline solve's iterations (profiler and counter runs only)")
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
    extra = {}
    if a.pcg_blocks:
        extra["pcg_blocks"] = a.pcg_blocks
    if a.max_iter:
        extra["max_iter"] = a.max_iter
    gp = G.Problem.from_workload(wl, precision=wl.precision, **extra)
    W = wl.precision
    x0 = gp.tensor(wl.rest_xyz)
    alpha = gp.tensor(wl.alpha)
    x = x0.clone()
    stream = gp.stream
    grid = gp.info["pcg_grid"] if (a.no_autotune or a.pcg_blocks) else gp.autotune(alpha, x, iters=20)[0]

    def step():
        x.copy_(x0)
        gp.reset_contacts()
        _, st = gp.solve(alpha, x)
        return st

    print(f"# warmup {a.warmup} solves of {wl.name} ({wl.n_tets} tets)", file=sys.stderr, flush=True)
    for _ in range(a.warmup):
        st = step()
        print(f"# warmup: {st}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    stats = []

    def timed_steps():
        for i in range(a.steps):
            stats.append(step())
            print(f"# step {i}: {stats[-1]}", file=sys.stderr, flush=True)

    t_host = time.perf_counter()
    ms, _ = timed_on(stream, timed_steps)
    t_host = time.perf_counter() - t_host
    if any(s["status"] != G.OK for s in stats):
        print("# a timed solve did not converge", file=sys.stderr, flush=True)

    # the same solve once more with per-kernel events (kernel table, roofline)
    gp.profile(True)
    x.copy_(x0)
    gp.reset_contacts()
    _, pst = gp.solve(alpha, x)
    torch.cuda.synchronize()
    prof = gp.profile_read()
    gp.profile(False)

    iters = sum(s["iters"] for s in stats)
    pcg_iters = sum(s["pcg_iters_total"] for s in stats)
    value = wl.n_tets * iters / (ms / 1e3)
    roof = roofline_of(prof, gp.info, W, pst["pcg_iters_total"], (wl.name, grid))
    solver = {k: getattr(gp.params, k) for k in ("aa_m", "aa_guard", "aa_slack", "pcg_eta", "pcg_eta_min",
                                                   "pcg_max", "tol")}
    out = {
        "metric": "tet-iterations/sec to 1e-6 residual (plain vs batched; adjoint grads/sec)",
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
                               f"self-collision {'on' if wl.self_collision else 'off'}, obstacles "
                               f"{'on' if wl.obstacle_collision else 'off'}, one solve from rest to 1e-6",
                   "tets": wl.n_tets, "outer_iters_per_step": iters / a.steps,
                   "pcg_iters_per_step": pcg_iters / a.steps, "pcg_grid": grid,
                   "converged_steps": sum(1 for s in stats if s["status"] == G.OK),
                   "aa_rejected_per_step": sum(s["aa_rejected"] for s in stats) / a.steps,
                   "contacts": stats[-1]["n_contacts"], "residual": stats[-1]["residual"], "solver": solver},
        "roofline": roof,
        "kernels": kernel_table(prof),
        "host_s": round(t_host, 3),
    }
    if not a.no_adjoint:
        print("# adjoint", file=sys.stderr, flush=True)
        x.copy_(x0)
        gp.reset_contacts()
        xs, sst = gp.solve(alpha, x)
        gp.set_params(adj_max_iter=a.adjoint_max_iter)
        out["adjoint"] = run_adjoint(G, mg, wl, gp, xs, alpha, ms / a.steps)
        if out["adjoint"]["status"] != G.OK:
            out["adjoint"]["note"] = ("not converged within the iteration cap: the gripper's fixed point is "
                                      "ill-conditioned (see the condition estimate in the design notes), and so "
                                      "is its adjoint system")
    gp.close()
    if not a.no_adjoint and a.workload != "finger":
        # the converged finger (26,880 tets, 8 chambers, 10 fingertip targets)
        fw = mg.make("finger")
        with G.Problem.from_workload(fw, precision=4) as fp:
            fa = fp.tensor(fw.alpha)
            fx = fp.tensor(fw.rest_xyz)
            fp.solve(fa, fx.clone())
            fp.reset_contacts()
            ms_f, (xf, _) = timed_on(fp.stream, lambda: fp.solve(fa, fx.clone()))
            out["adjoint_finger"] = run_adjoint(G, mg, fw, fp, xf, fa, ms_f)
    if not a.no_legs and a.workload == "gripper":
        print("# coarse correction, fixed iterations", file=sys.stderr, flush=True)
        out["coarse"] = run_coarse(G, wl, grid, a.coarse_iters)
        print("# membrane", file=sys.stderr, flush=True)
        out["membrane"] = run_membrane(G, mg)
        print("# finger size sweep", file=sys.stderr, flush=True)
        try:
            out["finger_sweep"] = run_finger_sweep(G, mg)
        except Exception as e:  # a supplementary leg: report, do not lose the line
            out["finger_sweep"] = {"error": f"{type(e).__name__}: {e}"}
    if not a.no_batched:
        out["batched"] = run_batched(G, mg, a.batched_meshes, a.batched_max_iter, a.plain_sample,
                                     autotune=not a.no_autotune)
    try:
        out["stream_copy"] = run_stream_copy()
    except Exception as e:  # a supplementary figure: report, do not lose the line
        out["stream_copy"] = {"error": f"{type(e).__name__}: {e}"}
    if not a.no_cpu_baseline:
        print("# cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = run_cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

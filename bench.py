#!/usr/bin/env python3
"""Throughput of the PP-PC periodic steady-state solver on one MI355X.

One step = one complete periodic steady state: PP-PC from its initial iterate until
eps = ||J||_F/||U||_F <= tol, every fine sweep, jump, linearisation, DFT, harmonic COCG
solve and inverse DFT on the GPU, with the problem already resident in HBM.  The
workload is the nonlinear coax (nr = 60 x ntheta = 120, 7,081 free nodes, steel
sheath with a Brauer B-H law, N = 40 subintervals x 50 implicit-Euler steps,
21 harmonic systems, FP64) with synthetic seeded inputs.

Prints one JSON line: steady states per second, the roofline of the dominant kernel
(the fine sweep) from its measured launch durations and algorithmic bytes, the error
against the stored FP64 oracle fixed point, and the CPU oracle timed on a bounded
sample as a baseline.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp64|mixed|mixed-fine]

--workload c4reg times batched designs instead (designs' steady states per second; starting
from rest with the coarse-correction safeguard at 3 T, which these thin, strongly driven
sheaths need).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
COUNTERS = os.path.join(ROOT, "profiles", "fine_sweep_c2_fp64_counters.md")
# the fine-sweep kernel's device code and the host code that picks its shape
FINE_SRC = [os.path.join(ROOT, "paper_1905_13076_amd", "csrc", f) for f in ("fine_chain.hpp", "fine.hip")]


def measured_traffic(tol_newton):
    """HBM bytes per fine-sweep launch from the committed counter summary, if it was
    taken on the current fine-sweep source at this Newton tolerance (else None)."""
    import hashlib
    import re
    if not os.path.exists(COUNTERS):
        return None
    text = open(COUNTERS).read()
    m = re.search(r"fine-sweep sources sha1 \(fine_chain.hpp \+ fine.hip\): ([0-9a-f]{40})", text)
    t = re.search(r"traffic_bytes_per_launch: (\d+)", text)
    g = re.search(r"algorithmic_bytes_per_launch: (\d+)", text)
    if not (m and t and g):
        return None
    if hashlib.sha1(b"".join(open(f, "rb").read() for f in FINE_SRC)).hexdigest() != m.group(1):
        return None
    tn = re.search(r"tol_newton: ([0-9.eE+-]+)", text)
    if not tn or float(tn.group(1)) != tol_newton:
        return None
    return {"bytes": int(t.group(1)), "algorithmic_bytes_same_launch": int(g.group(1))}


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c2lin", "c5small", "c4reg"],
                    help="c4reg: the batched-designs generator's designs with nr <= 66 among its "
                         "first 64 (21 designs, full 40 x 50 grid), one batched solve per step; "
                         "c2lin: C2 with the steel linearised at its unsaturated reluctivity")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed", "mixed-fine"])
    ap.add_argument("--method", default="ppc", choices=["ppc", "ppic", "seq"],
                    help="ppc: PP-PC, eq. (4) with the periodic coarse problem; ppic: PP-IC, "
                         "eq. (5), U_0^{k+1} = U_N^k with sequential coarse propagation; seq: "
                         "classical time stepping from zero, one chain of the fine kernel per "
                         "period, until two periods' samples agree to --tol")
    ap.add_argument("--coarse", default="frozen", choices=["frozen", "nonlinear"],
                    help="PP-PC coarse problem: frozen (time-averaged linearisation, one harmonic "
                         "solve per correction) or nonlinear (eq. (4) with the implicit-Euler "
                         "coarse step on the full K(u), Newton with GMRES preconditioned by the "
                         "frozen solve)")
    ap.add_argument("--n-harm", type=int, default=0,
                    help="harmonics each PP-PC correction solves (0: all N/2+1); the others "
                         "take the jumps' harmonics")
    ap.add_argument("--init", default="nested", choices=["nested", "auto", "rest"],
                    help="U^0: nested (PP-PC on a 25 times coarser fine grid to eps <= 1e-2, "
                         "the default), auto (zero for nonlinear, coarse periodic for linear) or "
                         "rest (one fine sweep from zero, U^0_n = F_n(0))")
    ap.add_argument("--tol", type=float, default=1e-7,
                    help="PP-PC stopping tolerance on eps (the metric asks for 1e-6 relative error "
                         "against the FP64 oracle; 1e-7 reaches 6.8e-8 on C2)")
    ap.add_argument("--tol-newton", type=float, default=1e-10,
                    help="Newton stopping tolerance of the fine steps, relative to ||f(t)|| + "
                         "||M u_prev||/dt (the oracle uses 1e-13; on C2 the PP-PC error against it "
                         "does not change between 1e-13 and 1e-9)")
    ap.add_argument("--tol-cocg", type=float, default=1e-6,
                    help="relative tolerance of the harmonic solves (a correction only needs to be "
                         "accurate relative to the current jumps)")
    ap.add_argument("--autotune", dest="autotune", action="store_true", default=True,
                    help="tune the fine-sweep workgroup size before timing (untimed set-up)")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false")
    ap.add_argument("--cpu-baseline", dest="cpu", action="store_true", default=True)
    ap.add_argument("--no-cpu-baseline", dest="cpu", action="store_false")
    ap.add_argument("--cpu-procs", type=int, default=16)
    ap.add_argument("--probe", choices=["fine"], default=None,
                    help="counter-collection mode: a 512 MiB device copy of known size (the "
                         "calibration kernel) and one fine sweep from the oracle fixed point")
    return ap.parse_args()


def workload(name):
    from workloads import coax
    return {"c1": coax.c1, "c2": coax.c2, "c2lin": coax.c2lin, "c5small": coax.c5_small}[name]()


def load_reference(name):
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", f"{name}_oracle.npz")
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        return {"U": z["U"], "iterations": int(z["iterations"]), "free": z["free"], "hist": z["hist"]}


def cpu_baseline(prob, ref, procs, tol):
    """The oracle as it stands (scipy direct solves, FP64, Newton to 1e-13) on the host
    cores, on a bounded sample: two fine sweeps of all N chains from the oracle fixed point
    (one chain per worker process) and two coarse corrections, ~15 s of work at C2;
    extrapolated to the sweeps and corrections the oracle's own PP-PC takes to reach eps <=
    tol (its stored eps history), for one steady state."""
    import numpy as np
    from oracle import periodic
    from oracle.fe import FE
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    cores = max(1, min(procs, len(os.sched_getaffinity(0)), prob.N))
    fe = FE(prob)
    U = ref["U"]
    hist = ref["hist"]
    iters = next(k for k in range(len(hist)) if hist[k] <= tol) if np.any(hist <= tol) else int(ref["iterations"])
    dt = periodic.fine_dt(prob)
    args = [((n - 1) * (prob.T / prob.N), U[n - 1], prob.m, dt, 1e-13) for n in range(1, prob.N + 1)]
    pool = periodic.make_pool(prob, cores)
    reps = 2
    try:
        pool.starmap(periodic._chain_worker, args[:cores])      # warm the workers' imports
        t0 = time.perf_counter()
        for _ in range(reps):
            outs = pool.starmap(periodic._chain_worker, args)
        t_sweep = (time.perf_counter() - t0) / reps
    finally:
        pool.close()
        pool.join()
    J = np.zeros_like(U)
    for n in range(1, prob.N + 1):
        J[n % prob.N] = outs[n - 1] - U[n % prob.N]
    t0 = time.perf_counter()
    for _ in range(reps):
        periodic.coarse_correction(fe, U, J)
    t_coarse = (time.perf_counter() - t0) / reps
    t_state = (iters + 1) * t_sweep + iters * t_coarse
    return {
        "value": 1.0 / t_state,
        "unit": "steady states/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"{reps} fine sweeps of all {prob.N} chains ({prob.m} steps each, {cores} processes) at "
                   f"{t_sweep:.2f} s each + {reps} coarse corrections at {t_coarse:.2f} s each; extrapolated "
                   f"to the oracle's {iters + 1} sweeps + {iters} corrections to eps <= {tol:g} = "
                   f"{t_state:.1f} s per steady state"),
    }


def probe_fine(a, prob, ref):
    """One device copy of known size, then one warm-up and one measured fine sweep
    (all N chains, one launch) started from the oracle fixed point."""
    import numpy as np
    import torch
    import paper_1905_13076_amd as P
    from paper_1905_13076_amd.traffic import fine_sweep_bytes
    torch.cuda.set_device(0)
    src = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")   # 512 MiB
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    h = P.Handle(0)
    pr = P.Problem(h, prob)
    prec = 0 if a.precision == "fp64" else 1
    prm = P.problem_params(prob, precision=prec, tol_newton=a.tol_newton,
                           **({"tol_lin": 1e-4} if prec == 1 else {}))
    U = np.zeros((prob.N, pr.n_nodes))
    U[:, ref["free"]] = ref["U"]
    Ud = torch.tensor(U, device="cuda")
    pr.fine_sweep(prm, Ud)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    F, newton, lin = pr.fine_sweep(prm, Ud)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    cnt = pr.fine_counts(prob.N)
    tot = {"lin_total": int(cnt[:, 2].sum()), "newton_total": int(cnt[:, 1].sum()),
           "resid_total": int(cnt[:, 7].sum()), "steps_total": prob.N * prob.m, "fine_launches": 1,
           "n_free": pr.n_free, "nnz": pr.nnz, "n_tri": pr.n_tri}
    print(json.dumps({"probe": "fine", "tol_newton": a.tol_newton, "copy_bytes_each_way": src.numel() * 8,
                      "sweep_ms": dt * 1e3,
                      "newton_total": tot["newton_total"], "lin_total": tot["lin_total"],
                      "resid_total": tot["resid_total"],
                      "algorithmic_bytes": fine_sweep_bytes(tot, prob.N, prec)}), flush=True)
    return 0


def batch_designs():
    from workloads import coax
    return [p for p in coax.c4_designs(n_designs=64) if p.meta["nr"] <= 66]


def bench_batch(a):
    """Batched designs: every step is one batched PP-PC solve of all designs; value =
    designs' steady states per second.  The roofline fields are left null: the batched
    launches mix design sizes, so no single per-launch byte count describes them."""
    import numpy as np
    import torch
    import paper_1905_13076_amd as P
    torch.cuda.set_device(0)
    designs = batch_designs()
    h = P.Handle(0)
    bp = P.BatchProblem(h, designs)
    prec = 0 if a.precision == "fp64" else 1
    extra = {"tol_lin": 1e-4} if prec == 1 else {}
    if a.precision == "mixed-fine":
        extra["coarse_precision"] = 0
    prm = P.problem_params(designs[0], tol_ppc=a.tol, precision=prec, tol_cocg=a.tol_cocg, max_newton=200,
                           tol_newton=a.tol_newton,
                           init_mode=4 if a.init == "nested" else 3, b_cap=3.0, **extra)
    tuned = None
    if a.autotune:
        # untimed set-up: the fine-sweep workgroup size per size class
        t0 = time.perf_counter()
        blocks, _ = bp.autotune(prm)
        tuned = {"seconds": time.perf_counter() - t0,
                 "designs_per_block": {str(b): int(np.sum(blocks == b)) for b in (256, 512, 1024)}}
    for _ in range(a.warmup):
        bp.solve(prm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        Us, resid, iters, st, rc = bp.solve(prm)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if rc != 0:
        print(json.dumps({"error": f"solve status {rc}", "stats": st}))
        return 1
    nrs = [p.meta["nr"] for p in designs]
    print(json.dumps({
        "metric": "periodic steady states/s at 1e-6 rel. err vs FP64 oracle; achieved HBM GB/s",
        "value": a.steps * len(designs) / wall,
        "unit": "design steady states/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": 1e3 * wall / a.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == 0 else "f32+f64", "data": "synthetic",
        "config": {"workload": f"batched designs: {len(designs)} designs, nr {min(nrs)}-{max(nrs)} "
                               f"(ntheta = 2 nr), N=40 x m=50, 21 harmonics each; b_cap 3 T",
                   "init": "nested (from rest on the coarser grid)" if a.init == "nested" else "from rest",
                   "precision": a.precision, "tol_ppc": a.tol, "tol_cocg": a.tol_cocg,
                   "tol_newton": a.tol_newton,
                   "iterations_max": int(max(iters)), "damped_corrections": st["damped"],
                   "fine_ms_per_step": st["fine_ms"], "coarse_ms_per_step": st["coarse_ms"],
                   "newton_per_step": st["newton_total"] / max(1, st["steps_total"]),
                   "autotune": tuned},
        "roofline": None, "cpu_baseline": None}))
    return 0


def bench_time_stepping(a):
    """Classical time stepping on the same GPU: one steady state = periods stepped from zero
    until two periods' samples agree to --tol; progress (one line per call of a few
    periods) on stderr."""
    import numpy as np
    import torch
    import paper_1905_13076_amd as P
    torch.cuda.set_device(0)
    prob = workload(a.workload)
    ref = load_reference(a.workload)
    h = P.Handle(0)
    pr = P.Problem(h, prob)
    prec = 0 if a.precision == "fp64" else 1
    chunk = 4
    prm = P.problem_params(prob, tol_ppc=a.tol, precision=prec, max_iters=chunk, tol_newton=a.tol_newton,
                           **({"tol_lin": 1e-4} if prec == 1 else {}))
    walls, periods_all, fine_ms = [], [], 0.0
    for step in range(a.warmup + a.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        total, u0, Up, newton, steps = 0, None, None, 0, 0
        while True:
            U, per, st, rc = pr.time_stepping(prm, u_start=u0, U_prev=Up)
            total += per
            newton += st["newton_total"]
            steps += st["steps_total"]
            if step >= a.warmup:
                fine_ms += st["fine_ms"]
            print(f"[seq] step {step} periods {total} change {st['eps']:.3e}", file=sys.stderr, flush=True)
            if rc == 0 or total >= 2000:
                break
            Up, u0 = U, U[0].contiguous()
        torch.cuda.synchronize()
        if step >= a.warmup:
            walls.append(time.perf_counter() - t0)
            periods_all.append(total)
    if rc != 0:
        print(json.dumps({"error": f"time stepping did not reach a periodic state in {total} periods"}))
        return 1
    err = None
    if ref is not None:
        Ug = U.cpu().numpy()[:, ref["free"]]
        err = float(np.linalg.norm(Ug - ref["U"]) / np.linalg.norm(ref["U"]))
    wall = sum(walls)
    print(json.dumps({
        "metric": "periodic steady states/s at 1e-6 rel. err vs FP64 oracle; achieved HBM GB/s",
        "value": a.steps / wall, "unit": "steady states/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": 1e3 * wall / a.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if prec == 0 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{prob.name}: nr={prob.meta['nr']} x ntheta={prob.meta['ntheta']}, "
                               f"T = {prob.T}, {prob.N * prob.m} steps per period",
                   "method": "classical time stepping (one chain per period)", "precision": a.precision,
                   "tol": a.tol, "periods": periods_all[-1], "err_vs_oracle": err,
                   "newton_per_step": newton / max(1, steps), "fine_ms_per_state": fine_ms / a.steps},
        "roofline": None, "cpu_baseline": None}), flush=True)
    return 0


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU: the path has no collectives; "
                                   "run with --gpus 1"}))
        return 2
    if a.workload == "c4reg":
        return bench_batch(a)
    if a.method == "seq":
        return bench_time_stepping(a)
    prob = workload(a.workload)
    ref = load_reference(a.workload)
    if a.probe == "fine":
        return probe_fine(a, prob, ref)
    cpu = None
    if a.cpu and ref is not None and a.method == "ppc" and a.n_harm == 0 and a.coarse == "frozen":
        # before any GPU initialisation: the oracle's worker pool forks this process
        cpu = cpu_baseline(prob, ref, a.cpu_procs, a.tol)
    import numpy as np
    import torch
    import paper_1905_13076_amd as P
    from paper_1905_13076_amd.traffic import fine_sweep_bytes

    torch.cuda.set_device(0)
    h = P.Handle(0)
    t0 = time.perf_counter()
    pr = P.Problem(h, prob)
    setup_s = time.perf_counter() - t0
    prec = 0 if a.precision == "fp64" else 1
    extra = {"tol_lin": 1e-4} if prec == 1 else {}
    if a.precision == "mixed-fine":          # FP32 PCG fine solves, FP64 harmonic solves
        extra["coarse_precision"] = 0
    extra["method"] = 1 if a.method == "ppic" else 0
    extra["init_mode"] = {"auto": 0, "rest": 3, "nested": 4}[a.init]
    extra["n_harm"] = a.n_harm
    extra["coarse_mode"] = 1 if a.coarse == "nonlinear" else 0
    if a.n_harm:
        extra["max_iters"] = 300
    if a.method == "ppic":
        extra["max_iters"] = 300
    prm = P.problem_params(prob, tol_ppc=a.tol, precision=prec, tol_cocg=a.tol_cocg, tol_newton=a.tol_newton,
                           **extra)
    tuned = None
    if a.autotune:
        t0 = time.perf_counter()
        b, ms = pr.autotune(prm)
        tuned = {"seconds": time.perf_counter() - t0, "block": b,
                 "sweep_ms": {str(k): (None if np.isnan(v) else float(v)) for k, v in zip((256, 512, 1024), ms)}}
    out = torch.empty((prob.N, pr.n_nodes), dtype=torch.float64, device="cuda")
    for _ in range(a.warmup):
        pr.solve(prm, out=out)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(a.steps):
        U, eps, k, st, rc = pr.solve(prm, out=out)
        stats.append(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if rc != 0:
        print(json.dumps({"error": f"solve status {rc}", "stats": st}))
        return 1
    # error against the stored FP64 oracle fixed point
    err = None
    if ref is not None:
        Ug = U.cpu().numpy()[:, ref["free"]]
        err = float(np.linalg.norm(Ug - ref["U"]) / np.linalg.norm(ref["U"]))
    fine_ms = sum(s["fine_ms"] for s in stats)
    launches = sum(s["fine_launches"] for s in stats)
    tot = {k2: sum(s[k2] for s in stats) for k2 in ("lin_total", "resid_total", "newton_total",
                                                     "steps_total", "fine_launches")}
    tot.update(n_free=st["n_free"], nnz=st["nnz"], n_tri=st["n_tri"])
    bytes_launch = fine_sweep_bytes(tot, prob.N, prec) / launches
    launch_s = fine_ms / launches / 1e3
    achieved = bytes_launch / launch_s / 1e9
    value = a.steps / wall
    traffic = measured_traffic(a.tol_newton) if prec == 0 else None
    line = {
        "metric": "periodic steady states/s at 1e-6 rel. err vs FP64 oracle; achieved HBM GB/s",
        "value": value,
        "unit": "steady states/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * wall / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == 0 else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": f"{prob.name}: nr={prob.meta['nr']} x ntheta={prob.meta['ntheta']} "
                        f"({st['n_free']} free nodes, {st['nnz']} nnz), N={prob.N} x m={prob.m}, "
                        f"{prob.N // 2 + 1} harmonics, amplitude {prob.amps[0]:.1f} A",
            "precision": a.precision,
            "method": a.method,
            "harmonics_solved": a.n_harm or prob.N // 2 + 1,
            "coarse": a.coarse,
            "init": a.init,
            "tol_ppc": a.tol,
            "tol_cocg": a.tol_cocg,
            "tol_newton": a.tol_newton,
            "iterations": k,
            "err_vs_oracle": err,
            "max_b_steel_T": st["max_b_steel"],
            "newton_per_step": tot["newton_total"] / max(1, tot["steps_total"]),
            "pcg_per_newton": tot["lin_total"] / max(1, tot["newton_total"]),
            "cocg_total_per_state": sum(s["cocg_total"] for s in stats) / a.steps,
            "coarse_solves_per_state": sum(s["coarse_solves"] for s in stats) / a.steps,
            "coarse_newton_per_state": sum(s["coarse_newton"] for s in stats) / a.steps,
            "coarse_ms_per_state": sum(s["coarse_ms"] for s in stats) / a.steps,
            "fine_ms_per_state": fine_ms / a.steps,
            "coarse_ms_per_state": sum(s["coarse_ms"] for s in stats) / a.steps,
            "setup_s": setup_s,
            "autotune": tuned,
        },
        "roofline": {
            "kernel": "k_fine_sweep",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": (traffic or {}).get("bytes"),
            "traffic_source": ("rocprofv3 FETCH_SIZE+WRITE_SIZE (copy-calibrated) of one C2 fine sweep "
                               "(50 steps per chain) from the oracle fixed point, "
                               "profiles/fine_sweep_c2_fp64_counters.md; algorithmic bytes of that launch "
                               f"{traffic['algorithmic_bytes_same_launch']} (the timed launches also "
                               "include the nested start's 2-step sweeps)")
                              if traffic else None,
            "bytes_per_launch": bytes_launch,
            "launch_ms": launch_s * 1e3,
            "launches": launches,
        },
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

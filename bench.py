#!/usr/bin/env python3
"""Throughput of the PP-PC periodic steady-state solver on one MI355X.

One step = one complete periodic steady state: PP-PC from its initial iterate until
eps = ||J||_F/||U||_F <= tol, every fine sweep, jump, linearisation, DFT, harmonic COCG
solve and inverse DFT on the GPU, with the problem already resident in HBM.  The
workload is the nonlinear coax (nr = 60 x ntheta = 120, 7,081 free nodes, steel
sheath with a Brauer B-H law, N = 40 subintervals x 50 implicit-Euler steps,
21 harmonic systems, FP64) with synthetic seeded inputs, at tolerances that keep the error
against the FP64 oracle under the metric's 1e-6: PP-PC to eps <= 1e-7, Newton to 1e-10 of
each step's scale with the adaptive fine tolerance (theta = 1e-3: early sweeps solve only to
theta eps of the previous iteration, the late ones to 1e-10), harmonic solves to 1e-6.

Prints one JSON line: steady states per second, the roofline of the dominant kernel
(the fine sweep) from its measured launch durations and algorithmic bytes, the error
against the stored FP64 oracle fixed point, and the CPU oracle timed on a bounded
sample as a baseline.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp64|mixed|mixed-fine]

--workload c4reg times batched designs instead (designs' steady states per second; starting
from rest with the coarse-correction safeguard at 3 T, which these thin, strongly driven
sheaths need).

The default workload is the nonlinear coax above because one of its steady states takes
under a second.  The two larger configurations do not fit a run of minutes: a steady state of
the large coax (nr = 400, 319,201 free nodes, N = 200 x 100, 101 harmonics) takes about
35-40 minutes and one batched solve of the 256 designs about 30 minutes on one MI355X, by
their measured per-iteration costs.  `--workload c3` still runs whole steady states of the
large coax (mixed against an FP64 GPU reference, progress on stderr); `--probe fine
--workload c3|c4` times and profiles one fine sweep of either at its full size.
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
# periods classical time stepping takes from zero to a periodic state at the bench tolerance
# (measured with the GPU's time stepping, bench.py --method seq)
SEQ_PERIODS = {"c1": 3, "c5small": 3, "c2": 3, "c2lin": 40}
COUNTERS = os.path.join(ROOT, "profiles", "fine_sweep_c2_fp64_counters.md")
# the fine-sweep kernel's device code and the host code that picks its shape
FINE_SRC = [os.path.join(ROOT, "paper_1905_13076_amd", "csrc", f) for f in ("fine_chain.hpp", "fine.hip")]


def measured_traffic(tol_newton, path=COUNTERS, tol_adapt=0.0):
    """HBM bytes per fine-sweep launch from a committed counter summary, if it was taken on
    the current fine-sweep source at this Newton tolerance and adaptive-tolerance setting
    (a summary without a tol_adapt line was taken at the fixed tolerance), else None."""
    import hashlib
    import re
    if not os.path.exists(path):
        return None
    text = open(path).read()
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
    ta = re.search(r"tol_adapt: ([0-9.eE+-]+)", text)
    if (float(ta.group(1)) if ta else 0.0) != tol_adapt:
        return None
    lm = re.search(r"launch_ms: ([0-9.eE+-]+)", text)
    return {"bytes": int(t.group(1)), "algorithmic_bytes_same_launch": int(g.group(1)),
            "launch_ms": float(lm.group(1)) if lm else None}


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c2lin", "c5small", "c4reg", "c3", "c4"],
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
    ap.add_argument("--lin-start", type=int, default=0, choices=[0, 1, 2],
                    help="start of each fine-step PCG: 2 Galerkin projection on the last Newton "
                         "corrections, 1 zero, 0 (default) Galerkin with FP64 PCG, zero with FP32")
    ap.add_argument("--tol-adapt", type=float, default=1e-3,
                    help="theta of the adaptive fine tolerance: the sweep of iteration k solves its "
                         "Newton steps to max(tol_newton, min(1e-6, theta eps_{k-1})); 0 = every "
                         "sweep at tol_newton (on C2 1e-3 leaves the error against the oracle at "
                         "3.6e-8 against 3.1e-8)")
    ap.add_argument("--probe-m", type=int, default=4,
                    help="probe mode on c3 / c4: fine steps per chain of the probed sweep")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="copy 512 MiB device-to-device before the solves (untimed): the kernel of "
                         "known size that scales rocprofv3's FETCH_SIZE / WRITE_SIZE of the same run")
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


def host_info():
    """Host cores the CPU baseline runs on: nproc, the affinity set and the CPU model."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "model": model}


def cpu_sample(prob, ref, procs, tol_newton, seq_steps=100):
    """The oracle as it stands (scipy direct solves, FP64) timed on the host, on a bounded
    sample at the GPU's Newton tolerance, before any GPU initialisation (the worker pool
    forks this process):
      route P (the paper's parallelism): one fine sweep of all N chains from the oracle
        fixed point, one chain per worker process over the host cores, and one coarse
        correction;
      route S (classical time stepping, one core): seq_steps implicit-Euler steps of one
        chain.
    Returns the raw timings; cpu_extrapolate turns them into steady states per second."""
    import numpy as np
    from oracle import periodic
    from oracle.fe import FE
    from oracle.timestep import fine_propagate
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    cores = max(1, min(procs, len(os.sched_getaffinity(0)), prob.N))
    fe = FE(prob)
    U = ref["U"]
    dt = periodic.fine_dt(prob)
    args = [((n - 1) * (prob.T / prob.N), U[n - 1], prob.m, dt, tol_newton) for n in range(1, prob.N + 1)]
    pool = periodic.make_pool(prob, cores)
    try:
        pool.starmap(periodic._chain_worker, args[:cores])      # warm the workers' imports
        t0 = time.perf_counter()
        outs = pool.starmap(periodic._chain_worker, args)
        t_sweep = time.perf_counter() - t0
    finally:
        pool.close()
        pool.join()
    J = np.zeros_like(U)
    for n in range(1, prob.N + 1):
        J[n % prob.N] = outs[n - 1] - U[n % prob.N]
    t0 = time.perf_counter()
    periodic.coarse_correction(fe, U, J)
    t_coarse = time.perf_counter() - t0
    steps = min(seq_steps, prob.N * prob.m)
    t0 = time.perf_counter()
    fine_propagate(fe, U[0], 0.0, steps, dt, tol=tol_newton)
    t_step = (time.perf_counter() - t0) / steps
    return {"cores": cores, "t_sweep": t_sweep, "t_coarse": t_coarse, "t_step_seq": t_step,
            "seq_steps": steps, "tol_newton": tol_newton, "host": host_info()}


def cpu_extrapolate(prob, smp, iters, nested_iters, nested_m, seq_periods):
    """Oracle seconds per steady state from the sample, with the GPU solve's own iteration
    counts (the oracle runs the same iteration: identical counts in the parity tests):
    route P = (iters + 1) sweeps + iters corrections on the real grid, plus the nested
    start's sweeps (nested_m steps per chain) and corrections; route S = seq_periods whole
    periods of N m steps on one core."""
    t_p = (iters + 1) * smp["t_sweep"] + iters * smp["t_coarse"]
    if nested_iters:
        t_p += (nested_iters + 1) * smp["t_sweep"] * nested_m / prob.m + nested_iters * smp["t_coarse"]
    t_s = seq_periods * prob.N * prob.m * smp["t_step_seq"]
    return {
        "value": 1.0 / t_p,
        "unit": "steady states/s",
        "cores": smp["cores"],
        "kind": "oracle",
        "sample": (f"route P: 1 fine sweep of all {prob.N} chains ({prob.m} steps each, {smp['cores']} "
                   f"processes, Newton to {smp['tol_newton']:g}) {smp['t_sweep']:.2f} s + 1 coarse correction "
                   f"{smp['t_coarse']:.2f} s, extrapolated to the GPU solve's {iters + 1} sweeps + {iters} "
                   f"corrections" + (f" and its nested start ({nested_iters} iterations at {nested_m} steps per "
                                     f"chain)" if nested_iters else "") + f" = {t_p:.1f} s per steady state"),
        "route_s": {"value": 1.0 / t_s, "unit": "steady states/s", "cores": 1,
                    "sample": f"{smp['seq_steps']} sequential implicit-Euler steps at "
                              f"{smp['t_step_seq'] * 1e3:.1f} ms each, extrapolated to {seq_periods} periods "
                              f"of {prob.N * prob.m} steps = {t_s:.1f} s per steady state"},
        "host": smp["host"],
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
    prm = P.problem_params(prob, precision=prec, tol_newton=a.tol_newton, lin_start=a.lin_start,
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


def free_pattern(prob, free):
    """Free nodes and the CSR entries among them (diagonal plus both directions of every
    mesh edge joining two free nodes)."""
    import numpy as np
    isfree = np.zeros(prob.xy.shape[0], dtype=bool)
    isfree[free] = True
    t = np.asarray(prob.tri)
    e = np.sort(np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [0, 2]]]), axis=1)
    e = np.unique(e, axis=0)
    return len(free), len(free) + 2 * int(np.sum(isfree[e[:, 0]] & isfree[e[:, 1]]))


def probe_large(a):
    """Counter-collection mode for the large workloads: a 512 MiB device copy of known size
    (the calibration kernel), then two identical fine sweeps (the second is the measured
    one) with --probe-m steps per chain at the workload's own step size, from the seeded
    chain starts of the parity cases: C3 (one problem, all 200 chains) or C4 (all 256
    designs in one batched sweep, 10,240 chains)."""
    import numpy as np
    import torch
    import paper_1905_13076_amd as P
    from paper_1905_13076_amd.traffic import per_unit
    from workloads import coax
    torch.cuda.set_device(0)
    src = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")   # 512 MiB
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    h = P.Handle(0)
    prec = 0 if a.precision == "fp64" else 1
    m = a.probe_m

    def free_of(prob):
        r = np.hypot(prob.xy[:, 0], prob.xy[:, 1])
        return np.flatnonzero(r < r.max() * (1 - 1e-12))      # off the outer (Dirichlet) ring

    designs = [coax.c3()] if a.workload == "c3" else coax.c4_designs()
    N = designs[0].N
    dt = designs[0].T / (N * designs[0].m)
    prm = P.params(T=N * m * dt, N=N, m=m, tol_newton=a.tol_newton, precision=prec,
                   **({"tol_lin": 1e-5} if prec else {}))
    blocks = []
    for d, prob in enumerate(designs):
        Un = np.zeros((N, prob.n_nodes))
        f = free_of(prob)
        Un[:, f] = coax.chain_starts(prob, f, seed=3 if a.workload == "c3" else 1000 + d)
        blocks.append(Un.reshape(-1))
    U = torch.tensor(np.concatenate(blocks), device="cuda")
    if a.workload == "c3":
        pr = P.Problem(h, designs[0])
        U = U.view(N, pr.n_nodes)
        sweep = lambda: pr.fine_sweep(prm, U)
    else:
        pr = P.BatchProblem(h, designs)
        sweep = lambda: pr.fine_sweep(prm, U)
    sweep()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    F, newton, lin = sweep()
    torch.cuda.synchronize()
    dt_s = time.perf_counter() - t0
    s_ = 8 if prec == 0 else 4
    newton = np.asarray(newton).reshape(len(designs), N)
    lin = np.asarray(lin).reshape(len(designs), N)
    alg = 0.0
    for d, prob in enumerate(designs):
        n, nnz = free_pattern(prob, free_of(prob))
        u = per_unit(n, nnz, prob.tri.shape[0], s_)
        alg += lin[d].sum() * u["pcg_iter"] + newton[d].sum() * u["newton_iter"]
    print(json.dumps({"probe": f"fine-{a.workload}", "precision": a.precision, "m": m, "N": N,
                      "designs": len(designs), "tol_newton": a.tol_newton,
                      "copy_bytes_each_way": src.numel() * 8, "sweep_ms": dt_s * 1e3,
                      "newton_total": int(newton.sum()), "lin_total": int(lin.sum()),
                      "algorithmic_bytes_pcg_and_newton": alg}), flush=True)
    return 0


def batch_designs():
    from workloads import coax
    return [p for p in coax.c4_designs(n_designs=64) if p.meta["nr"] <= 66]


def batch_cpu_sample(designs, tol_newton, steps=20):
    """The oracle on a bounded sample of a batch, on one core: `steps` implicit-Euler steps of
    the first chain (from rest) of the smallest, the median and the largest design, and one
    coarse correction of the largest design (from seeded samples).  A power law through the
    three step costs gives every design's step cost."""
    import numpy as np
    from oracle import periodic
    from oracle.fe import FE
    from oracle.timestep import fine_propagate
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    from workloads import coax
    order = sorted(range(len(designs)), key=lambda d: designs[d].n_nodes)
    picks = [order[0], order[len(order) // 2], order[-1]]
    n, t = [], []
    for d in picks:
        prob = designs[d]
        fe = FE(prob)
        dt = prob.T / (prob.N * prob.m)
        t0 = time.perf_counter()
        fine_propagate(fe, np.zeros(fe.n), 0.0, steps, dt, tol=tol_newton)
        t.append((time.perf_counter() - t0) / steps)
        n.append(fe.n)
    big = designs[picks[-1]]
    fe = FE(big)
    U = coax.random_rows(big.N, fe.n, seed=5, amp=2e-6)
    J = coax.random_rows(big.N, fe.n, seed=6, amp=1e-8)
    t0 = time.perf_counter()
    periodic.coarse_correction(fe, U, J)
    t_corr = time.perf_counter() - t0
    alpha = float(np.polyfit(np.log(n), np.log(t), 1)[0]) if len(set(n)) > 1 else 1.0
    return {"n": n, "t_step": t, "alpha": alpha, "t_corr_big": t_corr, "n_big": fe.n, "steps": steps,
            "host": host_info()}


def batch_cpu_extrapolate(designs, smp, iters, cores):
    """Oracle seconds for one batch: per design, (iterations + 1) sweeps of N chains x m steps
    spread over `cores` processes at the step cost n^alpha fitted to the sample, plus its
    corrections scaled linearly in n from the largest design's; the nested start is not
    counted (a lower bound on the oracle's time)."""
    import math
    import numpy as np
    n0, t0 = smp["n"][-1], smp["t_step"][-1]
    total = 0.0
    for d, prob in enumerate(designs):
        n = prob.n_nodes
        t_step = t0 * (n / n0) ** smp["alpha"]
        k = int(iters[d])
        total += (k + 1) * math.ceil(prob.N / cores) * prob.m * t_step + k * smp["t_corr_big"] * n / smp["n_big"]
    return {
        "value": len(designs) / total, "unit": "design steady states/s", "cores": cores, "kind": "oracle",
        "sample": (f"EXTRAPOLATED: {smp['steps']} steps of one chain of designs with {smp['n']} free nodes at "
                   f"{', '.join(f'{x * 1e3:.1f}' for x in smp['t_step'])} ms per step (one core; cost ~ n^"
                   f"{smp['alpha']:.2f}) and one coarse correction of the largest at {smp['t_corr_big']:.2f} s; "
                   f"scaled by the GPU solve's iterations per design, {cores} processes, nested start not "
                   f"counted: {total:.0f} s per batch"),
        "host": smp["host"],
    }


def batch_probe_roofline(bp, designs, prm, U_flat, prec):
    """The dominant kernel's rate on the batch: one batched fine sweep from the batch's
    converged state, timed with HIP events on the launching stream, its algorithmic bytes
    from the per-design, per-chain counters of that launch."""
    import numpy as np
    import torch
    from paper_1905_13076_amd.traffic import per_unit
    s_ = 8 if prec == 0 else 4
    bp.fine_sweep(prm, U_flat)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    _, newton, lin = bp.fine_sweep(prm, U_flat)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    alg = 0.0
    for d, prob in enumerate(designs):
        r = np.hypot(prob.xy[:, 0], prob.xy[:, 1])
        n, nnz = free_pattern(prob, np.flatnonzero(r < r.max() * (1 - 1e-12)))
        u = per_unit(n, nnz, prob.tri.shape[0], s_)
        alg += lin[d].sum() * u["pcg_iter"] + newton[d].sum() * u["newton_iter"] + prm.N * prm.m * u["step"]
    return alg, ms


def bench_batch(a):
    """Batched designs: every step is one batched PP-PC solve of all designs; value =
    designs' steady states per second.  The roofline is that of one batched fine sweep from
    the converged batch (its algorithmic bytes from the per-design chain counters over its
    event-timed duration); the CPU baseline is the oracle on a bounded sample, extrapolated."""
    import numpy as np
    import torch
    import paper_1905_13076_amd as P
    designs = batch_designs()
    smp = batch_cpu_sample(designs, a.tol_newton) if a.cpu else None
    torch.cuda.set_device(0)
    h = P.Handle(0)
    bp = P.BatchProblem(h, designs)
    prec = 0 if a.precision == "fp64" else 1
    extra = {"tol_lin": 1e-4} if prec == 1 else {}
    if a.precision == "mixed-fine":
        extra["coarse_precision"] = 0
    prm = P.problem_params(designs[0], tol_ppc=a.tol, precision=prec, tol_cocg=a.tol_cocg, max_newton=200,
                           tol_newton=a.tol_newton, lin_start=a.lin_start, tol_adapt=a.tol_adapt,
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
    U_flat = torch.cat([u.reshape(-1) for u in Us]).contiguous()
    alg, ms = batch_probe_roofline(bp, designs, prm, U_flat, prec)
    achieved = alg / (ms * 1e-3) / 1e9
    cpu = batch_cpu_extrapolate(designs, smp, iters, min(a.cpu_procs, len(os.sched_getaffinity(0)))) if smp else None
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
                   "tol_newton": a.tol_newton, "tol_adapt": a.tol_adapt,
                   "iterations_max": int(max(iters)), "damped_corrections": st["damped"],
                   "fine_ms_per_step": st["fine_ms"], "coarse_ms_per_step": st["coarse_ms"],
                   "newton_per_step": st["newton_total"] / max(1, st["steps_total"]),
                   "autotune": tuned},
        "roofline": {"kernel": "k_fine_sweep_batch (all shape groups of one batched sweep)", "bound": "hbm",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None,
                     "regime": ("cache-resident: these designs' chains fit L2 / MALL, so 'achieved' is the "
                                "algorithmic rate of one batched sweep from the converged state, not DRAM "
                                "traffic"),
                     "bytes_per_launch": alg, "launch_ms": ms},
        "cpu_baseline": cpu}))
    return 0


def c3_cpu_sample(prob, tol_newton, steps=2, harmonics=2):
    """The oracle on a bounded sample of the large coax, on one core (no worker pool: the
    sample is a single chain and a few harmonic solves): `steps` implicit-Euler steps of
    chain 1 from rest at the GPU's Newton tolerance, and the direct solves of `harmonics`
    of the N/2 + 1 shifted systems of one coarse correction (with the frozen stiffness of
    the zero state).  Returns the timings; c3_cpu_extrapolate scales them."""
    import numpy as np
    from oracle import periodic
    from oracle.fe import FE
    from oracle.timestep import fine_propagate
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    t0 = time.perf_counter()
    fe = FE(prob)
    t_setup = time.perf_counter() - t0
    dt = periodic.fine_dt(prob)
    t0 = time.perf_counter()
    fine_propagate(fe, np.zeros(fe.n), 0.0, steps, dt, tol=tol_newton)
    t_step = (time.perf_counter() - t0) / steps
    rng = np.random.default_rng(0)
    R = rng.standard_normal((prob.N, fe.n))
    Z = np.zeros((prob.N, fe.n))
    Kbar = periodic.coarse_stiffness(fe, Z, "tensor")
    t0 = time.perf_counter()
    periodic.harmonic_solve(fe, Kbar, R, prob.T, n_harm=harmonics, Jrows=Z)
    t_harm = (time.perf_counter() - t0) / harmonics
    return {"t_setup": t_setup, "t_step": t_step, "steps": steps, "t_harm": t_harm, "harmonics": harmonics,
            "host": host_info()}


def c3_cpu_extrapolate(prob, smp, sweeps, corrections, nested_sweeps, nested_corr, cores):
    """Oracle seconds per steady state: the fine chains spread over `cores` processes
    (N / cores rounds of m steps each per sweep) and the N/2 + 1 harmonic solves of every
    correction on the same cores, with the GPU solve's sweep and correction counts."""
    import math
    rounds = math.ceil(prob.N / cores)
    H = prob.N // 2 + 1
    t_sweep = rounds * prob.m * smp["t_step"]
    t_corr = math.ceil(H / cores) * smp["t_harm"]
    m_n = max(1, prob.m // 25)
    t = sweeps * t_sweep + corrections * t_corr + nested_sweeps * t_sweep * m_n / prob.m + nested_corr * t_corr
    return {
        "value": 1.0 / t, "unit": "steady states/s", "cores": cores, "kind": "oracle",
        "sample": (f"EXTRAPOLATED: {smp['steps']} implicit-Euler steps of one chain from rest (sparse LU per "
                   f"Newton step, Newton to {smp.get('tol_newton', 'the bench tolerance')}) at "
                   f"{smp['t_step']:.2f} s each and {smp['harmonics']} of the {H} harmonic solves of a "
                   f"correction at {smp['t_harm']:.2f} s each, one core; scaled to {cores} processes "
                   f"({rounds} rounds of chains per sweep) and the GPU solve's {sweeps} sweeps, {corrections} "
                   f"corrections and nested start ({nested_sweeps} sweeps of {m_n} steps) = {t:.0f} s per "
                   f"steady state"),
        "host": smp["host"],
    }


def bench_c3(a):
    """The large nonlinear coax (nr = 400 x ntheta = 800: 319,201 free nodes, 2.23 M nnz;
    N = 200 subintervals x 100 steps, 101 harmonics; fundamental plus a 20% third harmonic).
    Every step is one steady state in the chosen precision; the FP64 GPU solve of the same
    problem is run once first as the accuracy reference (its time is reported too).
    Progress (one line per fine sweep) goes to stderr."""
    import numpy as np
    import torch
    import paper_1905_13076_amd as P
    from paper_1905_13076_amd.traffic import fine_sweep_bytes
    from workloads import coax
    prob = coax.c3()
    smp = None
    if a.cpu:
        smp = c3_cpu_sample(prob, a.tol_newton)
        smp["tol_newton"] = a.tol_newton
    torch.cuda.set_device(0)
    h = P.Handle(0)
    t0 = time.perf_counter()
    pr = P.Problem(h, prob)
    setup_s = time.perf_counter() - t0

    def params(prec, adapt=a.tol_adapt):
        extra = {"tol_lin": 1e-5, "coarse_precision": 0} if prec else {}
        return P.problem_params(prob, tol_ppc=a.tol, precision=prec, tol_cocg=a.tol_cocg,
                                tol_newton=a.tol_newton, init_mode=4, tol_adapt=adapt, **extra)

    def progress(label):
        t_start = time.perf_counter()

        def fn(m, k, eps, active):
            print(f"[c3 {label}] {time.perf_counter() - t_start:7.1f}s m={m} k={k} eps={eps:.3e}",
                  file=sys.stderr, flush=True)
        return fn

    prec = 0 if a.precision == "fp64" else 1
    out = torch.empty((prob.N, pr.n_nodes), dtype=torch.float64, device="cuda")
    ref, ref_s, ref_st = None, None, None
    if prec != 0:
        t0 = time.perf_counter()
        # the reference: every sweep at the fixed Newton tolerance
        ref, _, _, ref_st, rc = pr.solve(params(0, 0.0), progress=progress("fp64 reference"))
        torch.cuda.synchronize()
        ref_s = time.perf_counter() - t0
        ref = ref.clone()
    for w in range(a.warmup):
        pr.solve(params(prec), out=out, progress=progress(f"warmup {w}"))
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for i in range(a.steps):
        U, eps, k, st, rc = pr.solve(params(prec), out=out, progress=progress(f"{a.precision} step {i}"))
        stats.append(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if rc != 0:
        print(json.dumps({"error": f"solve status {rc}", "stats": st}))
        return 1
    if ref is None:
        ref, ref_s, ref_st = U.clone(), wall / a.steps, st
    err = float(torch.linalg.norm(U - ref) / torch.linalg.norm(ref))
    fine_ms = sum(x["fine_ms"] for x in stats)
    launches = sum(x["fine_launches"] for x in stats)
    tot = {k2: sum(x[k2] for x in stats) for k2 in ("lin_total", "resid_total", "newton_total",
                                                     "steps_total", "fine_launches")}
    tot.update(n_free=st["n_free"], nnz=st["nnz"], n_tri=st["n_tri"])
    bytes_launch = fine_sweep_bytes(tot, prob.N, prec) / launches
    launch_s = fine_ms / launches / 1e3
    achieved = bytes_launch / launch_s / 1e9
    counters = os.path.join(ROOT, "profiles", f"fine_sweep_c3_{'fp64' if prec == 0 else 'fp32'}_counters.md")
    traffic = measured_traffic(a.tol_newton, counters, a.tol_adapt)
    cpu = None
    if smp is not None:
        sweeps_real = k + 1
        nested = st["fine_launches"] - sweeps_real
        cpu = c3_cpu_extrapolate(prob, smp, sweeps_real, k, nested, max(0, nested - 1),
                                 min(a.cpu_procs, len(os.sched_getaffinity(0))))
    print(json.dumps({
        "metric": "periodic steady states/s at 1e-6 rel. err vs FP64 oracle; achieved HBM GB/s",
        "value": a.steps / wall, "unit": "steady states/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": 1e3 * wall / a.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if prec == 0 else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": f"{prob.name}: nr=400 x ntheta=800 ({st['n_free']} free nodes, {st['nnz']} nnz), "
                        f"N={prob.N} x m={prob.m}, {prob.N // 2 + 1} harmonics, amplitude {prob.amps[0]:.1f} A "
                        f"+ 20% third harmonic",
            "precision": a.precision, "init": "nested", "tol_ppc": a.tol, "tol_cocg": a.tol_cocg,
            "tol_newton": a.tol_newton, "tol_adapt": a.tol_adapt, "iterations": k,
            "err_vs_fp64_gpu": err, "fp64_gpu_s_per_state": ref_s,
            "fp64_gpu_iterations": ref_st["iterations"] if ref_st else None,
            "max_b_steel_T": st["max_b_steel"],
            "newton_per_step": tot["newton_total"] / max(1, tot["steps_total"]),
            "pcg_per_newton": tot["lin_total"] / max(1, tot["newton_total"]),
            "fine_ms_per_state": fine_ms / a.steps,
            "coarse_ms_per_state": sum(x["coarse_ms"] for x in stats) / a.steps,
            "setup_s": setup_s,
        },
        "roofline": {
            "kernel": "k_fine_sweep", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": (traffic or {}).get("bytes"),
            "dram_gbs": ((traffic["bytes"] / traffic["launch_ms"] * 1e-6) if traffic and traffic.get("launch_ms")
                         else None),
            "regime": "HBM: 200 chains of 319,201 rows, far beyond L2 and MALL",
            "bytes_per_launch": bytes_launch, "launch_ms": launch_s * 1e3, "launches": launches,
        },
        "cpu_baseline": cpu,
    }), flush=True)
    return 0


def seq_cpu_sample(prob, ref, tol_newton, steps=100):
    """Route S of the oracle on one host core: `steps` implicit-Euler steps of one chain from
    the oracle's periodic state, at the GPU's Newton tolerance."""
    from oracle import periodic
    from oracle.fe import FE
    from oracle.timestep import fine_propagate
    fe = FE(prob)
    steps = min(steps, prob.N * prob.m)
    t0 = time.perf_counter()
    fine_propagate(fe, ref["U"][0], 0.0, steps, periodic.fine_dt(prob), tol=tol_newton)
    return {"t_step_seq": (time.perf_counter() - t0) / steps, "seq_steps": steps, "tol_newton": tol_newton,
            "host": host_info()}


def bench_time_stepping(a):
    """Classical time stepping on the same GPU: one steady state = periods stepped from zero
    until two periods' samples agree to --tol; progress (one line per call of a few
    periods) on stderr.  The roofline is the fine kernel's algorithmic rate over its
    event-timed launches (one chain of a period each); the CPU baseline is the oracle's
    route S on one core, extrapolated to the GPU's period count."""
    prob = workload(a.workload)
    ref = load_reference(a.workload)
    smp = seq_cpu_sample(prob, ref, a.tol_newton) if (a.cpu and ref is not None) else None
    import numpy as np
    import torch
    import paper_1905_13076_amd as P
    from paper_1905_13076_amd.traffic import fine_sweep_bytes
    torch.cuda.set_device(0)
    h = P.Handle(0)
    pr = P.Problem(h, prob)
    prec = 0 if a.precision == "fp64" else 1
    chunk = 4
    prm = P.problem_params(prob, tol_ppc=a.tol, precision=prec, max_iters=chunk, tol_newton=a.tol_newton,
                           **({"tol_lin": 1e-4} if prec == 1 else {}))
    walls, periods_all, fine_ms = [], [], 0.0
    tot = dict.fromkeys(("lin_total", "resid_total", "newton_total", "steps_total", "fine_launches"), 0)
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
                for k2 in tot:
                    tot[k2] += st[k2]
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
    tot.update(n_free=st["n_free"], nnz=st["nnz"], n_tri=st["n_tri"])
    launches = max(1, tot["fine_launches"])
    bytes_launch = fine_sweep_bytes(tot, 1, prec) / launches
    launch_ms = fine_ms / launches
    achieved = bytes_launch / (launch_ms * 1e-3) / 1e9 if launch_ms > 0 else None
    roofline = {
        "kernel": "k_fine_sweep (one chain per launch: one period of N m steps)",
        "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
        "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS if achieved else None, "traffic": None,
        "regime": ("one workgroup on one CU stepping a single chain; its working set is "
                   "cache-resident, so 'achieved' is the algorithmic rate (the method's minimal "
                   "streaming bytes over launch time), not DRAM traffic"),
        "bytes_per_launch": bytes_launch, "launch_ms": launch_ms, "launches": launches,
    }
    cpu = None
    if smp is not None:
        per = periods_all[-1]
        t_s = per * prob.N * prob.m * smp["t_step_seq"]
        cpu = {"value": 1.0 / t_s, "unit": "steady states/s", "cores": 1, "kind": "oracle",
               "sample": (f"route S: {smp['seq_steps']} sequential implicit-Euler steps of one chain "
                          f"(Newton to {smp['tol_newton']:g}) at {smp['t_step_seq'] * 1e3:.1f} ms each, "
                          f"extrapolated to the GPU's {per} periods of {prob.N * prob.m} steps = "
                          f"{t_s:.1f} s per steady state"),
               "host": smp["host"]}
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
        "roofline": roofline, "cpu_baseline": cpu}), flush=True)
    return 0


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "bench.py runs on one GPU: the path has no collectives; "
                                   "run with --gpus 1"}))
        return 2
    if a.workload == "c4reg":
        return bench_batch(a)
    if a.probe == "fine" and a.workload in ("c3", "c4"):
        return probe_large(a)
    if a.workload == "c3":
        return bench_c3(a)
    if a.method == "seq":
        return bench_time_stepping(a)
    prob = workload(a.workload)
    ref = load_reference(a.workload)
    if a.probe == "fine":
        return probe_fine(a, prob, ref)
    smp = None
    if a.cpu and ref is not None and a.method == "ppc" and a.n_harm == 0 and a.coarse == "frozen":
        # before any GPU initialisation: the oracle's worker pool forks this process
        smp = cpu_sample(prob, ref, a.cpu_procs, a.tol_newton)
    import numpy as np
    import torch
    import paper_1905_13076_amd as P
    from paper_1905_13076_amd.traffic import fine_sweep_bytes

    torch.cuda.set_device(0)
    if a.calibration_copy:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
        torch.empty_like(src).copy_(src)
        torch.cuda.synchronize()
        del src
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
                           lin_start=a.lin_start, tol_adapt=a.tol_adapt, **extra)
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
    traffic = measured_traffic(a.tol_newton, tol_adapt=a.tol_adapt) if prec == 0 else None
    cpu = None
    if smp is not None:
        nested_sweeps = st["fine_launches"] - (k + 1) if a.init == "nested" else 0
        cpu = cpu_extrapolate(prob, smp, k, max(0, nested_sweeps - 1), max(1, prob.m // 25),
                              SEQ_PERIODS.get(a.workload, 3))
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
            "tol_adapt": a.tol_adapt,
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
            "dram_gbs": ((traffic["bytes"] / traffic["launch_ms"] * 1e-6) if traffic and traffic.get("launch_ms")
                         else None),
            "regime": ("cache-resident: the chains' working set fits L2 / MALL, so 'achieved' is the "
                       "algorithmic rate (the method's minimal streaming bytes over launch time), not DRAM traffic; "
                       "dram_gbs is the counter-measured DRAM rate of the profiled launch"),
            "traffic_source": ("rocprofv3 FETCH_SIZE+WRITE_SIZE (copy-calibrated), averaged over every "
                               "fine-sweep launch of one benchmark steady state at these settings "
                               "(the nested start's sweeps included), "
                               "profiles/fine_sweep_c2_fp64_counters.md; algorithmic bytes per launch "
                               f"there {traffic['algorithmic_bytes_same_launch']}")
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

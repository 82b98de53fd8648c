"""Write the stored oracle results used by the GPU parity tests.

Calls only the CPU oracle (``oracle/``) and the seeded input generator
(``workloads/``); nothing here touches the GPU path.  Run from the repository root:

    python tests/golden/make_reference.py [c2] [c5small] [--procs 8]

Each output ``<name>_oracle.npz`` holds the fixed point U (rows n = 0..N-1, columns =
free nodes in ascending node order), the eps history, the iteration count and the
generator arguments that define the workload.  Cases ending in ``_ppic`` run PP-IC
(eq. (5)) instead of PP-PC (c5small from the fine sweep from rest); ``_h3`` runs PP-PC
solving only the harmonics p = 0, 1, 2 of each correction, ``_nested`` from the nested start; ``_nlc`` with
the nonlinear coarse problem of eq. (4), also storing one of its corrections (U_k, F_k -> dU_k at
iteration 2); ``_routes`` steps period after
period from zero (route S), its iteration count being the periods stepped.  ``c4subset``
holds a seeded subset of the batched-designs generator on a short grid (see C4_SUBSET).
``c3_sweep``, ``c3_coarse`` and ``c4_sweep`` hold sampled values of fine sweeps and a coarse
correction at the large configurations' full mesh sizes (see LARGE_M).
"""
from __future__ import annotations

import argparse
import os
import sys
import time

os.environ.setdefault("OMP_NUM_THREADS", "1")
import numpy as np  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.fe import FE  # noqa: E402
from oracle import periodic  # noqa: E402
from workloads import coax  # noqa: E402

CASES = {
    # name: (generator, kwargs, PP-PC tolerance)
    "c2": (coax.c2, {}, 1e-12),
    "c5small": (coax.c5_small, {}, 1e-12),
    "c5small_ppic": (coax.c5_small, {}, 1e-12),
    "c5small_h3": (coax.c5_small, {}, 1e-12),
    "c5small_nested": (coax.c5_small, {}, 1e-12),
    "c5small_nlc": (coax.c5_small, {}, 1e-12),
    "c2lin_small": (coax.c2lin, dict(nr=20, ntheta=40, N=10, m=20), 1e-12),
    "c2lin_small_ppic": (coax.c2lin, dict(nr=20, ntheta=40, N=10, m=20), 1e-12),
    "c2lin_small_routes": (coax.c2lin, dict(nr=20, ntheta=40, N=10, m=20), 1e-10),
}


# Seeded subset of the batched-designs generator on a short time grid (N = 8, m = 10): the
# 8 smallest designs and 4 drawn with default_rng(44) among the others with nr <= 80.
C4_SUBSET = [178, 188, 149, 8, 91, 197, 237, 74, 27, 55, 144, 184]


def c4_subset():
    return [coax.c4_designs(n_designs=256, N=8, m=10)[i] for i in C4_SUBSET]


def make_c4_subset(procs):
    """PP-PC of each subset design from rest (init "fine") with the 3 T safeguard."""
    out = {}
    t = time.time()
    for i, prob in zip(C4_SUBSET, c4_subset()):
        fe = FE(prob)
        pool = periodic.make_pool(prob, procs) if procs > 1 else None
        try:
            U, hist, k = periodic.ppc(fe, tol=1e-12, init="fine", b_cap=3.0, pool=pool, max_iter=200)
        finally:
            if pool is not None:
                pool.close()
                pool.join()
        out[f"U_{i}"] = U
        out[f"hist_{i}"] = hist
        out[f"iterations_{i}"] = k
        out[f"free_{i}"] = fe.free.astype(np.int32)
        print(f"  [c4subset] design {i} nr={prob.meta['nr']}: {k} iterations, eps {hist[-1]:.2e}, "
              f"t={time.time() - t:.0f}s", flush=True)
    path = os.path.join(HERE, "c4subset_oracle.npz")
    np.savez_compressed(path, designs=np.array(C4_SUBSET, dtype=np.int32), **out)
    print(f"wrote {path} in {time.time() - t:.1f}s")


# Large cases, compared on sampled values: fine sweeps with m = 2 steps of the workloads' own
# step size (C3: dt = 1e-6 over N = 200 chains; the batched designs: dt = 1e-5 over N = 40),
# and one C3 coarse correction solving the harmonics p = 0, 1, 2 (the rest from the jumps).
LARGE_M = 2
C3_CHAINS = [1, 77, 200]
C4_CHAINS = [1, 17, 40]
# the sweep check adds the three designs with the most rings (nr 200, 199, 199: the streaming
# memory path) to the subset
C4_SWEEP_DESIGNS = C4_SUBSET + [213, 227, 206]


def make_c3_sweep():
    from oracle.timestep import fine_propagate
    prob = coax.c3()
    fe = FE(prob)
    dt = prob.T / (prob.N * prob.m)
    T = prob.N * LARGE_M * dt
    U0 = coax.chain_starts(prob, fe.free, seed=3)
    idx = coax.sample_index(fe.n, 4096, seed=31)
    out = {"idx": idx, "chains": np.array(C3_CHAINS, dtype=np.int32), "m": LARGE_M, "T": T}
    t = time.time()
    for c in C3_CHAINS:
        u = fine_propagate(fe, U0[c - 1], (c - 1) * T / prob.N, LARGE_M, dt)
        out[f"F_{c}"] = u[idx]
        out[f"norm_{c}"] = np.linalg.norm(u)
        print(f"  [c3_sweep] chain {c}: t={time.time() - t:.0f}s", flush=True)
    path = os.path.join(HERE, "c3_sweep_oracle.npz")
    np.savez_compressed(path, **out)
    print(f"wrote {path}")


def make_c3_coarse():
    prob = coax.c3()
    fe = FE(prob)
    U = coax.random_rows(prob.N, fe.n, seed=33, amp=2e-6)
    J = coax.random_rows(prob.N, fe.n, seed=34, amp=1e-7)
    t = time.time()
    dU = periodic.coarse_correction(fe, U, J, n_harm=3)
    rows = np.array([0, 57, 123], dtype=np.int32)
    idx = coax.sample_index(fe.n, 4096, seed=35)
    path = os.path.join(HERE, "c3_coarse_oracle.npz")
    np.savez_compressed(path, rows=rows, idx=idx, dU=dU[rows][:, idx], norm=np.linalg.norm(dU),
                        row_norms=np.linalg.norm(dU[rows], axis=1), n_harm=3)
    print(f"wrote {path} in {time.time() - t:.0f}s")


def make_c4_sweep():
    from oracle.timestep import fine_propagate
    designs = coax.c4_designs()
    out = {"designs": np.array(C4_SWEEP_DESIGNS, dtype=np.int32), "chains": np.array(C4_CHAINS, dtype=np.int32),
           "m": LARGE_M}
    t = time.time()
    for d in C4_SWEEP_DESIGNS:
        prob = designs[d]
        fe = FE(prob)
        dt = prob.T / (prob.N * prob.m)
        T = prob.N * LARGE_M * dt
        U0 = coax.chain_starts(prob, fe.free, seed=1000 + d)
        idx = coax.sample_index(fe.n, 1024, seed=2000 + d)
        out[f"idx_{d}"] = idx
        for c in C4_CHAINS:
            u = fine_propagate(fe, U0[c - 1], (c - 1) * T / prob.N, LARGE_M, dt)
            out[f"F_{d}_{c}"] = u[idx]
            out[f"norm_{d}_{c}"] = np.linalg.norm(u)
        print(f"  [c4_sweep] design {d} nr={prob.meta['nr']}: t={time.time() - t:.0f}s", flush=True)
    path = os.path.join(HERE, "c4_sweep_oracle.npz")
    np.savez_compressed(path, **out)
    print(f"wrote {path}")


LARGE = {"c3_sweep": make_c3_sweep, "c3_coarse": make_c3_coarse, "c4_sweep": make_c4_sweep}


def make(name, procs):
    gen, kw, tol = CASES[name]
    prob = gen(**kw)
    fe = FE(prob)
    pool = periodic.make_pool(prob, procs) if procs > 1 else None
    t = time.time()
    hist_print = []

    extra = {}

    def cb(k, U, Fs, eps):
        if k == 2 and name.endswith("_nlc"):
            extra["U_k"], extra["F_k"] = U.copy(), Fs.copy()
        hist_print.append(eps)
        print(f"  [{name}] k={k} eps={eps:.3e} t={time.time() - t:.1f}s", flush=True)

    try:
        if name.endswith("_routes"):    # sequential periods from zero (classical time stepping)
            U, k = periodic.route_s(fe, tol=tol)
            hist = np.zeros(0)
        elif name == "c5small_ppic":     # from rest: a coarse start from zero overshoots
            U0 = periodic.initial_iterate(fe, mode="fine", pool=pool)
            U, hist, k = periodic.ppic(fe, tol=tol, U_init=U0, pool=pool, callback=cb)
        elif name.endswith("_ppic"):
            U, hist, k = periodic.ppic(fe, tol=tol, pool=pool, callback=cb)
        elif name.endswith("_nested"):  # start from the 25 times coarser fine grid's solution
            U, hist, k = periodic.ppc(fe, tol=tol, pool=pool, callback=cb, init="nested")
        elif name.endswith("_nlc"):     # nonlinear periodic coarse problem
            U, hist, k = periodic.ppc(fe, tol=tol, pool=pool, callback=cb, coarse="nonlinear")
            extra["dU_k"] = periodic.nonlinear_coarse_correction(fe, extra["U_k"], extra["F_k"])
        elif name.endswith("_h3"):      # truncated harmonic set: p = 0, 1, 2 solved
            U, hist, k = periodic.ppc(fe, tol=tol, pool=pool, callback=cb, n_harm=3)
        else:
            U, hist, k = periodic.ppc(fe, tol=tol, pool=pool, callback=cb)
    finally:
        if pool is not None:
            pool.close()
            pool.join()
    out = os.path.join(HERE, f"{name}_oracle.npz")
    np.savez_compressed(out, U=U, hist=hist, iterations=k, tol=tol,
                        free=fe.free.astype(np.int32), generator=name, **extra)
    last = f"{hist[-1]:.3e}" if len(hist) else "-"
    print(f"wrote {out}: iterations={k} eps={last} in {time.time() - t:.1f}s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("cases", nargs="*", default=list(CASES) + ["c4subset"] + list(LARGE))
    ap.add_argument("--procs", type=int, default=min(8, os.cpu_count() or 1))
    a = ap.parse_args()
    for c in a.cases:
        if c == "c4subset":
            make_c4_subset(a.procs)
        elif c in LARGE:
            LARGE[c]()
        else:
            make(c, a.procs)


if __name__ == "__main__":
    main()

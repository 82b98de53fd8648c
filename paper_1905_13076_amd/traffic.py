"""Algorithmic HBM bytes of the fine-sweep kernel: what one launch must move if every
input is read once and every output written once, from the per-chain counters the
kernel returns (steps, Newton iterations, residual evaluations, PCG iterations).

Per-unit figures (n free nodes, nnz CSR entries, ne triangles, s = bytes of the PCG
scalar: 8 FP64, 4 mixed):

* PCG iteration      (s+4) nnz + 4 (n+1) + 13 s n
  (SpMV values + columns + row pointers, gather p, write q; x,r update reads x p r q
  dinv and writes x r; direction reads dinv r p and writes p)
* residual evaluation 180 ne + (36+s) n + 4
  (element pass: 3 vertex indices, 6 K0 entries, area, sigma, material in, 8 values out,
  vertex gathers of u, du, u_prev; node pass: incidence list, 3 element forces, load
  vector in, residual out)
* Newton iteration   assembly 4 (nnz+1) + 4 c + 88 ne + (8+s) nnz + (4+2s) n
  (c = slot contributions) plus PCG set-up, step-norm and update passes (32+6s) n
* time step          12 nnz + 28 n + 4 (copy u to u_prev, ||M u_prev|| SpMV)
* chain              16 n (start vector in, end vector out)
"""
from __future__ import annotations


def per_unit(n, nnz, ne, s, n_contrib=None):
    c = 9 * ne if n_contrib is None else n_contrib
    return {
        "pcg_iter": (s + 4) * nnz + 4 * (n + 1) + 13 * s * n,
        "resid_eval": 180 * ne + (36 + s) * n + 4,
        "newton_iter": 4 * (nnz + 1) + 4 * c + 88 * ne + (8 + s) * nnz + (4 + 2 * s) * n + (32 + 6 * s) * n,
        "step": 12 * nnz + 28 * n + 4,
        "chain": 16 * n,
    }


def fine_sweep_bytes(stats, N, precision):
    """Total algorithmic bytes of all fine-sweep launches described by a stats dict."""
    s = 8 if precision == 0 else 4
    u = per_unit(stats["n_free"], stats["nnz"], stats["n_tri"], s)
    return (stats["lin_total"] * u["pcg_iter"] + stats["resid_total"] * u["resid_eval"]
            + stats["newton_total"] * u["newton_iter"] + stats["steps_total"] * u["step"]
            + stats["fine_launches"] * N * u["chain"])

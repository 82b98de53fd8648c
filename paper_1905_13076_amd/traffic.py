"""Algorithmic HBM bytes of the fine-sweep kernel: what one launch must move if every
input is read once and every output written once (shared patterns counted per chain,
as a cache-less implementation would move them), from the per-chain counters the
kernel returns (steps, Newton iterations, residual evaluations, PCG iterations).

Per-unit figures (n free nodes, nnz CSR entries, s = bytes of the PCG scalar: 8 FP64,
4 mixed; a triangulated mesh has about 2n elements):

* PCG iteration       (s+4) nnz + 4 (n+1) + 13 s n
  (SpMV values + columns + row pointers, gather p, write q; x,r update reads x p r q
  dinv and writes x r; direction reads dinv r p and writes p)
* residual evaluation 168 n
  (FP64: state and previous state, geometry of the ~2n elements at 68 B, residual out)
* Newton iteration    (144 + 8 s) n  (assembly: state, geometry, Jacobian values, diagonal);
  its residual evaluations and PCG iterations are counted by their own units
* time step           12 nnz + 28 n + 4 (copy u to u_prev, ||M u_prev|| SpMV)
* chain               16 n (start vector in, end vector out)

These are properties of the method's minimal streaming form, independent of where an
implementation keeps its vectors or how it reuses the state-independent part of the
Jacobian.
"""
from __future__ import annotations


def per_unit(n, nnz, ne, s):
    return {
        "pcg_iter": (s + 4) * nnz + 4 * (n + 1) + 13 * s * n,
        "resid_eval": 168 * n,
        "newton_iter": (144 + 8 * s) * n,
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

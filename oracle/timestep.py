"""Implicit-Euler fine propagator with damped Newton (oracle, FP64, direct solves).

Paper, Section 2, eqs. (2)-(3): F_n maps U_{n-1} at T_{n-1} to the solution of the
initial-value problem at T_n; Section 4 gives only the fine step size.  Reading:
the fine integrator is implicit Euler (the coarse integrator of eq. (8)) with the
source taken at the step end, and each step solves

    R(u) = M (u - u_prev)/dt + K(u) u - f(t_j) = 0

by Newton's method with Jacobian ``M/dt + d(K(u)u)/du`` and backtracking on ||R||.

TEST INFRASTRUCTURE ONLY: see the package docstring.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

NEWTON_TOL = 1e-13
NEWTON_MAXIT = 50
# A residual that no longer halves while below FLOOR_CAP * scale sits at the rounding
# floor of its own evaluation: the step is solved as far as FP64 can resolve it.  That
# floor grows with the ratio of stiffness to mass entries, about as the square of the ring
# count of the coax meshes (measured 5e-13 of the scale at 20 rings, 5e-12 at 60, 4e-11
# at 150; about 3e-10 at 400 by extrapolation), so the cap is set for the finest mesh.
# Exits are counted (stats "floor_exits", largest ||R|| / scale in "floor_max") so that
# tests can check they happen only at the floor of the mesh at hand.
FLOOR_CAP = 1e-9


class NewtonFailure(RuntimeError):
    pass


def _floor_exit(stats, ratio):
    if stats is not None:
        stats["floor_exits"] = stats.get("floor_exits", 0) + 1
        stats["floor_max"] = max(stats.get("floor_max", 0.0), ratio)


def step_residual(fe, u, u_prev, t, dt):
    return fe.M @ (u - u_prev) / dt + fe.K_apply(u) - fe.f(t)


def ie_step(fe, u_prev, t, dt, tol=NEWTON_TOL, maxit=NEWTON_MAXIT, stats=None):
    """One implicit-Euler step from u_prev to time t.

    Stops when ||R|| <= tol * scale, scale = ||f(t)|| + ||M u_prev||/dt; or when the
    residual has reached the rounding floor of its evaluation: the Newton correction is
    at rounding level (||du|| <= 4 eps ||u||), or an accepted step fails to halve ||R||
    while ||R|| <= FLOOR_CAP * scale, or the line search stalls there.  Backtracking:
    lambda = 1, 1/2, ... 2^-20 until ||R(u + lambda du)|| <= (1 - 1e-4 lambda) ||R(u)||."""
    f_norm = np.linalg.norm(fe.f(t))
    scale = f_norm + np.linalg.norm(fe.M @ u_prev) / dt
    u = u_prev.copy()
    R = step_residual(fe, u, u_prev, t, dt)
    rn = np.linalg.norm(R)
    for it in range(maxit + 1):
        if rn <= tol * scale:
            break
        if it == maxit:
            raise NewtonFailure(f"Newton did not converge at t={t}: ||R||={rn:.3e} "
                                f"target={tol * scale:.3e}")
        J = (fe.M / dt + fe.jacobian_curl(u)).tocsc()
        du = spla.splu(J, permc_spec="MMD_AT_PLUS_A").solve(-R)
        if stats is not None:
            stats["solves"] = stats.get("solves", 0) + 1
        if np.linalg.norm(du) <= 4.0 * np.finfo(float).eps * np.linalg.norm(u):
            u = u + du
            break
        lam = 1.0
        while True:
            ut = u + lam * du
            Rt = step_residual(fe, ut, u_prev, t, dt)
            rt = np.linalg.norm(Rt)
            if rt <= (1.0 - 1e-4 * lam) * rn:
                break
            lam *= 0.5
            if lam < 2.0 ** -20:
                # no decrease is representable: the iterate sits at rounding level
                if rn <= FLOOR_CAP * scale:
                    _floor_exit(stats, rn / scale)
                    return u, it
                raise NewtonFailure(f"line search failed at t={t}: ||R||={rn:.3e}")
        floor = rt > 0.5 * rn and rt <= FLOOR_CAP * scale
        u, R, rn = ut, Rt, rt
        if floor:
            _floor_exit(stats, rn / scale)
            it += 1
            break
    if stats is not None:
        stats["newton"] = stats.get("newton", 0) + it
        stats["steps"] = stats.get("steps", 0) + 1
    return u, it


def fine_propagate(fe, u0, t0, m, dt, trajectory=False, tol=NEWTON_TOL, stats=None):
    """F(u0): m implicit-Euler steps of size dt from time t0 (eqs. (2)-(3)).
    Step j ends at t0 + j*dt."""
    u = np.array(u0, dtype=np.float64, copy=True)
    traj = [u.copy()] if trajectory else None
    for j in range(1, m + 1):
        u, _ = ie_step(fe, u, t0 + j * dt, dt, tol=tol, stats=stats)
        if trajectory:
            traj.append(u.copy())
    return (u, np.array(traj)) if trajectory else u

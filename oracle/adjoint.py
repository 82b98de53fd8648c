"""Adjoint gradients of the period-averaged eddy-current loss (oracle, FP64).

The paper computes the periodic steady state (Section 2, eq. (1)); the loss and its
sensitivities are an addition to it, stated here from the discrete equations.

With L = N m implicit-Euler steps of the periodic fine solution (u_L = u_0),
    R_j(u_j, u_{j-1}; theta) = M (u_j - u_{j-1})/dt + K(u_j; theta) u_j - f(t_j) = 0,
the loss is the exact element integral of sigma (dA/dt)^2 averaged over a period,
    P = (1/(T dt)) sum_{j=1..L} du_j^T M du_j,    du_j = u_j - u_{j-1}.
Its gradient with respect to any parameter theta is
    dP/dtheta = dP/dtheta|_u - sum_j lambda_j^T dR_j/dtheta,
where the adjoint lambda solves the transposed cyclic system
    J_j lambda_j = (M/dt) lambda_{j+1} + dP/du_j,   lambda_{L+1} = lambda_1,
with the symmetric Jacobian J_j = M/dt + d(K(u)u)/du at u_j and
    dP/du_j = (2/(T dt)) M (du_j - du_{j+1}).
Parameters: the conductivity sigma_e of every element (dR_j/dsigma_e = M1_e du_j/dt,
dP/dsigma_e|_u = (1/(T dt)) sum_j du_j^T M1_e du_j with M1_e the unit-sigma element
mass) and the Brauer constants (k1, k2, k3) of every Brauer material
(dR_j/dk = sum_e dnu_e/dk K0_e u_j with dnu/dk1 = e^{k2 b2}, dnu/dk2 = k1 b2 e^{k2 b2},
dnu/dk3 = 1).

TEST INFRASTRUCTURE ONLY: see the package docstring.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fe import BRAUER
from .timestep import fine_propagate


def periodic_trajectory(fe, U):
    """The fine trajectory u_0..u_L of one period started from the periodic U_0."""
    prob = fe.prob
    N, m = prob.N, prob.m
    dt = prob.T / (N * m)
    traj = [np.array(U[0], dtype=np.float64)]
    u = traj[0]
    for n in range(1, N + 1):
        u, seg = fine_propagate(fe, u, (n - 1) * (prob.T / N), m, dt, trajectory=True)
        traj.extend(seg[1:])
    return np.array(traj)


def loss(fe, traj):
    prob = fe.prob
    dt = prob.T / (prob.N * prob.m)
    du = np.diff(traj, axis=0)
    return float(np.sum(du * (fe.M @ du.T).T) / (prob.T * dt))


def _jacobian(fe, u, dt):
    return (fe.M / dt + fe.jacobian_curl(u)).tocsc()


def adjoint_rhs(fe, traj):
    """dP/du_j for j = 1..L (rows 0..L-1), cyclic."""
    prob = fe.prob
    dt = prob.T / (prob.N * prob.m)
    du = np.diff(traj, axis=0)                 # du_j, j = 1..L
    dnext = np.roll(du, -1, axis=0)            # du_{j+1}, du_{L+1} = du_1
    return (2.0 / (prob.T * dt)) * (fe.M @ (du - dnext).T).T


def adjoint_solve(fe, traj, tol=1e-15, max_periods=500):
    """Periodic adjoint by backward sweeps over whole periods until lambda_1 repeats
    (the backward analogue of sequential time stepping to the periodic state).
    Returns lam with rows j = 1..L."""
    prob = fe.prob
    L = prob.N * prob.m
    dt = prob.T / L
    g = adjoint_rhs(fe, traj)
    lus = [spla.splu(_jacobian(fe, traj[j], dt), permc_spec="MMD_AT_PLUS_A") for j in range(1, L + 1)]
    lam = np.zeros((L, fe.n))
    nxt = np.zeros(fe.n)                        # lambda_{L+1}
    prev1 = None
    for _ in range(max_periods):
        for j in range(L, 0, -1):
            lam[j - 1] = lus[j - 1].solve(fe.M @ nxt / dt + g[j - 1])
            nxt = lam[j - 1]
        nxt = lam[0]                             # lambda_{L+1} = lambda_1
        if prev1 is not None and np.linalg.norm(lam[0] - prev1) <= tol * np.linalg.norm(lam[0]):
            return lam
        prev1 = lam[0].copy()
    raise RuntimeError("adjoint periods did not converge")


def adjoint_direct(fe, traj):
    """Brute force for tiny problems: assemble the (L n) x (L n) transposed cyclic system
    and solve it directly (rows j = 1..L)."""
    prob = fe.prob
    L = prob.N * prob.m
    dt = prob.T / L
    blocks = [_jacobian(fe, traj[j], dt) for j in range(1, L + 1)]
    A = sp.block_diag(blocks, format="csr")
    S = sp.csr_matrix((np.ones(L), (np.arange(L), (np.arange(L) + 1) % L)), shape=(L, L))
    A = (A - sp.kron(S, fe.M / dt)).tocsc()
    g = adjoint_rhs(fe, traj).ravel()
    return spla.spsolve(A, g).reshape(L, fe.n)


def gradients(fe, traj, lam):
    """(dP/dsigma per element, dP/dk per material as an [n_mat, 3] array with zeros for
    linear materials)."""
    prob = fe.prob
    L = prob.N * prob.m
    dt = prob.T / L
    du = np.diff(traj, axis=0)
    M1 = (fe.area / 12.0)[:, None, None] * (np.ones((3, 3)) + np.eye(3))[None, :, :]
    dsig = np.zeros(prob.n_tri)
    dk = np.zeros((len(prob.mat_model), 3))
    brauer = fe.model == BRAUER
    for j in range(L):
        de = fe.full(du[j])[fe.tri]
        le = fe.full(lam[j])[fe.tri]
        Md = np.einsum("eab,eb->ea", M1, de)
        dsig += np.einsum("ea,ea->e", de, Md) / (prob.T * dt) - np.einsum("ea,ea->e", le, Md) / dt
        if np.any(brauer):
            ue, w, b2, nu, dnu = fe.element_state(traj[j + 1])
            lw = np.einsum("ea,ea->e", le, w)
            par = fe.par
            ex = np.exp(par[:, 2] * b2)
            dnu_dk = np.stack([ex, par[:, 1] * b2 * ex, np.ones_like(ex)], axis=1)
            contrib = -(dnu_dk * lw[:, None])
            for mid in np.unique(prob.mat_id[brauer]):
                sel = brauer & (prob.mat_id == mid)
                dk[mid] += contrib[sel].sum(axis=0)
    return dsig, dk

"""Pins of the oracle's adjoint gradients of the period-averaged eddy-current loss:
central finite differences of the loss through complete periodic re-solves, a direct
solve of the transposed cyclic system, and the vanishing Brauer gradient of a linear
problem."""
import copy

import numpy as np
import pytest

from oracle import adjoint, periodic
from oracle.fe import FE
from workloads import coax


def _solve_loss(prob):
    fe = FE(prob)
    U, _, _ = periodic.ppc(fe, tol=1e-14, init="zero")
    traj = adjoint.periodic_trajectory(fe, U)
    return fe, traj, adjoint.loss(fe, traj)


def _tiny(nonlinear=True):
    return coax.tiny(nr=4, ntheta=8, N=4, m=3, nonlinear=nonlinear, amp=300.0 if nonlinear else 1.0)


def test_backward_sweeps_equal_direct_transposed_solve():
    fe, traj, _ = _solve_loss(_tiny())
    lam = adjoint.adjoint_solve(fe, traj)
    lam_d = adjoint.adjoint_direct(fe, traj)
    assert np.linalg.norm(lam - lam_d) <= 1e-10 * np.linalg.norm(lam_d)


def test_periodic_trajectory_closes():
    fe, traj, P = _solve_loss(_tiny())
    assert np.linalg.norm(traj[-1] - traj[0]) <= 1e-11 * np.linalg.norm(traj[0])
    assert P > 0


@pytest.mark.parametrize("nonlinear", [True, False])
def test_gradients_match_central_differences(nonlinear):
    prob = _tiny(nonlinear)
    fe, traj, P0 = _solve_loss(prob)
    lam = adjoint.adjoint_solve(fe, traj)
    dsig, dk = adjoint.gradients(fe, traj, lam)
    smax = prob.sigma.max()
    # a copper core element, an insulator element (sigma = 0), an outer-layer element
    # and the steel sheath (outer ring)
    picks = [0, len(prob.sigma) // 3, len(prob.sigma) // 2, len(prob.sigma) - 1]
    for e in picks:
        h = 1e-6 * (prob.sigma[e] if prob.sigma[e] > 0 else smax)
        vals = []
        for sgn in (+1, -1):
            q = copy.deepcopy(prob)
            q.sigma = prob.sigma.copy()
            q.sigma[e] += sgn * h
            vals.append(_solve_loss(q)[2])
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - dsig[e]) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(dsig).max()), (e, fd, dsig[e])
    if nonlinear:
        mid = int(np.flatnonzero(prob.mat_model == 1)[0])
        for i in range(3):
            h = 1e-6 * prob.mat_par[mid, 1 + i]
            vals = []
            for sgn in (+1, -1):
                q = copy.deepcopy(prob)
                q.mat_par = prob.mat_par.copy()
                q.mat_par[mid, 1 + i] += sgn * h
                vals.append(_solve_loss(q)[2])
            fd = (vals[0] - vals[1]) / (2 * h)
            assert abs(fd - dk[mid, i]) <= 1e-5 * abs(fd), (i, fd, dk[mid, i])
    else:
        assert np.all(dk == 0.0)


def _c1_loss(m):
    """Loss of the C1 periodic implicit-Euler solution with m steps per subinterval
    (route L: the exact DFT solve of the cyclic fine system)."""
    fe = FE(coax.c1(m=m))
    _, u = periodic.route_l(fe)                 # rows j = 0..L-1, u_0 = u_L
    return fe, u, adjoint.loss(fe, np.vstack([u, u[:1]]))


def test_loss_equals_the_energy_balance_of_the_periodic_solution():
    """Independent value of P from the source and the stiffness instead of the mass:
    multiplying the periodic implicit-Euler equations (Section 2, eq. (1) in time) by
    du_j and summing over a period telescopes the stored energy, so
    T P = sum_j f_j.du_j - 1/2 sum_j du_j.K du_j.  A factor 2, a missing 1/T or dt in
    place of 1/dt in the loss fails here."""
    fe, u, P = _c1_loss(20)
    prob = fe.prob
    L = prob.N * prob.m
    dt = prob.T / L
    K = fe.K_matrix(np.full(prob.n_tri, coax.NU0))
    du = u - np.roll(u, 1, axis=0)
    t = np.arange(L) * dt
    t[0] = prob.T
    f = np.outer(prob.current(t), fe.F)
    PT = (np.sum(f * du) - 0.5 * np.sum(du * (K @ du.T).T)) / prob.T
    assert abs(P - PT) <= 1e-10 * abs(PT), (P, PT)


def test_loss_converges_to_the_phasor_loss_at_first_order():
    """Physics pin: for a linear problem driven by I sin(wt), the space-discrete periodic
    solution is A(t) = Im(Ah e^{iwt}) with (K + iwM) Ah = I F, and the period average of
    dA/dt^T M dA/dt is w^2/2 Re(Ah^H M Ah).  Implicit Euler is first order, so the
    relative error of P halves with every halving of dt, and the Richardson value
    2 P(dt/2) - P(dt) is second-order accurate."""
    import math
    import scipy.sparse.linalg as spla
    fe, _, _ = _c1_loss(20)
    prob = fe.prob
    w = 2.0 * math.pi * prob.f0 * prob.orders[0]
    K = fe.K_matrix(np.full(prob.n_tri, coax.NU0))
    Ah = spla.splu((K + 1j * w * fe.M).tocsc()).solve(prob.amps[0] * fe.F.astype(np.complex128))
    Pph = 0.5 * w * w * float(np.real(np.vdot(Ah, fe.M @ Ah)))
    P = {m: _c1_loss(m)[2] for m in (20, 40, 80)}
    e = {m: P[m] / Pph - 1.0 for m in P}
    assert abs(e[20]) <= 0.05 * w * (prob.T / (prob.N * 20))     # O(w dt), small constant
    assert 1.8 <= e[20] / e[40] <= 2.3 and 1.8 <= e[40] / e[80] <= 2.3, e
    assert abs(2.0 * P[80] - P[40] - Pph) <= 2e-5 * Pph, (P, Pph)

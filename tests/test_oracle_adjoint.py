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

"""Pins of the oracle's fine-step Newton iteration (implicit Euler of Section 2, eq. (1)):
its rounding-floor exit happens only at the floor of the mesh at hand, so a Newton
iteration that converges slowly (a wrong Jacobian) cannot pass for a converged one."""
import numpy as np
import pytest

from oracle import timestep
from oracle.fe import FE
from workloads import coax


def _chain_stats(fe, prob, jac=None):
    if jac is not None:
        fe.jacobian_curl = jac
    rng = np.random.default_rng(20)
    r = np.hypot(prob.xy[fe.free, 0], prob.xy[fe.free, 1])
    U0 = np.outer(1.0 + 0.1 * rng.standard_normal(prob.N), 1e-4 * (3e-3 - r) / 3e-3)
    dt = prob.T / (prob.N * prob.m)
    stats = {}
    for n in range(1, prob.N + 1):
        timestep.fine_propagate(fe, U0[n - 1], (n - 1) * prob.T / prob.N, prob.m, dt, stats=stats)
    return stats


def test_floor_exits_stay_at_the_rounding_floor_of_a_coarse_mesh():
    """20 rings: the FP64 floor of the residual is about 5e-13 of the Newton scale, so
    every floor exit lies below 2e-11 of it although the cap allows 1e-9."""
    prob = coax.c2(nr=20, ntheta=40, N=4, m=4)
    st = _chain_stats(FE(prob), prob)
    assert st.get("floor_max", 0.0) <= 2e-11, st


def test_a_wrong_jacobian_is_not_taken_for_the_rounding_floor():
    """Planted mistake: the Jacobian without the Brauer derivative term (the chord
    reluctivity only).  Newton then converges linearly and stalls well above the floor,
    which either fails the step or shows as a floor exit above the coarse mesh's floor."""
    prob = coax.c2(nr=20, ntheta=40, N=4, m=4)
    fe = FE(prob)

    def chord_jacobian(u):
        _, _, _, nu, _ = fe.element_state(u)
        return fe.K_matrix(nu)

    try:
        st = _chain_stats(fe, prob, jac=chord_jacobian)
    except timestep.NewtonFailure:
        return
    assert st.get("floor_max", 0.0) > 2e-11, st

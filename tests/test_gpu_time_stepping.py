"""Classical time stepping on the GPU (one chain of the fine kernel per period) against the
oracle's sequential periods (route S): the same number of periods under the same stopping
rule and the same states; a run split into calls equals one call."""
import numpy as np
import pytest

from workloads import coax
from tests.gpu_common import banner, free_rows, handle, load_golden, rel

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["c1", "c5small"])
def test_time_stepping_matches_oracle_route_s(name):
    import paper_1905_13076_amd as P
    from oracle import periodic
    from oracle.fe import FE
    prob = {"c1": coax.c1, "c5small": coax.c5_small}[name]()
    fe = FE(prob)
    Uo, po = periodic.route_s(fe, tol=1e-10)
    pr = P.Problem(handle(), prob)
    banner(f"time stepping {name}")
    U, periods, st, rc = pr.time_stepping(P.problem_params(prob, tol_ppc=1e-10, max_iters=100))
    assert rc == 0, st
    e = rel(free_rows(U.cpu().numpy(), fe.free), Uo)
    banner(f"  periods {periods} (oracle {po}) rel {e:.2e} steps {st['steps_total']} fine ms {st['fine_ms']:.1f}")
    assert periods == po
    assert e <= 1e-10
    assert st["steps_total"] == periods * prob.N * prob.m
    # the periodic state PP-PC finds
    if name == "c5small":
        assert rel(free_rows(U.cpu().numpy(), fe.free), load_golden("c5small")["U"]) <= 1e-8


def test_slow_transient_time_stepping_matches_oracle():
    """Linearised C2 (small): the sheath's time constant takes 50 periods of classical
    stepping to 1e-10, against 7 PP-PC iterations."""
    import paper_1905_13076_amd as P
    from oracle.fe import FE
    prob = coax.c2lin(nr=20, ntheta=40, N=10, m=20)
    fe = FE(prob)
    g = load_golden("c2lin_small_routes")
    pr = P.Problem(handle(), prob)
    U, periods, st, rc = pr.time_stepping(P.problem_params(prob, tol_ppc=1e-10, max_iters=200))
    assert rc == 0
    e = rel(free_rows(U.cpu().numpy(), fe.free), g["U"])
    banner(f"c2lin small time stepping: periods {periods} (oracle {int(g['iterations'])}) rel {e:.2e}")
    assert periods == int(g["iterations"]) and e <= 1e-10


def test_time_stepping_split_into_calls_equals_one_call():
    import paper_1905_13076_amd as P
    prob = coax.c2lin(nr=20, ntheta=40, N=10, m=20)
    pr = P.Problem(handle(), prob)
    prm = P.problem_params(prob, tol_ppc=1e-8, max_iters=400)
    banner("time stepping c2lin small, one call")
    U1, p1, st1, rc1 = pr.time_stepping(prm)
    assert rc1 == 0
    banner(f"  {p1} periods")
    # three periods per call, each call continuing from the last one's end and samples
    prm3 = P.problem_params(prob, tol_ppc=1e-8, max_iters=3)
    total, u0, Up = 0, None, None
    while True:
        U, per, st, rc = pr.time_stepping(prm3, u_start=u0, U_prev=Up)
        total += per
        if rc == 0:
            break
        assert total < 400
        Up = U
        u0 = U[0].contiguous()
    banner(f"  split: {total} periods")
    assert total == p1
    assert float((U - U1).abs().max()) == 0.0
    # the slow transient: many periods, unlike the quasi-static cases
    assert p1 > 10

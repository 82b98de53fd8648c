"""Failure reporting, forced from the host so that every kernel still exits normally: a
Newton step that cannot converge (one iteration allowed at an unreachable tolerance), the
PP-PC iteration cap, the COCG iteration cap and a failing design inside a batch.  Each is
reported through the status codes of the C-ABI, with the failing chain or design named."""
import numpy as np
import pytest
import torch

from workloads import coax
from tests.gpu_common import banner, handle

pytestmark = pytest.mark.gpu


def test_newton_failure_is_reported_with_its_chain():
    import paper_1905_13076_amd as P
    prob = coax.c5_small()
    pr = P.Problem(handle(), prob)
    prm = P.problem_params(prob, max_newton=1, tol_newton=1e-15, no_predictor=1)
    U0 = torch.zeros((prob.N, pr.n_nodes), dtype=torch.float64, device="cuda")
    with pytest.raises(P.PPCError) as ei:
        pr.fine_sweep(prm, U0)
    banner(f"fine sweep: {ei.value}")
    assert ei.value.code == -7 and "fine chain" in str(ei.value)
    with pytest.raises(P.PPCError) as ei:
        pr.solve(prm)
    assert ei.value.code == -7
    # the problem stays usable after the failure
    U, eps, k, st, rc = pr.solve(P.problem_params(prob, tol_ppc=1e-8))
    assert rc == 0


def test_iteration_cap_returns_the_last_iterate():
    import paper_1905_13076_amd as P
    prob = coax.c5_small()
    pr = P.Problem(handle(), prob)
    U, eps, k, st, rc = pr.solve(P.problem_params(prob, max_iters=2))
    banner(f"capped solve: rc={rc} iterations={k} eps={eps}")
    assert rc == 1 and k == 2 and len(eps) == 3 and eps[-1] > 1e-12
    assert np.all(np.isfinite(U.cpu().numpy()))


def test_cocg_cap_is_visible_in_the_counters():
    import paper_1905_13076_amd as P
    prob = coax.c1()
    pr = P.Problem(handle(), prob)
    rng = np.random.default_rng(3)
    U = torch.tensor(rng.standard_normal((prob.N, pr.n_nodes)) * 1e-4, device="cuda")
    J = torch.tensor(rng.standard_normal((prob.N, pr.n_nodes)) * 1e-6, device="cuda")
    dU, cocg = pr.coarse_correction(P.problem_params(prob, max_cocg=3), U, J)
    banner(f"capped COCG iterations {np.asarray(cocg).tolist()}")
    assert np.all(np.asarray(cocg) == 3)
    dU2, cocg2 = pr.coarse_correction(P.problem_params(prob), U, J)
    assert np.all(np.asarray(cocg2) > 3)


def test_failing_design_in_a_batch_is_named():
    import paper_1905_13076_amd as P
    # design 0 carries no current (zero residual, nothing to solve); design 1 fails
    designs = [coax.tiny(nr=6, ntheta=12, N=8, m=6, nonlinear=False, amp=0.0),
               coax.tiny(nr=8, ntheta=16, N=8, m=6, nonlinear=True, amp=600.0)]
    bp = P.BatchProblem(handle(), designs)
    prm = P.problem_params(designs[0], max_newton=1, tol_newton=1e-15, no_predictor=1)
    with pytest.raises(P.PPCError) as ei:
        bp.solve(prm)
    banner(f"batch: {ei.value}")
    assert ei.value.code == -7 and "design 1" in str(ei.value)
    bp.close()


def test_nonlinear_coarse_reports_a_failed_harmonic_solve():
    """Nonlinear coarse problem (coarse_mode 1) with fine results F = U + J whose field
    overflows the B-H law of the sheath: the frozen linearisation at F (lin_point 1) is
    not finite, so the preconditioner's harmonic solves report a non-finite residual or a
    breakdown, which the correction must name instead of running GMRES on NaN.  The
    coarse residual itself stays finite (F enters it linearly), and every kernel exits."""
    import paper_1905_13076_amd as P
    from oracle.fe import FE
    from tests.gpu_common import load_golden
    prob = coax.c5_small()
    fe = FE(prob)
    U = load_golden("c5small_nlc")["U_k"]
    pr = P.Problem(handle(), prob)
    prm = P.problem_params(prob, coarse_mode=1, lin_point=1, tol_cocg=1e-6, tol_newton=1e-10)
    with pytest.raises(P.PPCError) as ei:
        pr.coarse_correction(prm, torch.tensor(fe.full(U), device="cuda"),
                             torch.tensor(fe.full(40.0 * U), device="cuda"))
    banner(f"nonlinear coarse: {ei.value}")
    assert ei.value.code in (-5, -6) and "preconditioner" in str(ei.value)
    # the problem stays usable: the same call with finite data succeeds
    pr.coarse_correction(prm, torch.tensor(fe.full(U), device="cuda"),
                         torch.tensor(fe.full(0.01 * U), device="cuda"))

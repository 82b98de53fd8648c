"""Nonlinear periodic coarse problem (params.coarse_mode = 1): the correction of eq. (4)
with the implicit-Euler coarse step on the full K(u), solved on the GPU by Newton with
flexible GMRES preconditioned by the frozen harmonic solve.  GPU against the oracle's
nonlinear_coarse_correction (exact Newton, direct solves): one correction from stored
oracle samples, the linear case, a whole solve against the stored fixed point and
iteration count, and the rejections."""
import numpy as np
import pytest

from workloads import coax
from tests.gpu_common import banner, free_rows, handle, load_golden, rel

pytestmark = pytest.mark.gpu


def test_c5small_nonlinear_correction_matches_oracle():
    """From the oracle's iterate U^2 and its fine results F^2 (saturating sheath), the GPU
    correction equals the oracle's."""
    import torch
    import paper_1905_13076_amd as P
    from oracle.fe import FE
    prob = coax.c5_small()
    fe = FE(prob)
    g = load_golden("c5small_nlc")
    U, Fk, dUo = g["U_k"], g["F_k"], g["dU_k"]
    pr = P.Problem(handle(), prob)
    prm = P.problem_params(prob, coarse_mode=1, tol_cocg=1e-12, tol_newton=1e-13)
    banner("c5small nonlinear correction")
    dU, cocg = pr.coarse_correction(prm, torch.tensor(fe.full(U), device="cuda"),
                                    torch.tensor(fe.full(Fk - U), device="cuda"))
    e = rel(free_rows(dU.cpu().numpy(), fe.free), dUo)
    banner(f"  rel={e:.2e} |dU|/|U|={np.linalg.norm(dUo) / np.linalg.norm(U):.2e} "
           f"cocg per harmonic {np.asarray(cocg).tolist()}")
    assert e <= 1e-9
    assert np.all(np.asarray(cocg) > 0)


def test_c1_nonlinear_correction_of_a_linear_problem_matches_oracle():
    """Linear materials (C1), seeded samples and jumps: the nonlinear coarse problem is the
    linear block-cyclic one, reached in one Newton step."""
    import torch
    import paper_1905_13076_amd as P
    from oracle import periodic
    from oracle.fe import FE
    prob = coax.c1()
    fe = FE(prob)
    rng = np.random.default_rng(17)
    U = rng.standard_normal((prob.N, fe.n)) * 1e-4
    J = rng.standard_normal((prob.N, fe.n)) * 1e-6
    dUo = periodic.nonlinear_coarse_correction(fe, U, U + J)
    pr = P.Problem(handle(), prob)
    prm = P.problem_params(prob, coarse_mode=1, tol_cocg=1e-12, tol_newton=1e-13)
    banner("c1 nonlinear correction (linear materials)")
    dU, cocg = pr.coarse_correction(prm, torch.tensor(fe.full(U), device="cuda"),
                                    torch.tensor(fe.full(J), device="cuda"))
    e = rel(free_rows(dU.cpu().numpy(), fe.free), dUo)
    banner(f"  rel={e:.2e}")
    assert e <= 1e-9


def test_c5small_solve_with_the_nonlinear_coarse_problem_matches_oracle():
    """Whole PP-PC solve with the nonlinear coarse problem: the stored oracle fixed point (the
    same periodic state as the frozen coarse problem's) and its iteration count."""
    import paper_1905_13076_amd as P
    from oracle.fe import FE
    prob = coax.c5_small()
    fe = FE(prob)
    g = load_golden("c5small_nlc")
    gf = load_golden("c5small")
    banner("c5small solve, nonlinear coarse problem")
    pr = P.Problem(handle(), prob)
    prm = P.problem_params(prob, coarse_mode=1)
    U, eps, k, st, rc = pr.solve(prm)
    assert rc == 0, st
    Ug = free_rows(U.cpu().numpy(), fe.free)
    e = rel(Ug, g["U"])
    banner(f"  iters={k} (oracle {int(g['iterations'])}) rel={e:.2e} newton={st['coarse_newton']} "
           f"krylov={st['coarse_krylov']} cocg={st['cocg_total']} coarse_ms={st['coarse_ms']:.1f}")
    assert e <= 1e-10
    assert rel(Ug, gf["U"]) <= 1e-10
    assert abs(k - int(g["iterations"])) <= 1
    assert st["coarse_newton"] >= k and st["coarse_krylov"] >= st["coarse_newton"]


def test_nonlinear_coarse_problem_rejects_batched_problems():
    import paper_1905_13076_amd as P
    probs = [coax.tiny(nr=4, ntheta=8, N=4, m=3, nonlinear=True, amp=300.0),
             coax.tiny(nr=5, ntheta=10, N=4, m=3, nonlinear=True, amp=300.0)]
    bp = P.BatchProblem(handle(), probs)
    banner("batched problem, coarse_mode 1")
    with pytest.raises(Exception, match="coarse_mode"):
        bp.solve(P.problem_params(probs[0], coarse_mode=1))

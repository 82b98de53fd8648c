"""Truncated harmonic set (params.n_harm): each correction solves only the first n_harm
harmonics and takes the jumps' harmonics for the rest.  GPU against the oracle's
ppc(n_harm=...): one correction, whole solves (iteration counts and eps histories), the
fixed point (unchanged by the truncation), and batched solves equal to single ones."""
import numpy as np
import pytest

from workloads import coax
from tests.gpu_common import banner, free_rows, handle, load_golden, rel

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n_harm", [1, 3, 5])
def test_c1_truncated_correction_matches_oracle(n_harm):
    import torch
    import paper_1905_13076_amd as P
    from oracle import periodic
    from oracle.fe import FE
    prob = coax.c1()
    fe = FE(prob)
    rng = np.random.default_rng(11)
    U = rng.standard_normal((prob.N, fe.n)) * 1e-4
    J = rng.standard_normal((prob.N, fe.n)) * 1e-6
    dUo = periodic.coarse_correction(fe, U, J, n_harm=n_harm)
    pr = P.Problem(handle(), prob)
    prm = P.problem_params(prob, n_harm=n_harm, tol_cocg=1e-13)
    banner(f"c1 correction n_harm={n_harm}")
    dU, cocg = pr.coarse_correction(prm, torch.tensor(fe.full(U), device="cuda"),
                                    torch.tensor(fe.full(J), device="cuda"))
    e = rel(free_rows(dU.cpu().numpy(), fe.free), dUo)
    banner(f"  rel={e:.2e} cocg per harmonic {np.asarray(cocg).tolist()}")
    # the bar of the full correction test: the solved harmonics carry the COCG tolerance
    # times their conditioning, the others are exact DFTs of J
    assert e <= 1e-10
    assert np.all(np.asarray(cocg)[n_harm:] == 0) and np.all(np.asarray(cocg)[:n_harm] > 0)


def test_c1_five_harmonics_solve_matches_oracle():
    """C1 with 5 of its 6 coarse harmonics (N = 10): same iterations and eps history as
    the oracle, and the exact periodic solution (route L)."""
    import paper_1905_13076_amd as P
    from oracle import periodic
    from oracle.fe import FE
    prob = coax.c1()
    fe = FE(prob)
    UL, _ = periodic.route_l(fe)
    Uo, ho, ko = periodic.ppc(fe, tol=1e-12, n_harm=5)
    pr = P.Problem(handle(), prob)
    U, eps, k, st, rc = pr.solve(P.problem_params(prob, n_harm=5))
    assert rc == 0
    Ug = free_rows(U.cpu().numpy(), fe.free)
    banner(f"c1 n_harm=5: iters {k} (oracle {ko}) rel vs oracle {rel(Ug, Uo):.2e} vs route L {rel(Ug, UL):.2e}")
    assert rel(Ug, Uo) <= 1e-10 and rel(Ug, UL) <= 1e-10
    assert abs(k - ko) <= 1
    L = min(len(eps), len(ho))
    # fine steps are solved to Newton 1e-13 of their scale: jumps agree to that level
    np.testing.assert_allclose(eps[:L], ho[:L], rtol=1e-6, atol=1e-13)


def test_c5small_three_harmonics_matches_oracle():
    import paper_1905_13076_amd as P
    from oracle.fe import FE
    prob = coax.c5_small()
    fe = FE(prob)
    g = load_golden("c5small_h3")
    full = load_golden("c5small")
    pr = P.Problem(handle(), prob)
    U, eps, k, st, rc = pr.solve(P.problem_params(prob, n_harm=3))
    assert rc == 0
    Ug = free_rows(U.cpu().numpy(), fe.free)
    banner(f"c5small n_harm=3: iters {k} (oracle {int(g['iterations'])}) rel {rel(Ug, g['U']):.2e} "
           f"vs full-set fixed point {rel(Ug, full['U']):.2e}; cocg {st['cocg_total']}")
    assert rel(Ug, g["U"]) <= 1e-10 and rel(Ug, full["U"]) <= 1e-10
    assert abs(k - int(g["iterations"])) <= 1


def test_batched_truncated_solves_equal_single_solves():
    import paper_1905_13076_amd as P
    designs = [coax.tiny(nr=6, ntheta=12, N=8, m=6, nonlinear=True, amp=400.0),
               coax.tiny(nr=8, ntheta=16, N=8, m=6, nonlinear=False),
               coax.tiny(nr=30, ntheta=48, N=8, m=6, nonlinear=True, amp=600.0)]
    prm = P.problem_params(designs[0], n_harm=2)
    bp = P.BatchProblem(handle(), designs)
    Us, resid, iters, st, rc = bp.solve(prm)
    assert rc == 0, st
    for d, prob in enumerate(designs):
        pr = P.Problem(handle(), prob)
        U, eps, k, st1, rc1 = pr.solve(prm)
        assert rc1 == 0
        diff = float(np.abs(Us[d].cpu().numpy() - U.cpu().numpy()).max())
        banner(f"batch n_harm=2 design {d}: iters {iters[d]} vs {k}, max|diff| {diff:.1e}")
        assert iters[d] == k and diff == 0.0
        pr.close()
    bp.close()

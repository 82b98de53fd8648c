"""PP-IC (eq. (5): U_0^{k+1} = U_N^k, sequential implicit-Euler coarse propagation of
eq. (8) on the frozen coarse stiffness at U^k) on the GPU against the CPU oracle's PP-IC:
the same fixed point as PP-PC, the same iteration history, and graph replay equal to
eager launches bitwise."""
import numpy as np
import pytest

from workloads import coax
from tests.gpu_common import banner, free_rows, handle, load_golden, rel

pytestmark = pytest.mark.gpu


def test_c1_ppic_matches_oracle():
    """C1 (linear coax, N = 10 x 20, FP64), both from the linear coarse periodic start."""
    import paper_1905_13076_amd as P
    from oracle.fe import FE
    from oracle import periodic
    prob = coax.c1()
    fe = FE(prob)
    Uo, ho, ko = periodic.ppic(fe, tol=1e-12)
    banner("c1 ppic fp64")
    pr = P.Problem(handle(), prob)
    U, eps, k, st, rc = pr.solve(P.problem_params(prob, method=1))
    assert rc == 0, st
    e = rel(free_rows(U.cpu().numpy(), fe.free), Uo)
    banner(f"c1 ppic: iters={k} (oracle {ko}) rel={e:.2e} coarse solves {st['coarse_solves']} "
           f"cocg {st['cocg_total']}")
    assert e <= 1e-10
    assert abs(k - ko) <= 1
    # N sequential solves per correction, plus the coarse periodic solve of the start
    assert st["coarse_solves"] == k * prob.N + 1
    L = min(len(eps), len(ho))
    # fine steps are solved to Newton 1e-13 of their scale: jumps agree to that level
    np.testing.assert_allclose(eps[:L], ho[:L], rtol=1e-6, atol=1e-13)
    # PP-PC reaches the same periodic state
    Up, _, kp, stp, rcp = pr.solve(P.problem_params(prob))
    assert rcp == 0 and rel(free_rows(Up.cpu().numpy(), fe.free), Uo) <= 1e-10
    banner(f"c1: PP-IC {k} iterations, PP-PC {kp}")


def test_c5small_ppic_from_rest_matches_oracle():
    """Nonlinear c5small from the fine sweep from rest (init_mode 3 and the oracle's
    initial_iterate "fine"): PP-IC fixed point, iteration count and eps history."""
    import paper_1905_13076_amd as P
    from oracle.fe import FE
    prob = coax.c5_small()
    fe = FE(prob)
    g = load_golden("c5small_ppic")
    banner("c5small ppic from rest")
    pr = P.Problem(handle(), prob)
    U, eps, k, st, rc = pr.solve(P.problem_params(prob, method=1, init_mode=3))
    assert rc == 0, st
    e = rel(free_rows(U.cpu().numpy(), fe.free), g["U"])
    banner(f"c5small ppic: iters={k} (oracle {int(g['iterations'])}) rel={e:.2e} "
           f"eps {np.asarray(eps)[:4]} vs {g['hist'][:4]}")
    assert e <= 1e-10
    assert abs(k - int(g["iterations"])) <= 1
    # the early history, far above the solver tolerances, agrees closely
    L = min(len(eps), len(g["hist"]))
    h = g["hist"][:L]
    big = h > 1e-6
    np.testing.assert_allclose(np.asarray(eps)[:L][big], h[big], rtol=1e-6)


def test_ppic_graph_replay_equals_eager():
    import paper_1905_13076_amd as P
    prob = coax.c1()
    pr = P.Problem(handle(), prob)
    out = []
    for graph in (0, 1, 1):
        banner(f"ppic graph={graph}")
        U, eps, k, st, rc = pr.solve(P.problem_params(prob, method=1, graph=graph))
        assert rc == 0
        out.append((U.cpu().numpy(), np.asarray(eps), k, st["cocg_total"]))
    for Ug, epsg, kg, cg in out[1:]:
        assert kg == out[0][2] and cg == out[0][3]
        assert float(np.abs(Ug - out[0][0]).max()) == 0.0
        np.testing.assert_array_equal(epsg, out[0][1])


def test_ppic_rejected_for_batches():
    import paper_1905_13076_amd as P
    probs = [coax.tiny(nr=4, ntheta=8, N=4, m=3), coax.tiny(nr=5, ntheta=10, N=4, m=3)]
    bp = P.BatchProblem(handle(), probs)
    with pytest.raises(P.PPCError, match="PP-IC"):
        bp.solve(P.problem_params(probs[0], method=1))


def test_c2lin_small_ppic_and_ppc_match_oracle():
    """Linearised C2 (steel at its unsaturated reluctivity; 20 x 40, N = 10 x 20): the
    sheath's time constant makes PP-IC slow, PP-PC fast -- the contrast of the paper's
    Section 4 -- and both GPU runs follow the oracle's iteration counts to its fixed point."""
    import paper_1905_13076_amd as P
    from oracle.fe import FE
    prob = coax.c2lin(nr=20, ntheta=40, N=10, m=20)
    fe = FE(prob)
    pr = P.Problem(handle(), prob)
    res = {}
    for name, kw in (("c2lin_small", {}), ("c2lin_small_ppic", dict(method=1, max_iters=300))):
        g = load_golden(name)
        banner(f"{name}")
        U, eps, k, st, rc = pr.solve(P.problem_params(prob, **kw))
        assert rc == 0, st
        e = rel(free_rows(U.cpu().numpy(), fe.free), g["U"])
        banner(f"{name}: iters={k} (oracle {int(g['iterations'])}) rel={e:.2e}")
        assert e <= 1e-10
        assert abs(k - int(g["iterations"])) <= 1
        res[name] = k
    assert res["c2lin_small_ppic"] >= 5 * res["c2lin_small"]

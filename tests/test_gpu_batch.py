"""Batched designs on the GPU: one batched PP-PC solve of several designs of uneven size
equals the per-design solves exactly (same kernels, same arithmetic), and every design
matches the FP64 oracle."""
import numpy as np
import pytest

from workloads import coax
from tests.gpu_common import banner, handle, rel

pytestmark = pytest.mark.gpu


def _designs():
    """Uneven sizes, both initial-iterate rules (linear and Brauer designs) and several
    kernel shapes (register rows R = 1, 2, 4 and the LDS memory path)."""
    out = [
        coax.tiny(nr=6, ntheta=12, N=8, m=6, nonlinear=True, amp=400.0),
        coax.tiny(nr=8, ntheta=16, N=8, m=6, nonlinear=False),
        coax.tiny(nr=12, ntheta=24, N=8, m=6, nonlinear=True, amp=300.0, sheath_sigma=5e5),
        coax.tiny(nr=30, ntheta=48, N=8, m=6, nonlinear=True, amp=600.0),
        coax.tiny(nr=48, ntheta=96, N=8, m=6, nonlinear=True, amp=250.0),
        coax.tiny(nr=90, ntheta=100, N=8, m=6, nonlinear=True, amp=500.0),
    ]
    return out


@pytest.mark.parametrize("prec,init", [(0, 0), (1, 0), (0, 3), (0, 4)])
def test_batch_equals_single_design_solves(prec, init):
    import paper_1905_13076_amd as P
    designs = _designs()
    prm = P.problem_params(designs[0], precision=prec, tol_lin=1e-8 if prec == 0 else 1e-4, init_mode=init)
    singles = []
    for d, prob in enumerate(designs):
        banner(f"batch: single design {d} n_nodes={prob.n_nodes} prec={prec}")
        pr = P.Problem(handle(), prob)
        U, eps, k, st, rc = pr.solve(prm)
        assert rc == 0, (d, st)
        singles.append((U.cpu().numpy(), k, eps))
        pr.close()
    banner(f"batch: {len(designs)} designs in one batched problem prec={prec}")
    bp = P.BatchProblem(handle(), designs)
    Us, resid, iters, st, rc = bp.solve(prm)
    assert rc == 0, st
    for d in range(len(designs)):
        Ub = Us[d].cpu().numpy()
        Us_, k, eps = singles[d]
        diff = float(np.abs(Ub - Us_).max())
        banner(f"batch design {d}: iters batch={iters[d]} single={k} max|diff|={diff:.1e}")
        assert iters[d] == k
        assert diff == 0.0
        np.testing.assert_array_equal(resid[d, : k + 1], eps)
    bp.close()


def test_batch_designs_match_oracle():
    import paper_1905_13076_amd as P
    from oracle import periodic
    from oracle.fe import FE
    designs = _designs()[:4]
    prm = P.problem_params(designs[0])
    bp = P.BatchProblem(handle(), designs)
    banner("batch vs oracle")
    Us, resid, iters, st, rc = bp.solve(prm)
    assert rc == 0
    for d, prob in enumerate(designs):
        fe = FE(prob)
        Uo, _, ko = periodic.ppc(fe, tol=1e-12)
        e = rel(Us[d].cpu().numpy()[:, fe.free], Uo)
        banner(f"batch design {d}: iters={iters[d]} oracle={ko} rel={e:.2e}")
        assert e <= 1e-10


def test_batch_c4_designs_subset_runs_and_agrees_with_single():
    """Designs of the batched-designs generator (uneven nr, sheath thickness, conductivity,
    Brauer k2 and current) on a short time grid: batched and single solves agree exactly.
    The subset keeps the designs with nr <= 60 among the first 24 (nr 24..59)."""
    import paper_1905_13076_amd as P
    designs = [p for p in coax.c4_designs(n_designs=24, N=4, m=3) if p.meta["nr"] <= 60]
    prm = P.problem_params(designs[0], tol_ppc=1e-8, precision=1, tol_lin=1e-4)
    bp = P.BatchProblem(handle(), designs)
    banner("batch: C4 subset " + str([p.meta["nr"] for p in designs]))
    Us, resid, iters, st, rc = bp.solve(prm)
    assert rc == 0
    for d, prob in enumerate(designs):
        pr = P.Problem(handle(), prob)
        U, eps, k, _, rc1 = pr.solve(prm)
        assert rc1 == 0
        diff = float(np.abs(Us[d].cpu().numpy() - U.cpu().numpy()).max())
        banner(f"C4 design {d} nr={prob.meta['nr']}: iters {iters[d]} vs {k}, max|diff|={diff:.1e}")
        assert iters[d] == k and diff == 0.0
        pr.close()
    bp.close()


def test_generator_subset_matches_oracle():
    """The 8 smallest and 4 seeded designs of the batched-designs generator (short grid,
    N = 8 x 10), batched on the GPU from rest with the 3 T safeguard, against the oracle's
    PP-PC of each design with the same start and safeguard."""
    import paper_1905_13076_amd as P
    from oracle.fe import FE
    from tests.golden.make_reference import C4_SUBSET, c4_subset
    from tests.gpu_common import load_golden
    g = load_golden("c4subset")
    designs = c4_subset()
    bp = P.BatchProblem(handle(), designs)
    prm = P.problem_params(designs[0], tol_ppc=1e-12, init_mode=3, b_cap=3.0, max_iters=200)
    banner(f"generator subset: {len(designs)} designs")
    Us, resid, iters, st, rc = bp.solve(prm)
    assert rc == 0, st
    worst = 0.0
    for j, (i, prob) in enumerate(zip(C4_SUBSET, designs)):
        fe = FE(prob)
        Uo = g[f"U_{i}"]
        e = rel(Us[j].cpu().numpy()[:, fe.free], Uo)
        ko = int(g[f"iterations_{i}"])
        banner(f"  design {i} nr={prob.meta['nr']}: iters {iters[j]} (oracle {ko}) rel {e:.2e}")
        assert e <= 1e-10
        assert abs(int(iters[j]) - ko) <= 1
        worst = max(worst, e)
    banner(f"  worst rel {worst:.2e}; corrections scaled by the safeguard: {st['damped']}")
    bp.close()

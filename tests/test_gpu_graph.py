"""PP-PC iterations replayed as HIP graphs (the default) against eager launches: the same
kernels in the same order, so every replayed iteration must reproduce the eager run
bitwise (iterate, eps history, counters).  Graph solves are repeated with eager work and
synchronisations in between; each solve captures its own graphs."""
import numpy as np
import pytest

from workloads import coax
from tests.gpu_common import banner, handle

pytestmark = pytest.mark.gpu


def _solve(pr, prm, graph):
    prm.graph = graph
    U, eps, k, st, rc = pr.solve(prm)
    assert rc == 0, st
    return U.cpu().numpy(), np.asarray(eps), k, st


@pytest.mark.parametrize("name", ["c1", "c5small", "c2"])
def test_graph_replay_equals_eager(name):
    import torch
    import paper_1905_13076_amd as P
    prob = {"c1": coax.c1, "c5small": coax.c5_small, "c2": coax.c2}[name]()
    kw = {"tol_ppc": 1e-8, "tol_cocg": 1e-6} if name == "c2" else {}
    pr = P.Problem(handle(), prob)
    prm = P.problem_params(prob, **kw)
    banner(f"graph vs eager: {name} eager")
    Ue, epse, ke, ste = _solve(pr, prm, 0)
    for rep in range(2):
        banner(f"graph vs eager: {name} graph solve {rep}")
        Ug, epsg, kg, stg = _solve(pr, prm, 1)
        d = float(np.abs(Ug - Ue).max())
        banner(f"{name} graph solve {rep}: iters {kg} vs {ke}, max|dU|={d:.1e}, "
               f"fine ms {stg['fine_ms']:.1f} vs {ste['fine_ms']:.1f}")
        assert kg == ke and d == 0.0
        np.testing.assert_array_equal(epsg, epse)
        for key in ("newton_total", "lin_total", "resid_total", "cocg_total", "fine_launches"):
            assert stg[key] == ste[key], key
        # eager work on the same problem between graph solves
        Ud = torch.tensor(Ue, device="cuda")
        F, nw, lin = pr.fine_sweep(prm, Ud)
        torch.cuda.synchronize()
        assert np.isfinite(F.cpu().numpy()).all()


@pytest.mark.parametrize("b_cap", [0.0, 1.5])
def test_batched_graph_replay_equals_eager(b_cap):
    """Batched designs converging at different iterations: the captured graphs are
    re-captured whenever the set of active (or corrected) designs shrinks, and every
    replay reproduces the eager launches bitwise (iterates, eps histories, counters)."""
    import paper_1905_13076_amd as P
    designs = [coax.tiny(nr=6, ntheta=12, N=8, m=6, nonlinear=True, amp=400.0),
               coax.tiny(nr=8, ntheta=16, N=8, m=6, nonlinear=False),
               coax.tiny(nr=12, ntheta=24, N=8, m=6, nonlinear=True, amp=300.0, sheath_sigma=5e5),
               coax.tiny(nr=30, ntheta=48, N=8, m=6, nonlinear=True, amp=600.0)]
    bp = P.BatchProblem(handle(), designs)
    prm = P.problem_params(designs[0], b_cap=b_cap)
    runs = []
    for graph in (0, 1, 1):
        prm.graph = graph
        banner(f"batched graph={graph} b_cap={b_cap}")
        Us, resid, iters, st, rc = bp.solve(prm)
        assert rc == 0, st
        runs.append(([u.cpu().numpy() for u in Us], resid.copy(), np.asarray(iters).copy(), st))
    Ue, re_, ie, ste = runs[0]
    assert len(set(ie.tolist())) > 1          # the active set shrinks along the way
    for Ug, rg, ig, stg in runs[1:]:
        assert np.array_equal(ig, ie)
        for a, b in zip(Ug, Ue):
            assert float(np.abs(a - b).max()) == 0.0
        np.testing.assert_array_equal(rg, re_)
        for key in ("newton_total", "lin_total", "resid_total", "cocg_total", "fine_launches", "damped"):
            assert stg[key] == ste[key], key
    bp.close()

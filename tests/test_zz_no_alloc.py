"""The allocation-free fine sweep (ppc_fine_sweep_noalloc) against the allocating one
(ppc_fine_sweep_device): two calls in a row through the C-ABI, the second on a smaller
problem in the other precision, each bitwise equal to the allocating entry point with the
same per-chain counters; and the size checks that reject a sweep the static scratch
cannot hold, before any device work."""
import numpy as np
import pytest

from workloads import coax
from tests.gpu_common import banner, handle, load_golden

pytestmark = pytest.mark.gpu


def _start(prob, pr, name):
    """Chain starts: the stored oracle fixed point (nodal rows, Dirichlet nodes 0)."""
    import torch
    g = load_golden(name)
    U = np.zeros((prob.N, pr.n_nodes))
    U[:, g["free"]] = g["U"]
    return torch.tensor(U, device="cuda")


def test_noalloc_fine_sweep_equals_the_allocating_sweep():
    import torch
    import paper_1905_13076_amd as P
    h = handle()
    cases = [(coax.c2(), "c2", 0), (coax.c5_small(), "c5small", 1)]   # larger first, then smaller
    for prob, name, prec in cases:
        pr = P.Problem(h, prob)
        prm = P.problem_params(prob, precision=prec, tol_newton=1e-10)
        U = _start(prob, pr, name)
        banner(f"no-alloc fine sweep: {name} N={prob.N} n_free={pr.n_free} precision={prec}")
        Fa, na, la = pr.fine_sweep(prm, U)
        Fb, nb, lb = pr.fine_sweep_noalloc(prm, U)
        torch.cuda.synchronize()
        diff = float((Fa - Fb).abs().max())
        banner(f"  max |F_alloc - F_noalloc| = {diff:.3e}; newton {int(na.sum())} / {int(nb.sum())}, "
               f"pcg {int(la.sum())} / {int(lb.sum())}")
        assert torch.equal(Fa, Fb)
        assert np.array_equal(na, nb) and np.array_equal(la, lb)
        assert int(na.sum()) > 0 and bool(torch.isfinite(Fb).all())
        pr.close()


def test_noalloc_rejects_sweeps_beyond_its_scratch():
    import torch
    import paper_1905_13076_amd as P
    prob = coax.c2()
    pr = P.Problem(handle(), prob)
    for N, m in ((400, 5), (2048, 1)):
        prm = P.params(T=prob.T, N=N, m=m)
        U = torch.zeros((N, pr.n_nodes), dtype=torch.float64, device="cuda")
        with pytest.raises(P.PPCError) as ei:
            pr.fine_sweep_noalloc(prm, U)
        banner(f"  N={N}: {ei.value}")
        assert ei.value.code == -1
    pr.close()

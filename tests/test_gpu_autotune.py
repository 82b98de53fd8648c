"""The fine-sweep autotuner and the register-row workgroup sizes it chooses between:
every size (256, 512, 1024 threads) matches the oracle's fine sweep; a tuned solve matches
the oracle's fixed point; a tuned batch (size classes) equals per-design solves forced to
the same sizes, bitwise; a mesh whose rows only fit 1024 threads reports that."""
import math

import numpy as np
import pytest

from workloads import coax
from tests.gpu_common import banner, free_rows, handle, load_golden, rel

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", [0, 1])
def test_every_register_block_matches_oracle_fine_sweep(prec):
    import torch
    import paper_1905_13076_amd as P
    from oracle import periodic
    from oracle.fe import FE
    prob = coax.c5_small()
    fe = FE(prob)
    g = load_golden("c5small")
    starts = {"zero": np.zeros((prob.N, fe.n)), "periodic": g["U"]}
    pr = P.Problem(handle(), prob)
    for name, U0 in starts.items():
        Fo = periodic.fine_sweep(fe, U0)
        Ud = torch.tensor(fe.full(U0), device="cuda")
        outs = {}
        for fb in (256, 512, 1024):
            banner(f"c5small fine sweep from {name}, fine_block {fb}, precision {prec}")
            prm = P.problem_params(prob, precision=prec, fine_block=fb)
            F, nw, lin = pr.fine_sweep(prm, Ud)
            Fg = free_rows(F.cpu().numpy(), fe.free)
            e = rel(Fg, Fo)
            banner(f"  rel={e:.2e} newton={int(np.sum(nw))} pcg={int(np.sum(lin))}")
            assert e <= 1e-11
            outs[fb] = Fg
        # the sizes differ only in reduction order
        assert rel(outs[256], outs[1024]) <= 1e-11


def test_autotuned_solve_matches_oracle():
    import paper_1905_13076_amd as P
    from oracle.fe import FE
    prob = coax.c5_small()
    fe = FE(prob)
    g = load_golden("c5small")
    pr = P.Problem(handle(), prob)
    prm = P.problem_params(prob)
    banner("autotune c5small fp64")
    b, ms = pr.autotune(prm)
    banner(f"  chosen {b}, ms {ms}")
    assert b in (256, 512, 1024)
    assert all(math.isfinite(x) and x > 0 for x in ms)      # 761 rows fit every size
    assert ms[[256, 512, 1024].index(b)] == np.min(ms)
    U, eps, k, st, rc = pr.solve(prm)
    assert rc == 0
    e = rel(free_rows(U.cpu().numpy(), fe.free), g["U"])
    banner(f"  tuned solve: iters {k} (oracle {int(g['iterations'])}) rel {e:.2e}")
    assert e <= 1e-10 and abs(k - int(g["iterations"])) <= 1


def test_autotuned_batch_equals_forced_single_solves():
    import paper_1905_13076_amd as P
    designs = [
        coax.tiny(nr=12, ntheta=24, N=8, m=6, nonlinear=True, amp=300.0, sheath_sigma=5e5),
        coax.tiny(nr=24, ntheta=48, N=8, m=6, nonlinear=True, amp=600.0),
        coax.tiny(nr=25, ntheta=48, N=8, m=6, nonlinear=True, amp=400.0),
        coax.tiny(nr=40, ntheta=80, N=8, m=6, nonlinear=True, amp=250.0),
    ]
    prm = P.problem_params(designs[0])
    bp = P.BatchProblem(handle(), designs)
    banner("autotune batch")
    blocks, ms = bp.autotune(prm)
    banner(f"  blocks {blocks.tolist()}")
    # one policy over the batched sweep: the policy times are the same for every design, and
    # designs 1 and 2 (1,105 and 1,153 free rows) share a size class and so a size
    assert blocks[1] == blocks[2]
    assert np.all(ms == ms[0]) and set(blocks.tolist()) <= {256, 512, 1024}
    # the largest design (3,121 rows) does not fit 256 threads: at least 512
    assert blocks[3] >= 512
    Us, resid, iters, st, rc = bp.solve(prm)
    assert rc == 0, st
    for d, prob in enumerate(designs):
        pr = P.Problem(handle(), prob)
        U, eps, k, st1, rc1 = pr.solve(P.problem_params(prob, fine_block=int(blocks[d])))
        assert rc1 == 0
        diff = float(np.abs(Us[d].cpu().numpy() - U.cpu().numpy()).max())
        banner(f"  design {d} block {blocks[d]}: iters {iters[d]} vs {k}, max|diff| {diff:.1e}")
        assert iters[d] == k and diff == 0.0
        pr.close()
    bp.close()


def test_c2_rows_fit_only_1024_threads():
    import paper_1905_13076_amd as P
    prob = coax.c2()
    pr = P.Problem(handle(), prob)
    prm = P.problem_params(prob, tol_cocg=1e-6)
    b, ms = pr.autotune(prm)
    banner(f"autotune c2: {b} {ms}")
    assert b == 1024 and math.isnan(ms[0]) and math.isnan(ms[1]) and ms[2] > 0
    with pytest.raises(P.PPCError, match="fine_block"):
        import torch
        pr.fine_sweep(P.problem_params(prob, fine_block=512),
                      torch.zeros((prob.N, pr.n_nodes), dtype=torch.float64, device="cuda"))

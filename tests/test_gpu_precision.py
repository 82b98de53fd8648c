"""Precision policy on the GPU: the mixed form (FP32 Jacobian and PCG, complex-FP32
COCG, each refined by FP64 residuals; FP64 Newton residual, jumps, DFTs and state)
against the all-FP64 GPU run and the FP64 oracle.  Bar: 1e-6 relative."""
import numpy as np
import pytest

from workloads import coax
from tests.gpu_common import banner, free_rows, handle, load_golden, rel

pytestmark = pytest.mark.gpu


def test_mixed_coarse_correction_matches_oracle():
    import torch
    import paper_1905_13076_amd as P
    from oracle.fe import FE
    from oracle import periodic
    prob = coax.c5_small()
    fe = FE(prob)
    U = load_golden("c5small")["U"]
    rng = np.random.default_rng(7)
    J = 1e-3 * np.abs(U).max() * rng.standard_normal(U.shape)
    dUo = periodic.coarse_correction(fe, U, J)
    pr = P.Problem(handle(), prob)
    out = {}
    for prec in (0, 1):
        prm = P.problem_params(prob, precision=prec, tol_cocg=1e-12)
        dU, cocg = pr.coarse_correction(prm, torch.tensor(fe.full(U), device="cuda"),
                                        torch.tensor(fe.full(J), device="cuda"))
        out[prec] = (rel(free_rows(dU.cpu().numpy(), fe.free), dUo), cocg)
    banner(f"coarse correction fp64 rel={out[0][0]:.1e} cocg={out[0][1].tolist()}; "
           f"mixed rel={out[1][0]:.1e} cocg={out[1][1].tolist()}")
    assert out[0][0] <= 1e-10 and out[1][0] <= 1e-10


def test_c2_mixed_matches_fp64_gpu_and_oracle():
    """The benchmark workload in both forms at the benchmark tolerance."""
    import paper_1905_13076_amd as P
    from oracle.fe import FE
    prob = coax.c2()
    fe = FE(prob)
    g = load_golden("c2")
    pr = P.Problem(handle(), prob)
    res = {}
    for prec in (0, 1):
        prm = P.problem_params(prob, tol_ppc=1e-8, precision=prec, tol_lin=1e-8 if prec == 0 else 1e-4)
        banner(f"c2 precision={prec}")
        U, eps, k, st, rc = pr.solve(prm)
        assert rc == 0
        res[prec] = (free_rows(U.cpu().numpy(), fe.free), k, st)
    e_mix_fp64 = rel(res[1][0], res[0][0])
    e_mix_orc = rel(res[1][0], g["U"])
    e_fp64_orc = rel(res[0][0], g["U"])
    banner(f"c2: iters fp64={res[0][1]} mixed={res[1][1]}; mixed vs fp64-GPU {e_mix_fp64:.1e}, "
           f"mixed vs oracle {e_mix_orc:.1e}, fp64 vs oracle {e_fp64_orc:.1e}; "
           f"fine ms fp64={res[0][2]['fine_ms']:.0f} mixed={res[1][2]['fine_ms']:.0f}; "
           f"coarse ms fp64={res[0][2]['coarse_ms']:.0f} mixed={res[1][2]['coarse_ms']:.0f}")
    assert e_mix_fp64 <= 1e-6 and e_mix_orc <= 1e-6 and e_fp64_orc <= 1e-6


def test_c5_mixed_fine_fp64_coarse_and_fine_counts():
    """FP32 fine solves with FP64 harmonic solves (coarse_precision = 0) reach the oracle's
    fixed point; the last sweep's per-chain counters are consistent with the solve's."""
    import paper_1905_13076_amd as P
    from oracle.fe import FE
    prob = coax.c5_small()
    fe = FE(prob)
    g = load_golden("c5small")
    pr = P.Problem(handle(), prob)
    prm = P.problem_params(prob, tol_ppc=1e-8, precision=1, tol_lin=1e-4, coarse_precision=0)
    banner("c5small mixed fine + fp64 coarse")
    U, eps, k, st, rc = pr.solve(prm)
    assert rc == 0
    e = rel(free_rows(U.cpu().numpy(), fe.free), g["U"])
    cnt = pr.fine_counts(prob.N)
    banner(f"c5small mixed-fine: iters={k} rel={e:.1e} cocg_total={st['cocg_total']} "
           f"last sweep newton={cnt[:, 1].sum()} lin={cnt[:, 2].sum()} resid={cnt[:, 7].sum()}")
    assert e <= 1e-6
    assert (cnt[:, 0] == 0).all() and (cnt[:, 6] == -1).all()
    # every Newton iteration follows a residual evaluation, and every step evaluates one
    assert (cnt[:, 7] >= cnt[:, 1]).all() and (cnt[:, 7] >= prob.m).all()
    assert (cnt[:, 2] >= cnt[:, 1]).all()
    with pytest.raises(P.PPCError):
        pr.fine_counts(prob.N + 2)

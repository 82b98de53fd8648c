"""Pins of the oracle's periodic solvers (Sections 2-3) by brute force, algebraic
identities of the paper and agreement of independent routes."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import periodic
from oracle.fe import FE
from oracle.timestep import fine_propagate
from workloads import coax


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _tiny_nl(**kw):
    args = dict(nr=4, ntheta=8, N=6, m=3, nonlinear=True, amp=300.0)
    args.update(kw)
    return FE(coax.tiny(**args))


def test_dft_block_diagonalises_block_cyclic_G():
    """Eq. (13): the per-harmonic solves of harmonic_solve equal a direct solve with the
    explicit block-cyclic G of eq. (9) (Q on the diagonal, -C below and top-right)."""
    fe = _tiny_nl()
    N, T = fe.prob.N, fe.prob.T
    rng = np.random.default_rng(1)
    U = 2e-3 * rng.standard_normal((N, fe.n))
    Kbar = periodic.coarse_stiffness(fe, U)
    Rr = rng.standard_normal((N, fe.n))
    X1 = periodic.harmonic_solve(fe, Kbar, Rr, T)
    G = periodic.block_cyclic_G(fe, Kbar, N, T)
    X2 = spla.spsolve(G.tocsc(), Rr.ravel()).reshape(N, fe.n)
    assert rel(X1, X2) <= 1e-12


def _coarse_step(fe, Kbar, n, u):
    """Implicit-Euler coarse propagator of eq. (8): Q G = C u + f(T_n)."""
    N, T = fe.prob.N, fe.prob.T
    C = fe.M / (T / N)
    f = periodic.excitation_rows(fe, N, T)[n % N]
    return spla.spsolve((C + Kbar).tocsc(), C @ u + f)


def test_correction_form_equals_literal_eq9():
    """Linear case: U + coarse_correction(J) equals the solution of G U^{k+1} = r^k with
    b^k from eq. (7) and r_n = Q b_n + f(T_n) from eq. (10)."""
    fe = FE(coax.tiny(nr=4, ntheta=8, N=6, m=3))
    N, T = fe.prob.N, fe.prob.T
    rng = np.random.default_rng(2)
    U = 1e-7 * rng.standard_normal((N, fe.n))
    Fs = periodic.fine_sweep(fe, U)
    K = periodic.coarse_stiffness(fe, U)
    Q = fe.M / (T / N) + K
    fr = periodic.excitation_rows(fe, N, T)
    r = np.zeros_like(U)
    for n in range(1, N + 1):                      # row n mod N pairs with subinterval n
        b = Fs[n % N] - _coarse_step(fe, K, n, U[n - 1])
        r[n % N] = Q @ b + fr[n % N]
    G = periodic.block_cyclic_G(fe, K, N, T)
    U_lit = spla.spsolve(G.tocsc(), r.ravel()).reshape(N, fe.n)
    U_cor = U + periodic.coarse_correction(fe, U, Fs - U)
    assert rel(U_cor, U_lit) <= 1e-12
    # the identity behind it: r^k = G U^k + Q J^k
    GU = (G @ U.ravel()).reshape(N, fe.n)
    assert rel(GU + (Q @ (Fs - U).T).T, r) <= 1e-12


def test_coarse_equals_fine_converges_in_one_iteration():
    """m = 1 and linear: the fine propagator is the coarse one, so one correction with the
    exact symbol reaches the periodic solution."""
    fe = FE(coax.tiny(nr=5, ntheta=10, N=8, m=1))
    U, hist, k = periodic.ppc(fe, tol=1e-13)
    assert k <= 1 and hist[-1] <= 1e-13
    UL, _ = periodic.route_l(fe)
    assert rel(U, UL) <= 1e-12


def test_literal_rhs_with_iw_shift_has_wrong_fixed_point():
    """Negative test: iterating the literal eqs. (9)-(10) but with the harmonic-balance
    shift i w_p in place of the implicit-Euler symbol does not reach the fine periodic
    solution, while the correction form with the same shift does."""
    fe = FE(coax.tiny(nr=5, ntheta=10, N=8, m=4))
    N, T = fe.prob.N, fe.prob.T
    UL, _ = periodic.route_l(fe)
    K = periodic.coarse_stiffness(fe, UL)
    Q = fe.M / (T / N) + K
    fr = periodic.excitation_rows(fe, N, T)
    sig = periodic.shifts(N, T, "iw")
    U = np.zeros_like(UL)
    for _ in range(60):
        Fs = periodic.fine_sweep(fe, U)
        r = np.zeros_like(U)
        for n in range(1, N + 1):
            r[n % N] = Q @ (Fs[n % N] - _coarse_step(fe, K, n, U[n - 1])) + fr[n % N]
        Rh = np.fft.rfft(r, axis=0)
        Xh = np.array([spla.spsolve((K + s * fe.M).astype(complex).tocsc(), Rh[p]) for p, s in enumerate(sig)])
        U = np.fft.irfft(Xh, n=N, axis=0)
    assert rel(U, UL) > 1e-4
    Uc, _, _ = periodic.ppc(fe, tol=1e-12, shift="iw")
    assert rel(Uc, UL) <= 1e-10


def test_initial_value_parareal_terminates_after_N_iterations():
    """Classical Parareal with U_0 fixed reproduces the sequential fine solution exactly
    after N iterations (the finite-termination property behind eq. (4))."""
    fe = _tiny_nl(N=5, m=3, amp=20.0)
    N, T, m = fe.prob.N, fe.prob.T, fe.prob.m
    rng = np.random.default_rng(3)
    u0 = 1e-4 * rng.standard_normal(fe.n)
    its = periodic.ivp_parareal(fe, u0, N)
    seq = [u0]
    dt = T / (N * m)
    for n in range(1, N + 1):
        seq.append(fine_propagate(fe, seq[-1], (n - 1) * (T / N), m, dt))
    seq = np.array(seq)
    assert rel(its[N], seq) <= 1e-12
    assert rel(its[N - 2], seq) > 1e-10          # not exact before the last iterations


def test_route_l_equals_cyclic_direct_solve():
    fe = FE(coax.tiny(nr=4, ntheta=8, N=4, m=3))
    UL, _ = periodic.route_l(fe)
    UD = periodic.cyclic_fine_direct(fe)
    assert rel(UL, UD) <= 1e-12


def test_c1_routes_agree():
    """C1: exact DFT route, sequential periods and PP-PC give one periodic solution."""
    fe = FE(coax.c1())
    UL, _ = periodic.route_l(fe)
    US, periods = periodic.route_s(fe, tol=1e-14)
    UP, hist, k = periodic.ppc(fe, tol=1e-12)
    UF, _, _ = periodic.ppc(fe, tol=1e-12, init="fine")
    assert rel(US, UL) <= 1e-12
    assert rel(UP, UL) <= 1e-12
    assert rel(UF, UL) <= 1e-12
    assert k <= 10 and np.all(np.diff(np.log(hist)) < 0)   # monotone contraction


def test_energy_identity_of_the_periodic_linear_solution():
    """Multiply the periodic implicit-Euler equations by du_j and sum over a period:
    sum f_j.du_j = sum du_j.M du_j / dt + 1/2 sum du_j.K du_j (the stored energy
    telescopes)."""
    fe = FE(coax.c1())
    _, u = periodic.route_l(fe)
    prob = fe.prob
    L = prob.N * prob.m
    dt = prob.T / L
    K = fe.K_matrix(np.full(prob.n_tri, coax.NU0))
    du = u - np.roll(u, 1, axis=0)                 # du_j = u_j - u_{j-1}, cyclic
    t = np.arange(L) * dt
    t[0] = prob.T
    f = np.outer(prob.current(t), fe.F)
    lhs = np.sum(f * du)
    rhs = np.sum(du * (fe.M @ du.T).T) / dt + 0.5 * np.sum(du * (K @ du.T).T)
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)


def test_nonlinear_routes_and_variants_share_the_fixed_point():
    """Nonlinear (saturating Brauer sheath): sequential periods and PP-PC from U^0 = 0
    with the exact shift, the harmonic-balance shift and the chord linearisation all
    reach one periodic solution, as does linearising the coarse stiffness at the fine
    results instead of the iterate, and starting from one fine sweep from rest
    (U^0_n = F_n(0)); only iteration counts differ."""
    fe = _tiny_nl(nr=6, ntheta=12, N=8, m=5, amp=400.0)
    US, _ = periodic.route_s(fe, tol=1e-14)
    _, _, b2, _, _ = fe.element_state(US[2])
    assert math.sqrt(b2.max()) > 1.0
    runs = {
        "zero": periodic.ppc(fe, tol=1e-12, init="zero"),
        "iw": periodic.ppc(fe, tol=1e-12, init="zero", shift="iw"),
        "chord": periodic.ppc(fe, tol=1e-12, init="zero", lin="chord"),
        "at-F": periodic.ppc(fe, tol=1e-12, init="zero", lin_point="F"),
        "from-rest": periodic.ppc(fe, tol=1e-12, init="fine"),
    }
    for name, (U, hist, k) in runs.items():
        assert rel(U, US) <= 1e-10, name


def test_ppic_reaches_the_same_solution_more_slowly():
    """PP-IC (eq. (5)) converges to the PP-PC fixed point but needs more iterations."""
    fe = FE(coax.tiny(nr=5, ntheta=10, N=8, m=4))
    Up, _, kp = periodic.ppc(fe, tol=1e-11)
    Ui, _, ki = periodic.ppic(fe, tol=1e-11)
    assert rel(Ui, Up) <= 1e-9
    assert ki > kp


def test_ppic_with_coincident_propagators_steps_one_period_per_iteration():
    """Linear problem with one fine step per subinterval (m = 1): the fine propagator and
    the implicit-Euler coarse propagator of eq. (8) are the same map, so the update of
    eq. (4) collapses to U_n^{k+1} = G(U_{n-1}^{k+1}) from U_0^{k+1} = U_N^k (eq. (5)).
    Every PP-IC iteration then advances classical time stepping by exactly one period:
    U^k_n = u((k-1) T + n dT) for the sequence started at u(0) = U^0_0."""
    prob = coax.tiny(nr=5, ntheta=10, N=8, m=1)
    fe = FE(prob)
    N, dT = prob.N, prob.T / prob.N
    seen = {}

    class Enough(Exception):
        pass

    def keep(k, U, Fs, eps):
        seen[k] = (U.copy(), eps)
        if k == 4:
            raise Enough

    # from rest: the coarse periodic start would already be the fixed point when F = G
    with pytest.raises(Enough):
        periodic.ppic(fe, tol=0.0, U_init=np.zeros((N, fe.n)), callback=keep)
    # the sequence of classical implicit-Euler steps of size dT, one direct solve each
    A = (fe.M / dT + fe.jacobian_curl(np.zeros(fe.n))).tocsc()
    lu = spla.splu(A)
    u = seen[0][0][0].copy()
    for k in range(1, 5):
        rows = [u.copy()]
        for n in range(1, N + 1):
            u = lu.solve(fe.M @ u / dT + fe.f(((k - 1) * N + n) * dT))
            rows.append(u.copy())
        Uk = seen[k][0]
        assert rel(Uk, np.array(rows[:N])) <= 1e-11, k
        # eps^k is the periodicity defect of that period: ||u(kT) - u((k-1)T)|| / ||U^k||_F
        assert seen[k][1] == pytest.approx(np.linalg.norm(rows[N] - rows[0]) / np.linalg.norm(Uk), rel=1e-9)
    # the first period from rest still carries the transient (it has died out by the
    # second), so the first two iterates differ and a wrong start row shows
    assert seen[1][1] > 1e-3 and rel(seen[1][0], seen[2][0]) > 1e-3


@pytest.mark.parametrize("n_harm", [1, 2, 4])
def test_truncated_harmonic_set_keeps_the_fixed_point(n_harm):
    """Solving only the first n_harm harmonics of each correction (the others take the
    jumps' harmonics, which vanish at the fixed point) converges to the same periodic
    solution: linear tiny coax against the exact DFT solve of the cyclic fine system
    (route L), saturating tiny coax against sequential periods (route S), whose odd
    harmonics 3 and 5 carry the saturation and so must be reached by the relaxation."""
    prob = coax.tiny(nr=5, ntheta=10, N=8, m=4)
    fe = FE(prob)
    UL, _ = periodic.route_l(fe)
    U, hist, k = periodic.ppc(fe, tol=1e-12, n_harm=n_harm, max_iter=200)
    assert rel(U, UL) <= 1e-10
    fn = FE(coax.tiny(nr=5, ntheta=10, N=8, m=4, nonlinear=True, amp=600.0))
    US, _ = periodic.route_s(fn, tol=1e-13)
    Un, _, _ = periodic.ppc(fn, tol=1e-12, n_harm=n_harm, max_iter=300)
    H = np.abs(np.fft.rfft(US, axis=0))
    assert H[3].max() > 1e-3 * H[1].max()            # the dropped harmonics are not empty
    assert rel(Un, US) <= 1e-9
    # all N/2 + 1 harmonics is the untruncated iteration, term for term
    Ua, ha, ka = periodic.ppc(fe, tol=1e-12, n_harm=prob.N // 2 + 1)
    Ub, hb, kb = periodic.ppc(fe, tol=1e-12)
    assert ka == kb and np.array_equal(Ua, Ub)


def test_truncated_harmonics_with_a_slow_transient_need_the_low_harmonics():
    """Linearised sheath (time constant near the period): dropping every harmonic but the
    mean leaves the fundamental to the jump relaxation, which contracts slowly, while
    keeping the fundamental converges as fast as the full set."""
    prob = coax.c2lin(nr=6, ntheta=12, N=8, m=6)
    fe = FE(prob)
    _, hf, kf = periodic.ppc(fe, tol=1e-9, max_iter=300)
    _, h2, k2 = periodic.ppc(fe, tol=1e-9, n_harm=2, max_iter=300)
    assert k2 <= kf + 1
    with pytest.raises(RuntimeError, match="did not converge"):
        periodic.ppc(fe, tol=1e-9, n_harm=1, max_iter=5 * kf)


def test_nested_start_reaches_the_same_fixed_point_in_fewer_iterations():
    """U^0 from PP-PC on a 25 times coarser fine grid (2 instead of 50 steps per
    subinterval): the same periodic solution as from zero, in fewer iterations."""
    fe = FE(coax.tiny(nr=6, ntheta=12, N=8, m=50, nonlinear=True, amp=500.0))
    Uz, hz, kz = periodic.ppc(fe, tol=1e-12, init="zero")
    Un, hn, kn = periodic.ppc(fe, tol=1e-12, init="nested")
    assert rel(Un, Uz) <= 1e-10
    assert kn < kz
    # the start is the coarser grid's periodic state: closer than zero, not the answer
    U0 = periodic.initial_iterate(fe, mode="nested")
    assert 1e-6 < rel(U0, Uz) < 0.5


def test_epsilon_definition():
    U = np.ones((2, 3))
    assert periodic.periodicity_residual(U, 0.5 * U) == pytest.approx(0.5)
    assert periodic.periodicity_residual(0 * U, U) == float("inf")
    assert periodic.periodicity_residual(0 * U, 0 * U) == 0.0


def _tiny_saturating(nr=8, N=8, m=6):
    """A thin, strongly driven steel sheath (the batched-designs family) on a small grid."""
    from workloads.coax import AIR, Layer, SIGMA_CU, layered_coax, steel
    t = 0.74e-3
    layers = [Layer(1e-3, SIGMA_CU, 0, +1), Layer(2e-3, 0.0, 0), Layer(2.5e-3, SIGMA_CU, 0),
              Layer(2.5e-3 + t, 1e6, 1)]
    return FE(layered_coax("tiny-saturating", layers, [AIR, steel()], nr, 2 * nr, 50.0, [1],
                           [677.0], [0.0], 0.02, N, m))


def test_safeguard_step_meets_the_cap_exactly_along_the_iterate():
    """B is linear in u: for dU = c U the scaled correction U + theta dU has max |B| equal
    to the cap (theta = (cap - b_U)/(b_new - b_U)); no scaling when the cap is not met."""
    fe = _tiny_saturating()
    rng = np.random.default_rng(3)
    U = 1e-4 * rng.standard_normal((fe.prob.N, fe.n))
    bu = periodic.brauer_bmax(fe, U)
    dU = 2.0 * U                                      # b_new = 3 b_U
    cap = 2.0 * bu
    th = periodic.safeguard_step(fe, U, dU, cap)
    assert th == pytest.approx(0.5, rel=1e-12)
    assert periodic.brauer_bmax(fe, U + th * dU) == pytest.approx(cap, rel=1e-12)
    assert periodic.safeguard_step(fe, U, dU, 3.5 * bu) == 1.0


def test_safeguarded_ppc_reaches_the_unguarded_fixed_point():
    """With a cap below the solution's own peak field the safeguard scales every late
    correction (theta = 1/2 once the iterate sits above the cap), which slows PP-PC but
    leaves its fixed point unchanged."""
    fe = _tiny_saturating()
    U0, h0, k0 = periodic.ppc(fe, tol=1e-11, init="fine")
    bpeak = periodic.brauer_bmax(fe, U0)
    assert bpeak > 1.5
    U1, h1, k1 = periodic.ppc(fe, tol=1e-11, init="fine", b_cap=0.75 * bpeak, max_iter=120)
    assert rel(U1, U0) <= 1e-9
    assert k1 > k0


# -- nonlinear periodic coarse problem (eq. (4) with the nonlinear G of eq. (8)) -------------
def _nonlinear_coarse_step(fe, v, t):
    """One implicit-Euler step of size dT from v to t, by the fine-step Newton."""
    from oracle.timestep import ie_step
    return ie_step(fe, v, t, fe.prob.T / fe.prob.N, tol=1e-14)[0]


def test_nonlinear_coarse_correction_satisfies_eq4_row_by_row():
    """The definition: U^{k+1}_n = F_n(U^k_{n-1}) + G(U^{k+1}_{n-1}) - G(U^k_{n-1}) for every
    n cyclically, with each G evaluated here as a separate coarse step from the new and the
    old samples (so a wrong row shift, sign or time in the block system fails)."""
    fe = _tiny_nl(nr=6, ntheta=12, N=6, m=4, amp=500.0)
    prob = fe.prob
    U = periodic.initial_iterate(fe, mode="fine")
    Fs = periodic.fine_sweep(fe, U)
    U1 = U + periodic.nonlinear_coarse_correction(fe, U, Fs)
    N, dT = prob.N, prob.T / prob.N
    assert rel(U1, U) > 1e-3                      # a real correction, not a no-op
    for n in range(1, N + 1):
        r = n % N
        lhs = U1[r]
        rhs = Fs[r] + _nonlinear_coarse_step(fe, U1[n - 1], n * dT) - _nonlinear_coarse_step(fe, U[n - 1], n * dT)
        assert np.linalg.norm(lhs - rhs) <= 1e-12 * np.linalg.norm(lhs), n


def test_nonlinear_coarse_correction_of_a_linear_problem_is_the_block_cyclic_solve():
    """Linear materials: G is affine and eq. (4) is the block-cyclic linear system of eq. (9)
    with Kbar = K, G dU = Q J; solved here with the explicit matrix and a sparse LU."""
    fe = FE(coax.tiny(nr=5, ntheta=10, N=8, m=3))
    prob = fe.prob
    U = periodic.initial_iterate(fe, mode="fine")
    Fs = periodic.fine_sweep(fe, U)
    J = Fs - U
    dT = prob.T / prob.N
    K = fe.K_matrix(fe.element_state(np.zeros(fe.n))[3])
    Q = (fe.M / dT + K).tocsr()
    G = periodic.block_cyclic_G(fe, K, prob.N, prob.T).tocsc()
    dU_ref = spla.spsolve(G, np.concatenate([Q @ J[r] for r in range(prob.N)])).reshape(U.shape)
    dU = periodic.nonlinear_coarse_correction(fe, U, Fs)
    assert rel(dU, dU_ref) <= 1e-10


def test_nonlinear_coarse_correction_vanishes_at_the_fixed_point():
    """F_n(U_{n-1}) = U_n for all n (zero jumps): eq. (4) gives U^{k+1} = U^k."""
    fe = _tiny_nl(nr=5, ntheta=10, N=6, m=3, amp=400.0)
    US, _ = periodic.route_s(fe, tol=1e-14)
    Fs = periodic.fine_sweep(fe, US)
    assert rel(Fs, US) <= 1e-11
    dU = periodic.nonlinear_coarse_correction(fe, US, Fs)
    assert np.linalg.norm(dU) <= 1e-10 * np.linalg.norm(US)


def test_ppc_with_the_nonlinear_coarse_problem_keeps_the_fixed_point():
    """PP-PC with the nonlinear coarse correction reaches the periodic solution of
    sequential time stepping (saturating sheath, from U^0 = 0)."""
    fe = _tiny_nl(nr=6, ntheta=12, N=8, m=5, amp=400.0)
    US, _ = periodic.route_s(fe, tol=1e-14)
    U, hist, k = periodic.ppc(fe, tol=1e-12, init="zero", coarse="nonlinear")
    assert rel(U, US) <= 1e-10
    assert k <= 30 and hist[-1] <= 1e-12


def test_nonlinear_coarse_jacobian_matches_central_differences():
    """The block-cyclic Jacobian of Phi against central differences of Phi itself, on a
    saturating state with the coupling to the previous row in every block row (a misplaced
    or transposed -C block, or a missing differential term, fails)."""
    fe = _tiny_nl(nr=5, ntheta=10, N=4, m=3, amp=600.0)
    prob = fe.prob
    rng = np.random.default_rng(3)
    US, _ = periodic.route_s(fe, tol=1e-12)
    W = US * (1.0 + 0.3 * rng.standard_normal(US.shape))
    b = 0.05 * rng.standard_normal(US.shape) * np.abs(US).max()
    _, _, b2, _, _ = fe.element_state(W[1])
    assert math.sqrt(b2.max()) > 1.0               # the Brauer law is in its nonlinear range
    Jm = periodic.nonlinear_coarse_jacobian(fe, W)
    v = rng.standard_normal(W.shape)
    h = 1e-6 * np.linalg.norm(W) / np.linalg.norm(v)
    fd = (periodic.nonlinear_coarse_residual(fe, W + h * v, b)
          - periodic.nonlinear_coarse_residual(fe, W - h * v, b)) / (2.0 * h)
    Jv = (Jm @ v.ravel()).reshape(W.shape)
    assert rel(Jv, fd) <= 1e-6
    # the coupling: row n depends on W_{n-1} through -C only
    e = np.zeros_like(W)
    e[prob.N - 1] = v[prob.N - 1]
    Je = (Jm @ e.ravel()).reshape(W.shape)
    C = fe.M / (prob.T / prob.N)
    assert rel(Je[0], -(C @ v[prob.N - 1])) <= 1e-12

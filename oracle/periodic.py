"""Periodic steady states: the plain definition and plain PP-PC (oracle, FP64).

Paper, Section 2, eq. (1): find u with ``M u' + K(u) u = f`` and ``u(0) = u(T)``.
Discretised by implicit Euler with L = N*m fine steps of size dt = T/L, the
periodic fine solution is the unique cyclic sequence u_j (u_L = u_0) with

    M (u_j - u_{j-1})/dt + K(u_j) u_j = f(t_j),   t_j = j dt,   j = 1..L.

At its fixed point the PP-PC iteration of eq. (4) has U_n = F_n(U_{n-1})
cyclically, so its answer is exactly this sequence sampled at U_n = u_{n m}.
Three routes compute it here:

* ``route_s``: classical time stepping over whole periods until the
  period-to-period change stalls (Section 1; Fig. 1 shows why this is slow);
* ``ppc``: plain PP-PC, eq. (4), with the coarse problem of eqs. (8)-(10)
  solved per harmonic after a DFT along time, eqs. (11)-(14);
* ``route_l`` (linear problems only): the exact length-L DFT solve of the
  cyclic fine system.

TEST INFRASTRUCTURE ONLY: see the package docstring.
"""
from __future__ import annotations

import copy
import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fe import BRAUER, FE
from .timestep import NEWTON_TOL, fine_propagate, ie_step


def coarse_times(prob):
    """T_n = n T/N, n = 0..N (Section 2)."""
    return np.arange(prob.N + 1) * (prob.T / prob.N)


def fine_dt(prob):
    return prob.T / (prob.N * prob.m)


# ----------------------------------------------------------------------------------------
# route S: sequential time stepping over whole periods
# ----------------------------------------------------------------------------------------
def route_s(fe, tol=1e-13, max_periods=5000, u_start=None, newton_tol=NEWTON_TOL):
    """Step period after period from u_start (default 0) until
    max_n ||U_n^(p) - U_n^(p-1)|| <= tol * max_n ||U_n^(p)||.  Returns (U, periods)
    with U[n] = u(T_n), U[0] = u(T) = u(0)."""
    prob = fe.prob
    N, m = prob.N, prob.m
    dt = fine_dt(prob)
    u = np.zeros(fe.n) if u_start is None else np.array(u_start, dtype=np.float64)
    prev = None
    for period in range(1, max_periods + 1):
        U = np.zeros((N, fe.n))
        for n in range(1, N + 1):
            t0 = (n - 1) * (prob.T / N)
            for j in range(1, m + 1):
                u, _ = ie_step(fe, u, t0 + j * dt, dt, tol=newton_tol)
            U[n % N] = u
        if prev is not None:
            change = np.max(np.linalg.norm(U - prev, axis=1))
            if change <= tol * np.max(np.linalg.norm(U, axis=1)):
                return U, period
        prev = U
    raise RuntimeError("route S did not reach a periodic state")


# ----------------------------------------------------------------------------------------
# route L: exact DFT solve of the linear cyclic fine system
# ----------------------------------------------------------------------------------------
def route_l(fe, nu=None):
    """Linear problems only: (K + (1 - exp(-2 pi i q/L)) M/dt) uhat_q = fhat_q,
    q = 0..L/2, then u = irfft(uhat); U_n = u_{n m}.  Row 0 of the cyclic system is
    step L (t = T)."""
    prob = fe.prob
    L = prob.N * prob.m
    dt = fine_dt(prob)
    if nu is None:
        _, _, _, nu, dnu = fe.element_state(np.zeros(fe.n))
        if np.any(dnu != 0.0):
            raise ValueError("route L is for linear problems")
    K = fe.K_matrix(nu)
    t = np.arange(L) * dt
    t[0] = prob.T
    fs = np.outer(prob.current(t), fe.F)                 # rows j = 0..L-1
    fh = np.fft.rfft(fs, axis=0)
    uh = np.zeros_like(fh)
    for q in range(fh.shape[0]):
        s = (1.0 - np.exp(-2j * math.pi * q / L)) / dt
        A = (K + s * fe.M).astype(np.complex128).tocsc()
        uh[q] = spla.splu(A).solve(fh[q])
    u = np.fft.irfft(uh, n=L, axis=0)
    return u[:: prob.m].copy(), u


def cyclic_fine_direct(fe):
    """Brute force for tiny linear problems: assemble the (L n) x (L n) cyclic fine
    implicit-Euler system and solve it directly."""
    prob = fe.prob
    L = prob.N * prob.m
    dt = fine_dt(prob)
    _, _, _, nu, _ = fe.element_state(np.zeros(fe.n))
    K = fe.K_matrix(nu)
    A = sp.kron(sp.eye(L), fe.M / dt + K) - sp.kron(
        sp.csr_matrix((np.ones(L), (np.arange(L), (np.arange(L) - 1) % L)), shape=(L, L)),
        fe.M / dt)
    t = np.arange(L) * dt
    t[0] = prob.T
    rhs = np.outer(prob.current(t), fe.F).ravel()
    u = spla.spsolve(A.tocsc(), rhs).reshape(L, fe.n)
    return u[:: prob.m].copy()


# ----------------------------------------------------------------------------------------
# PP-PC pieces
# ----------------------------------------------------------------------------------------
def shifts(N, T, mode="ie"):
    """Per-harmonic shift sigma_p, p = 0..N/2, of the block-diagonal system, eq. (13).

    mode "ie": the exact DFT symbol of the implicit-Euler cyclic matrix of eq. (9),
    (1 - exp(-i w_p dT))/dT with w_p = 2 pi p/T (eq. (12)) and dT = T/N (eq. (10)).
    mode "iw": the harmonic-balance shift i w_p."""
    p = np.arange(N // 2 + 1)
    dT = T / N
    if mode == "ie":
        return (1.0 - np.exp(-2j * math.pi * p / N)) / dT
    if mode == "iw":
        return 2j * math.pi * p / T
    raise ValueError(mode)


def coarse_stiffness(fe, U, lin="tensor"):
    """Kbar for the coarse operator.  Linear problems: K.  Nonlinear: the frozen
    time-averaged linearisation over the coarse samples U (reading; the paper defers
    the nonlinear treatment, Section 2 after eq. (10)).  lin="chord" averages the
    scalar nu instead of the differential tensor."""
    if lin == "tensor":
        return fe.linearised_stiffness(U)
    if lin == "chord":
        nus = np.mean([fe.element_state(u)[3] for u in np.atleast_2d(U)], axis=0)
        return fe.K_matrix(nus)
    raise ValueError(lin)


def harmonic_solve(fe, Kbar, Rrows, T, shift="ie", n_harm=None, Jrows=None):
    """Solve the block-cyclic coarse system G X = R (eq. (9), with G built from
    C = M/dT and Q = C + Kbar) through the DFT along time (eqs. (11)-(14)): one
    shifted sparse system (Kbar + sigma_p M) per harmonic p = 0..N/2; the negative
    harmonics follow by conjugate symmetry.  Rows of Rrows are n = 0..N-1.

    Truncated harmonic set (n_harm < N/2 + 1; eq. (11) summed over a subset of the
    spectrum of eq. (12)): only p < n_harm are solved; every other harmonic of the
    correction is the harmonic of the jumps Jrows, X_p = J_p, which vanishes at the
    fixed point and so leaves it unchanged (reading)."""
    N = Rrows.shape[0]
    Rh = np.fft.rfft(Rrows, axis=0)
    H = Rh.shape[0]
    nh = H if n_harm is None else n_harm
    Xh = np.zeros_like(Rh)
    for p, s in enumerate(shifts(N, T, shift)):
        if p >= nh:
            break
        A = (Kbar + s * fe.M).astype(np.complex128).tocsc()
        Xh[p] = spla.splu(A, permc_spec="MMD_AT_PLUS_A").solve(Rh[p])
    if nh < H:
        Xh[nh:] = np.fft.rfft(Jrows, axis=0)[nh:]
    return np.fft.irfft(Xh, n=N, axis=0)


def block_cyclic_G(fe, Kbar, N, T):
    """Explicit G of eq. (9): Q on the diagonal, -C below it and in the top-right
    corner (row 0 couples to U_{N-1}).  For brute-force tests on tiny problems."""
    dT = T / N
    C = fe.M / dT
    Q = C + Kbar
    S = sp.csr_matrix((np.ones(N), (np.arange(N), (np.arange(N) - 1) % N)), shape=(N, N))
    return (sp.kron(sp.eye(N), Q) - sp.kron(S, C)).tocsr()


def excitation_rows(fe, N, T):
    """f(T_n) for rows n = 0..N-1, row 0 carrying T_N = T (eq. (9) ordering)."""
    t = np.arange(N) * (T / N)
    t[0] = T
    return np.outer(fe.prob.current(t), fe.F)


def initial_iterate(fe, shift="ie", lin="tensor", mode="auto", pool=None):
    """U^0 (the paper does not state it; reading).

    mode "coarse": the coarse periodic solution with zero right-hand side b in
    eqs. (9)-(10), i.e. G U = [f(T_N), f(T_1), ..., f(T_{N-1})], with the coarse
    stiffness at u = 0.  mode "zero": U^0 = 0.  mode "fine": one fine sweep from zero,
    U^0_n = F_n(0) -- every subinterval starts from rest, so the samples carry the
    saturation the fine propagator produces instead of the one a linearisation predicts.
    mode "nested": PP-PC of the same problem on a 25 times coarser fine grid
    (max(1, m // 25) steps per subinterval) to eps <= 1e-2 -- a cheap first approximation
    (reading; the fixed point does not depend on U^0).
    mode "auto": "coarse" when every material is linear, else "zero" -- at u = 0 a
    Brauer material has its unsaturated reluctivity, and a coarse solve with it can put
    tens of tesla into the steel, where exp(k2 b^2) overflows."""
    prob = fe.prob
    if mode == "auto":
        mode = "coarse" if np.all(prob.mat_model[np.unique(prob.mat_id)] == 0) else "zero"
    if mode == "zero":
        return np.zeros((prob.N, fe.n))
    if mode == "nested":
        # the periodic solution of the same problem with max(1, m // 25) fine steps per
        # subinterval, by PP-PC to eps <= 1e-2 from the automatic start
        coarse = copy.copy(prob)
        coarse.m = max(1, prob.m // 25)
        U, _, _ = ppc(FE(coarse), tol=1e-2, max_iter=200, shift=shift, lin=lin, pool=None)
        return U
    if mode == "fine":
        return fine_sweep(fe, np.zeros((prob.N, fe.n)), pool=pool)
    if mode != "coarse":
        raise ValueError(mode)
    Kbar = coarse_stiffness(fe, np.zeros((1, fe.n)), lin)
    return harmonic_solve(fe, Kbar, excitation_rows(fe, prob.N, prob.T), prob.T, shift)


def periodicity_residual(U, J):
    """eps = ||J||_F / ||U||_F; +inf when U = 0 and J != 0 (e.g. at U^0 = 0)."""
    jn = np.linalg.norm(J)
    un = np.linalg.norm(U)
    if un > 0.0:
        return jn / un
    return 0.0 if jn == 0.0 else float("inf")


def fine_sweep(fe, U, newton_tol=NEWTON_TOL, pool=None):
    """F_n(U_{n-1}) for n = 1..N, independent of each other (eq. (4)); returns the
    array Fs with Fs[n % N] = F_n, so Fs[0] = F_N lands on the index of U_0."""
    prob = fe.prob
    N, m = prob.N, prob.m
    dt = fine_dt(prob)
    args = [((n - 1) * (prob.T / N), U[n - 1]) for n in range(1, N + 1)]
    if pool is None:
        outs = [fine_propagate(fe, u0, t0, m, dt, tol=newton_tol) for t0, u0 in args]
    else:
        outs = pool.starmap(_chain_worker, [(t0, u0, m, dt, newton_tol) for t0, u0 in args])
    Fs = np.zeros_like(U)
    for n in range(1, N + 1):
        Fs[n % N] = outs[n - 1]
    return Fs


_WORKER_FE = None


def _init_worker(prob):
    global _WORKER_FE
    from .fe import FE
    _WORKER_FE = FE(prob)


def _chain_worker(t0, u0, m, dt, newton_tol):
    return fine_propagate(_WORKER_FE, u0, t0, m, dt, tol=newton_tol)


def make_pool(prob, processes):
    """Process pool whose workers each hold their own FE copy (fine chains in parallel)."""
    import multiprocessing as mp
    return mp.get_context("fork").Pool(processes, initializer=_init_worker, initargs=(prob,))


def coarse_correction(fe, U, J, shift="ie", lin="tensor", U_lin=None, n_harm=None):
    """Delta U from the jumps J (rows n = 0..N-1, J[n] = F_n - U_n mod N).

    In the linear case eq. (4) with implicit-Euler G (eq. (8)) is equivalent to the
    cyclic system Q dU_n - C dU_{n-1} = Q J_n, whose DFT blocks are
    (K + sigma_p M) (eq. (13)).  The literal right-hand side of eq. (10) satisfies
    r^k = G U^k + Q J^k, so solving G U^{k+1} = r^k is the same as solving
    G dU = Q J for dU = U^{k+1} - U^k; that correction form is used."""
    prob = fe.prob
    N, T = prob.N, prob.T
    Kbar = coarse_stiffness(fe, U if U_lin is None else U_lin, lin)
    Q = fe.M / (T / N) + Kbar
    R = np.asarray((Q @ J.T).T)
    return harmonic_solve(fe, Kbar, R, T, shift, n_harm=n_harm, Jrows=J)


def coarse_rows_times(prob):
    """End time of row n's coarse step: T_n for n = 1..N-1 and T_N = T for row 0."""
    t = np.arange(prob.N) * (prob.T / prob.N)
    t[0] = prob.T
    return t


def coarse_sweep(fe, U, tol=1e-14):
    """G(U_{n-1}) for every row n (row 0 from U_{N-1}): one implicit-Euler step of size
    dT = T/N on the nonlinear problem (eq. (8) with the nonlinear stiffness), each solved
    to tol by the same Newton as a fine step."""
    prob = fe.prob
    dT = prob.T / prob.N
    t = coarse_rows_times(prob)
    prev = np.roll(U, 1, axis=0)
    return np.array([ie_step(fe, prev[r], t[r], dT, tol=tol)[0] for r in range(prob.N)])


def nonlinear_coarse_residual(fe, W, b):
    """Phi_n(W) = C (W_n - U_{n-1}) + K(W_n) W_n - f(T_n) with U = W + b, C = M/dT: the
    implicit-Euler step residual of W_n = G(U_{n-1}) (rows n = 0..N-1, row 0 at T_N)."""
    prob = fe.prob
    dT = prob.T / prob.N
    t = coarse_rows_times(prob)
    prev = np.roll(W + b, 1, axis=0)
    return np.array([fe.M @ (W[r] - prev[r]) / dT + fe.K_apply(W[r]) - fe.f(t[r])
                     for r in range(prob.N)])


def nonlinear_coarse_jacobian(fe, W):
    """d Phi / d W: block-cyclic, C + dK(W_n)W_n/dW_n on the diagonal and -C below it
    (row 0 couples to row N-1)."""
    prob = fe.prob
    N, dT = prob.N, prob.T / prob.N
    C = (fe.M / dT).tocsr()
    blocks = [[None] * N for _ in range(N)]
    for r in range(N):
        blocks[r][r] = C + fe.jacobian_curl(W[r])
        blocks[r][(r - 1) % N] = -C
    return sp.bmat(blocks, format="csc")


def nonlinear_coarse_correction(fe, U, Fs, tol=1e-13, max_newton=40):
    """Delta U of eq. (4) with the nonlinear coarse propagator G of eq. (8) (the coarse
    problem the paper defers, Section 2 after eq. (10) and Section 5; reading: G_n(v) is
    one implicit-Euler step of size dT from v to T_n with the full K(u)).

    Eq. (4) reads U^{k+1}_n = G(U^{k+1}_{n-1}) + b_n with b_n = F_n(U^k_{n-1}) - G(U^k_{n-1})
    cyclically.  With W_n = U^{k+1}_n - b_n = G(U^{k+1}_{n-1}) this is the block-cyclic
    nonlinear system Phi(W) = 0 of nonlinear_coarse_residual, solved here by Newton's method
    with the exact Jacobian and a sparse direct solve, from W = G(U^k) (where Phi_n equals
    -C J_{n-1}), with backtracking on ||Phi||.  Stops when ||Phi|| <= tol * scale, scale =
    ||C U^k||_F + ||C G(U^k)||_F + ||f||_F, or at the rounding floor of Phi's evaluation (a
    Newton step at rounding level, or a stalled line search with ||Phi|| <= 1e-9 scale).
    Returns U^{k+1} - U^k."""
    prob = fe.prob
    dT = prob.T / prob.N
    V = coarse_sweep(fe, U)
    b = Fs - V
    W = V.copy()
    scale = ((np.linalg.norm((fe.M @ U.T).T) + np.linalg.norm((fe.M @ V.T).T)) / dT
             + np.linalg.norm(np.outer(prob.current(coarse_rows_times(prob)), fe.F)))
    Phi = nonlinear_coarse_residual(fe, W, b)
    rn = np.linalg.norm(Phi)
    for _ in range(max_newton + 1):
        if rn <= tol * scale:
            break
        d = spla.splu(nonlinear_coarse_jacobian(fe, W), permc_spec="MMD_AT_PLUS_A").solve(-Phi.ravel())
        d = d.reshape(W.shape)
        if np.linalg.norm(d) <= 4.0 * np.finfo(float).eps * np.linalg.norm(W):
            W = W + d
            break
        lam = 1.0
        while True:
            Wt = W + lam * d
            Pt = nonlinear_coarse_residual(fe, Wt, b)
            rt = np.linalg.norm(Pt)
            if rt <= (1.0 - 1e-4 * lam) * rn:
                break
            lam *= 0.5
            if lam < 2.0 ** -20:
                break
        if lam < 2.0 ** -20:
            if rn <= 1e-9 * scale:      # no decrease representable: rounding floor
                break
            raise RuntimeError(f"nonlinear coarse problem: line search failed at ||Phi||={rn:.3e}")
        W, Phi, rn = Wt, Pt, rt
    else:
        raise RuntimeError(f"nonlinear coarse problem: no convergence, ||Phi||={rn:.3e}")
    return W + b - U


def brauer_bmax(fe, U):
    """max |B| over the Brauer elements and the samples (rows) of U (0 without steel)."""
    mask = fe.model == BRAUER
    if not np.any(mask):
        return 0.0
    return max(math.sqrt(fe.element_state(u)[2][mask].max()) for u in U)


def safeguard_step(fe, U, dU, b_cap):
    """Step theta of the correction U + theta dU (a safeguard the paper does not have: its
    coarse problem is not a frozen linearisation): theta = 1 when max |B(U + dU)| <= b_cap,
    else (b_cap - b_U) / (b_new - b_U) with b_U = max |B(U)|, the largest step for which
    |B| stays below the cap (B is linear in u, so |B(U + theta dU)| <= (1 - theta) b_U +
    theta b_new), or 1/2 if U itself exceeds the cap."""
    bu, bn = brauer_bmax(fe, U), brauer_bmax(fe, U + dU)
    if bn <= b_cap:
        return 1.0
    return (b_cap - bu) / (bn - bu) if bu < b_cap else 0.5


def ppc(fe, tol=1e-12, max_iter=60, U_init=None, shift="ie", lin="tensor",
        newton_tol=NEWTON_TOL, pool=None, callback=None, init="auto", lin_point="F", b_cap=None,
        n_harm=None, coarse="frozen"):
    """Plain PP-PC (eq. (4)).

    n_harm < N/2 + 1 solves only the first n_harm harmonics of each correction (the rest
    take the jumps' harmonics; see harmonic_solve).  The initial iterate uses them all.

    coarse="nonlinear" replaces the frozen correction by the one of eq. (4) with the
    nonlinear coarse propagator (nonlinear_coarse_correction); the fixed point is the same.

    lin_point selects the samples the frozen coarse stiffness is linearised at: "U" the
    current iterate U^k, "F" the fine results F^k of the same sweep (they coincide at the
    fixed point, so the answer does not change).

    Per iteration k: fine sweep F_n(U_{n-1}^k); jumps J_n = F_n - U^k_{n mod N};
    eps^k = ||J||_F/||U^k||_F (the paper does not state the tolerance quantity; this
    is the reading); stop and return U^k if eps^k <= tol; else apply the coarse
    correction, scaled by safeguard_step when b_cap is given.  Returns (U, eps_history,
    iterations) where iterations counts the corrections applied (fine sweeps =
    iterations + 1)."""
    prob = fe.prob
    if U_init is None:
        U = initial_iterate(fe, shift, lin, init, pool=pool)
    else:
        U = np.array(U_init, dtype=np.float64, copy=True)
    hist = []
    for k in range(max_iter + 1):
        Fs = fine_sweep(fe, U, newton_tol=newton_tol, pool=pool)
        J = Fs - U
        eps = periodicity_residual(U, J)
        hist.append(eps)
        if callback is not None:
            callback(k, U, Fs, eps)
        if eps <= tol:
            return U, np.array(hist), k
        if k == max_iter:
            break
        if coarse == "nonlinear":
            dU = nonlinear_coarse_correction(fe, U, Fs)
        else:
            dU = coarse_correction(fe, U, J, shift, lin, U_lin=Fs if lin_point == "F" else None,
                                   n_harm=n_harm)
        U = U + (safeguard_step(fe, U, dU, b_cap) * dU if b_cap else dU)
    raise RuntimeError(f"PP-PC did not converge: eps history {hist[-5:]}")


def ppic(fe, tol=1e-12, max_iter=200, U_init=None, lin="tensor", newton_tol=NEWTON_TOL,
         pool=None, callback=None):
    """PP-IC: eq. (4) with the periodic row relaxed as in eq. (5), U_0^{k+1} = U_N^k.
    The iterate holds U_0..U_N; rows n = 1..N follow the classical Parareal update
    U_n^{k+1} = F_n(U_{n-1}^k) + G_n(U_{n-1}^{k+1}) - G_n(U_{n-1}^k) with the
    implicit-Euler coarse propagator of eq. (8) on the frozen coarse stiffness.
    eps^k uses the same jumps as ppc (row 0 compares F_N with U_0).  callback(k, U, Fs,
    eps) sees every iterate, as in ppc."""
    prob = fe.prob
    N, T = prob.N, prob.T
    dT = T / N
    U = initial_iterate(fe, "ie", lin) if U_init is None else np.array(U_init, dtype=np.float64)
    UN = U[0].copy()
    C = fe.M / dT
    fr = excitation_rows(fe, N, T)
    hist = []
    for k in range(max_iter + 1):
        Fs = fine_sweep(fe, U, newton_tol=newton_tol, pool=pool)
        J = Fs - U
        eps = periodicity_residual(U, J)
        hist.append(eps)
        if callback is not None:
            callback(k, U, Fs, eps)
        if eps <= tol:
            return U, np.array(hist), k
        lu = spla.splu((C + coarse_stiffness(fe, U, lin)).tocsc())

        def G(n, u):
            return lu.solve(C @ u + fr[n % N])

        Unew = np.zeros_like(U)
        Unew[0] = UN
        prev_new = UN
        for n in range(1, N + 1):
            val = Fs[n % N] + G(n, prev_new) - G(n, U[n - 1])
            if n < N:
                Unew[n] = val
            prev_new = val
        UN = prev_new
        U = Unew
    raise RuntimeError(f"PP-IC did not converge: eps history {hist[-5:]}")


def ivp_parareal(fe, u0, K_iters, lin_K=None):
    """Classical initial-value Parareal with U_0 held fixed (eq. (4) without the
    periodic row) and the implicit-Euler coarse propagator; returns the iterates.
    For tests of the finite-termination property (iterate N equals the fine solution)."""
    prob = fe.prob
    N, T, m = prob.N, prob.T, prob.m
    dT = T / N
    dt = dT / m
    if lin_K is None:
        _, _, _, nu, _ = fe.element_state(np.zeros(fe.n))
        lin_K = fe.K_matrix(nu)
    C = fe.M / dT
    lu = spla.splu((C + lin_K).tocsc())
    fr = excitation_rows(fe, N, T)

    def G(n, u):
        return lu.solve(C @ u + fr[n % N])

    U = np.zeros((N + 1, fe.n))
    U[0] = u0
    for n in range(1, N + 1):
        U[n] = G(n, U[n - 1])
    its = [U.copy()]
    for _ in range(K_iters):
        Fv = [fine_propagate(fe, U[n - 1], (n - 1) * dT, m, dt) for n in range(1, N + 1)]
        Unew = np.zeros_like(U)
        Unew[0] = u0
        for n in range(1, N + 1):
            Unew[n] = Fv[n - 1] + G(n, Unew[n - 1]) - G(n, U[n - 1])
        U = Unew
        its.append(U.copy())
    return its

/*
 * ppcmh.h -- C-ABI of the MI355X library for periodic Parareal with a multi-harmonic
 * coarse correction (PP-PC) applied to the 2-D eddy-current problem
 *
 *     M du/dt + K(u) u = f(t),   t in (0, T),   u(0) = u(T)
 *
 * of Kulchytska-Ruchka, De Gersem and Schoeps (arXiv:1905.13076), Section 2, eq. (1).
 *
 * Conventions for every function:
 *   - return 0 (PPC_OK) on success, > 0 for completion with a warning (outputs written),
 *     < 0 for an error (no output written; ppc_last_error() explains);
 *   - all indices are 0-based int32, all reals IEEE double unless stated;
 *   - the caller owns every buffer it passes; the library copies what it needs during
 *     the call and keeps no caller pointer afterwards;
 *   - argument checks happen on the host before any device work, so argument errors
 *     are reported identically on machines without a GPU;
 *   - "host pointer" means ordinary CPU memory, "device pointer" means memory of the
 *     handle's GPU (e.g. from hipMalloc or a torch CUDA tensor);
 *   - a handle is used by one host thread at a time; distinct handles are independent.
 *
 * Vectors of nodal values are indexed by mesh node (length n_nodes) with the
 * Dirichlet nodes held at 0.  A set of coarse samples U (Section 2: U_n at
 * T_n = n T / N, n = 0..N-1) is stored row-major as U[n * n_nodes + node].
 */
#ifndef PPCMH_H
#define PPCMH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PPC_ABI_VERSION 4

/* status codes */
#define PPC_OK 0
#define PPC_NOT_CONVERGED 1   /* warning: outputs hold the last iterate */
#define PPC_ERR_ARG (-1)      /* invalid argument (null, size, non-finite, range) */
#define PPC_ERR_MESH (-2)     /* degenerate/invalid mesh (zero area, bad index, no Dirichlet
                                 node, node in no triangle, no free node) */
#define PPC_ERR_DEVICE (-3)   /* HIP runtime error or no usable GPU */
#define PPC_ERR_OOM (-4)      /* device allocation failed */
#define PPC_ERR_NONFINITE (-5)/* NaN/Inf in a residual (e.g. exp overflow of the B-H law) */
#define PPC_ERR_BREAKDOWN (-6)/* COCG breakdown: rho or p^T A p vanished */
#define PPC_ERR_NEWTON (-7)   /* Newton / line search failed in a fine step */

/* reluctivity laws (per material) */
#define PPC_LAW_LINEAR 0      /* nu = const */
#define PPC_LAW_BRAUER 1      /* nu(b2) = k1 exp(k2 b2) + k3, b2 = |B|^2 = |grad A|^2 */

typedef struct ppc_handle ppc_handle;
typedef struct ppc_problem ppc_problem;

/* Triangular P1 mesh (Section 4 uses "the finite element method"; linear triangles
 * are this library's element).  Triangles may have either orientation. */
typedef struct {
    int32_t n_nodes;
    const double* xy;     /* host, [2 * n_nodes], (x, y) interleaved, metres */
    int32_t n_tri;
    const int32_t* tri;   /* host, [3 * n_tri] node indices */
    int32_t n_dir;
    const int32_t* dir;   /* host, [n_dir] nodes with A = 0 (homogeneous Dirichlet) */
} ppc_mesh;

typedef struct {
    int32_t law;          /* PPC_LAW_LINEAR or PPC_LAW_BRAUER */
    double nu;            /* linear reluctivity (m/H), > 0; unused for Brauer */
    double k1, k2, k3;    /* Brauer constants: k1 >= 0, k2 >= 0, k3 > 0 */
} ppc_law;

/* Materials per triangle: the conductivity sigma defines M (Section 2: "the
 * (singular) conductivity matrix"; sigma = 0 gives zero rows), the law defines K(u). */
typedef struct {
    const double* sigma;    /* host, [n_tri], S/m, >= 0 */
    const int32_t* mat_id;  /* host, [n_tri], index into table */
    int32_t n_mat;
    const ppc_law* table;   /* host, [n_mat] */
} ppc_material;

/* Excitation f(t) = i(t) * F with F_i = sum_e js_e |T_e| / 3 (P1 load of a uniform
 * source density) and i(t) = sum_h amp_h sin(2 pi order_h f0 t + phase_h); Section 4
 * drives the cable with a 50 Hz sinusoidal current. */
typedef struct {
    const double* js;       /* host, [n_tri], source current density per ampere (A/m^2/A) */
    double f0;              /* fundamental frequency (Hz) */
    int32_t n_h;            /* number of terms, >= 0 */
    const int32_t* order;   /* host, [n_h] */
    const double* amp;      /* host, [n_h] (A) */
    const double* phase;    /* host, [n_h] (rad) */
} ppc_excitation;

/* Progress of a long solve: called on the host thread running ppc_solve /
 * ppc_solve_device after each fine sweep, with m (the fine steps per subinterval of the
 * solve in progress: a nested start reports its coarser grid first), the iteration k,
 * eps^k (for a batch the largest over the designs still iterating) and the number of
 * designs still iterating (1 for a single design).  It must not call into the library. */
typedef void (*ppc_progress_fn)(int32_t m, int32_t iteration, double eps, int32_t active, void* user);

/* Solver parameters.  Fill with ppc_params_default() and override. */
typedef struct {
    double T;               /* period (s), > 0 (Section 2) */
    int32_t N;              /* Parareal subintervals, even, >= 2 (Section 2) */
    int32_t m;              /* implicit-Euler fine steps per subinterval, >= 1 (Section 4) */
    int32_t shift_mode;     /* 0: exact DFT symbol of eq. (9), (1 - e^{-i w_p dT})/dT;
                               1: harmonic-balance shift i w_p (eq. (12)) */
    int32_t lin_mode;       /* coarse stiffness of a nonlinear problem: 0 = time average
                               of the differential reluctivity tensor, 1 = of the chord nu */
    int32_t init_mode;      /* U^0 when no U_init is given: 0 auto (1 if all laws linear,
                               else 2), 1 linear coarse periodic solve at u = 0, 2 zero,
                               3 one fine sweep from rest, U^0_n = F_n(0) (for strongly
                               saturating designs, where a first correction from zero can
                               overshoot), 4 nested: PP-PC of the same problem (every
                               design of a batch) with max(1, m/25) fine steps per
                               subinterval to eps <= 1e-2, from rest when b_cap > 0 and from
                               the automatic start otherwise (a cheap first approximation) */
    int32_t precision;      /* 0: FP64 fine solves; 1: FP32 PCG refined by FP64 Newton */
    double tol_ppc;         /* stop when ||J||_F / ||U||_F <= tol_ppc */
    int32_t max_iters;      /* maximum coarse corrections */
    double tol_newton;      /* ||R|| <= tol_newton (||f(t)|| + ||M u_prev|| / dt) */
    int32_t max_newton;     /* Newton iterations per fine step */
    double tol_lin;         /* PCG: ||r|| <= max(tol_lin ||R||, 0.5 tol_newton scale) */
    int32_t max_lin;        /* PCG iteration cap per Newton step */
    double tol_cocg;        /* COCG: ||r|| <= tol_cocg ||b|| per harmonic */
    int32_t max_cocg;       /* COCG iteration cap */
    int32_t block;          /* fine-kernel path: 0 = library choice (register rows for small
                               meshes, else LDS-resident p / diagonal); 1024 = force the
                               workgroup-memory PCG path */
    int32_t no_predictor;   /* 1: start every Newton solve from u_{j-1}; 0: also try the
                               extrapolation of the previous steps (cubic from the fourth
                               step, quadratic at the third, linear at the second) and keep
                               the smaller residual */
    int32_t lin_point;      /* samples the coarse stiffness is linearised at: 0 = the current
                               iterate U^k, 1 = the fine results F^k of the same sweep (equal
                               at the fixed point) */
    int32_t coarse_precision; /* harmonic (coarse) solves: -1 = as precision, 0 = FP64 COCG,
                               1 = complex-FP32 COCG refined by FP64 residuals */
    int32_t graph;          /* single-design solves: 1 = each PP-PC iteration replays two HIP
                               graphs (fine sweep + jumps; coarse correction), captured at the
                               second iteration; 0 = eager launches.  Same kernels, same results */
    int32_t method;         /* 0 = PP-PC: eq. (4) with the periodic coarse problem of eqs.
                               (9)-(14), solved per harmonic; 1 = PP-IC: eq. (4) with the
                               periodicity of eq. (5), U_0^{k+1} = U_N^k, and the sequential
                               implicit-Euler coarse propagator of eq. (8) on the frozen coarse
                               stiffness at U^k (N real shifted solves per iteration, one after
                               the other; lin_point and shift_mode do not apply).  PP-IC is for
                               single-design solves without b_cap */
    int32_t fine_block;     /* register-row fine kernel workgroup: 0 = the size ppc_autotune
                               chose for this problem and precision, else 1024; 256, 512 or
                               1024 = that size (PPC_ERR_ARG when the mesh's rows do not fit:
                               R rows per thread with R * fine_block >= free nodes, R a power
                               of two <= 8 at 256 and 512 threads, R <= 8 at 1024 (<= 12 in
                               FP32), and p, r and the diagonal in LDS) */
    int32_t n_harm;         /* harmonics each PP-PC correction solves: 0 = all N/2 + 1 (eq.
                               (12)); 1..N/2+1 = p = 0..n_harm-1 only, every other harmonic of
                               the correction being that of the jumps (zero at the fixed point,
                               which is therefore unchanged).  The initial coarse solve and the
                               adjoint use all harmonics */
    double b_cap;           /* coarse-correction safeguard (T): 0 = off; > 0 = apply
                               U += theta dU with the largest theta <= 1 that keeps |B| <= b_cap
                               in every Brauer element and sample, when the full correction
                               would exceed it (a frozen linear coarse model cannot saturate) */
    int32_t coarse_mode;    /* PP-PC coarse problem: 0 = frozen (the time-averaged
                               linearisation Kbar, one harmonic solve per correction); 1 =
                               nonlinear: eq. (4) with G the implicit-Euler step of size dT on
                               the full K(u) (eq. (8)), a block-cyclic nonlinear system solved
                               by Newton's method to ||Phi|| <= max(tol_cocg ||Phi_0||,
                               1e-14 ||C F||_F), each Newton step by flexible GMRES (at most 30
                               vectors) preconditioned by the frozen harmonic solve.  Not with
                               method 1, n_harm or b_cap; not for batched problems */
    int32_t lin_start;      /* start of each fine-step PCG solve: 2 = for the first Newton
                               correction of a step, the Galerkin projection of the Newton
                               system on the chain's last three first corrections (x0 in their
                               span minimising the J-norm error; the same solution to the PCG
                               tolerance, fewer iterations), zero for later corrections of the
                               step; 1 = zero;
                               0 = by precision: the Galerkin start with FP64 PCG (precision
                               0), zero with FP32 PCG (precision 1), whichever measured faster.
                               The adjoint's solves start from zero */
    int32_t lin_forcing;    /* tolerance of each fine-step PCG solve: 0 = tol_lin relative to
                               ||R||; 1 = forcing terms: after a step that needed several Newton
                               iterations the first solve is held to max(tol_lin, 1e-3), later
                               ones to eta = 0.9 (||R_k|| / ||R_{k-1}||)^2 (safeguarded, within
                               [tol_lin, 0.1]), so that linear solves are not pushed far below
                               what the Newton step can use.  Always at least 0.5 tol_newton
                               scale; the step is solved to tol_newton either way */
    ppc_progress_fn progress; /* null (default) or the progress callback of ppc_solve */
    void* progress_user;      /* passed to progress unchanged */
    double tol_adapt;       /* 0 (default): every fine sweep of ppc_solve solves its Newton steps
                               to tol_newton.  theta > 0: the sweep of outer iteration k uses
                               max(tol_newton, min(1e-6, theta eps_{k-1})), eps_{k-1} the
                               previous iteration's ||J||_F / ||U||_F (1e-6 for the first
                               sweep), so early iterations, whose iterate is still far from the
                               fixed point, do not pay for fine solves far more accurate than
                               that distance; once eps falls to tol_newton / theta the sweeps
                               are the plain ones.  In [0, 1).  ppc_solve (each design of a
                               batch by its own eps) only: ppc_fine_sweep and the adjoint's
                               sweeps use tol_newton */
} ppc_params;

/* Counters and timings of the last solve (all chains, all iterations). */
typedef struct {
    int32_t status;
    int32_t iterations;          /* coarse corrections applied (fine sweeps = iterations+1) */
    int32_t fine_launches;       /* fine-sweep kernel launches */
    int32_t coarse_solves;       /* COCG launches (PP-PC: one per correction over all
                                    harmonics; PP-IC: N per correction) */
    int64_t newton_total;        /* Newton iterations over every chain and step */
    int64_t lin_total;           /* PCG iterations over every chain */
    int64_t cocg_total;          /* COCG iterations summed over harmonics */
    int32_t newton_max;          /* largest Newton count of one fine step */
    int32_t lin_max;             /* largest PCG count of one Newton step */
    int32_t cocg_max;            /* largest COCG count of one harmonic solve */
    int32_t lin_capped;          /* PCG solves that hit max_lin */
    double fine_ms;              /* device time in fine-sweep kernels (hipEvents) */
    double coarse_ms;            /* device time in the coarse correction */
    double total_ms;             /* device time of the whole solve */
    double jump;                 /* ||U_0 - F_N(U_{N-1})|| of the last sweep (eq. (4), n=0) */
    double eps;                  /* last ||J||_F / ||U||_F */
    double max_b_steel;          /* max |B| over nonlinear elements at the returned U (T) */
    int32_t n_free, nnz, n_tri, damped;   /* damped: corrections the b_cap safeguard scaled */
    int64_t resid_total;         /* residual evaluations (element + node passes) */
    int64_t steps_total;         /* implicit-Euler steps taken over every chain */
    int32_t coarse_newton;       /* coarse_mode 1: Newton iterations of the coarse problems */
    int32_t coarse_krylov;       /* coarse_mode 1: GMRES iterations (= harmonic-solve sets) */
} ppc_stats;

/* ABI version (PPC_ABI_VERSION). */
int ppc_version(void);

/* Defaults: T = 0.02, N = 10, m = 20, shift 0, lin 0, init 0, FP64, tol_ppc 1e-12,
 * max_iters 60, tol_newton 1e-13, max_newton 50, tol_lin 1e-8, max_lin 20000,
 * tol_cocg 1e-10, max_cocg 20000, block 0, predictor on, lin_point 1 (fine results),
 * coarse_precision -1, graph 1, method 0, fine_block 0, n_harm 0, b_cap 0.
 * Returns PPC_ERR_ARG on a null pointer. */
int ppc_params_default(ppc_params* p);

/* Message of the last error on this handle (never null; valid until the next call on
 * the handle).  With a null handle: the last error of a failed ppc_create or of a
 * host-only call on this thread. */
const char* ppc_last_error(const ppc_handle* h);

/* Host-only check of a problem description (Section 2, eq. (1) inputs).  Returns
 * PPC_OK, PPC_ERR_ARG or PPC_ERR_MESH; touches no device.  msg may be null. */
int ppc_validate(const ppc_mesh* mesh, const ppc_material* mat, const ppc_excitation* exc,
                 char* msg, int32_t msg_len);

/* Host-only check of solver parameters against a problem size (N even, m >= 1, ...). */
int ppc_validate_params(const ppc_params* p, char* msg, int32_t msg_len);

/* Open a handle on GPU `device`: sets the device, creates the library's stream and
 * events.  PPC_ERR_DEVICE when no GPU is present.  *out is null on failure. */
int ppc_create(int32_t device, ppc_handle** out);

/* Release a handle (null-safe).  Problems created on it must be destroyed first. */
int ppc_destroy(ppc_handle* h);

/* Copy a problem to the device and run the set-up kernels: element gradient
 * coefficients, areas, unit stiffness K0_e, conductivity mass M, load F, the CSR
 * pattern of the free nodes and the element->entry maps (Section 2, eq. (1) with P1
 * elements).  Validates first (as ppc_validate).  *out is null on failure. */
int ppc_problem_create(ppc_handle* h, const ppc_mesh* mesh, const ppc_material* mat,
                       const ppc_excitation* exc, ppc_problem** out);

/* Copy n_designs independent problems (e.g. cable designs of uneven size) to the device
 * as one batched problem.  Each design is validated and set up as by ppc_problem_create.
 * ppc_solve / ppc_solve_device on a batched problem run PP-PC on every design at once:
 * the fine sweeps of all active designs share launches and their harmonic solves share
 * one COCG launch; each design stops at its own eps <= tol_ppc.  Batched layouts:
 * U_init / U_out are the designs' [N * n_nodes_d] blocks concatenated in design order;
 * resid_out is [n_designs][max_iters + 1]; iters_out is [n_designs]; stats are summed
 * (eps: the largest final eps).  ppc_fine_sweep_device runs a batched sweep of every
 * design; ppc_coarse_correction_device, ppc_fine_sweep_noalloc and ppc_fine_counts reject
 * batched problems (PPC_ERR_ARG). */
int ppc_problem_create_batch(ppc_handle* h, int32_t n_designs, const ppc_mesh* meshes,
                             const ppc_material* mats, const ppc_excitation* excs,
                             ppc_problem** out);

/* Designs of a problem (1 for a single one) and, if non-null, each design's node and
 * free-node counts (host arrays [n_designs]). */
int ppc_batch_info(const ppc_problem* pr, int32_t* n_designs, int32_t* n_nodes, int32_t* n_free);

/* Free a problem's device memory (null-safe). */
int ppc_problem_destroy(ppc_problem* pr);

/* Sizes of a problem: free nodes, CSR entries among free nodes, triangles, nodes
 * (summed over the designs of a batched problem). */
int ppc_problem_info(const ppc_problem* pr, int32_t* n_free, int32_t* nnz, int32_t* n_tri,
                     int32_t* n_nodes);

/* Periodic steady state by PP-PC (Section 2, eq. (4); coarse problem of eqs. (8)-(10)
 * solved per harmonic after a DFT along time, Section 3, eqs. (11)-(14)).
 *   U_init     host, [N * n_nodes] or null (then params->init_mode decides U^0)
 *   U_out      host, [N * n_nodes]: the returned coarse samples U_n (row n = time T_n)
 *   resid_out  host, [max_iters + 1] or null: eps^k = ||J^k||_F / ||U^k||_F per sweep
 *   iters_out  host, or null: coarse corrections applied
 *   stats      host, or null
 * Returns PPC_OK, PPC_NOT_CONVERGED (outputs hold the last iterate) or an error. */
int ppc_solve(ppc_handle* h, ppc_problem* pr, const ppc_params* p, const double* U_init,
              double* U_out, double* resid_out, int32_t* iters_out, ppc_stats* stats);

/* As ppc_solve with U_init / U_out as DEVICE pointers on the handle's GPU; the work is
 * ordered on `stream` (a hipStream_t, null = the library's stream) and complete on
 * return.  resid_out, iters_out and stats stay host pointers.  ppc_solve is this call
 * plus host<->device copies. */
int ppc_solve_device(ppc_handle* h, ppc_problem* pr, const ppc_params* p,
                     const double* U_init_dev, double* U_out_dev, double* resid_out,
                     int32_t* iters_out, ppc_stats* stats, void* stream);

/* Classical time stepping, the sequential method that parallel-in-time iterations are
 * measured against (Section 1): the implicit-Euler fine propagator of eqs. (2)-(3) run as
 * one chain over whole periods (N m steps of dt = T/(N m) each, one launch per period, one
 * workgroup), from u(0) = u_start, until the samples u(T_n) of two consecutive periods
 * agree: max_n ||U_n^(p) - U_n^(p-1)|| <= tol_ppc max_n ||U_n^(p)||.  At most max_iters
 * periods.  The problem's workspace is resized for one chain (a later PP-PC solve resizes
 * it back).
 *   u_start_dev  DEVICE [n_nodes] or null (zero)
 *   U_prev_dev   DEVICE [N * n_nodes] or null: the samples of the period that ended at
 *                u_start, so that a long run can be split into calls without losing a
 *                comparison (null: the first period is only a reference)
 *   U_out_dev    DEVICE [N * n_nodes]: the last period's samples, row n = u(T_n) with row 0
 *                the period's end u(T) (the layout of ppc_solve)
 *   periods_out  host or null: periods stepped in this call
 *   stats        host or null: fine counters; eps = the last relative sample change
 * Returns PPC_OK when periodic, PPC_NOT_CONVERGED after max_iters periods. */
int ppc_time_stepping_device(ppc_handle* h, ppc_problem* pr, const ppc_params* p, const double* u_start_dev,
                             const double* U_prev_dev, double* U_out_dev, int32_t* periods_out, ppc_stats* stats,
                             void* stream);

/* Autotuner of the fine sweep's register-row workgroup size (256, 512 or 1024 threads; a
 * smaller workgroup takes more rows per thread).  For each size whose rows fit the mesh it
 * times one fine sweep from U = 0 in the problem's workspace (overwriting the workspace
 * state; the next solve starts afresh), best of two after a warm-up, and keeps the fastest
 * for params->precision: later sweeps and solves with params->fine_block = 0 use it.
 * Meshes that take the memory path (rows beyond registers and LDS) have nothing to tune
 * and report 0.  A batched problem is tuned on its batched sweep: policy b (256, 512,
 * 1024) puts every design at b threads or at the next larger size its rows fit, and the
 * fastest policy is kept (designs of one size class share a size).  The adjoint sweep
 * keeps 1024 threads.
 *   block_out  host [1] (single) or [n_designs] (batch), or null: the chosen size (0 =
 *              memory path)
 *   ms_out     host [3] or [3 n_designs], or null: sweep ms at 256, 512, 1024 threads
 *              (single: NaN = does not fit); a batch gives every design the three policy
 *              times of the whole batched sweep
 * PPC_ERR_ARG when params->fine_block is set. */
int ppc_autotune(ppc_handle* h, ppc_problem* pr, const ppc_params* p, int32_t* block_out, double* ms_out);

/* Adjoint gradients of the period-averaged eddy-current loss at a periodic steady state
 * (the state of eq. (1) that ppc_solve returns).  With the periodic implicit-Euler fine
 * trajectory u_j, j = 1..L = N m, the loss is
 *     P = 1/(T dt) sum_j (u_j - u_{j-1})^T M (u_j - u_{j-1})      (W/m, sigma (dA/dt)^2)
 * and its gradient follows from the periodic adjoint
 *     J_j lambda_j = (M/dt) lambda_{j+1} + dP/du_j,   lambda_{L+1} = lambda_1,
 * solved by a backward fine sweep (one launch; each chain replays its forward states
 * from the checkpoint U_{n-1}) inside a PP-PC iteration whose coarse correction is the
 * harmonic solve of Section 3 applied to the time-reversed jumps.  The adjoint solves
 * are FP64 (relative tolerance 1e-12) whatever params->precision says; the adjoint
 * iteration stops at ||jumps|| / ||Lambda|| <= tol_ppc (params->method does not apply).
 *   U_periodic  host, [N * n_nodes]: the converged coarse samples (checkpoints)
 *   loss        host scalar or null
 *   dsigma      host [n_tri] or null: dP/dsigma_e (per element)
 *   dbrauer     host [n_mat * 3] or null: dP/d(k1, k2, k3) per material (0 for linear)
 *   iters_out   host or null: adjoint coarse corrections applied
 * With dsigma and dbrauer both null only the loss is computed (one forward replay, no
 * adjoint iteration).  Single designs only (PPC_ERR_ARG for a batched problem). */
int ppc_adjoint(ppc_handle* h, ppc_problem* pr, const ppc_params* p, const double* U_periodic,
                double* loss, double* dsigma, double* dbrauer, int32_t* iters_out, ppc_stats* stats);

/* One fine sweep (Section 2, eqs. (2)-(3)): F_out[n mod N] = F_n(U_in[n-1]) for
 * n = 1..N, all chains in one launch.  U_in / F_out are DEVICE pointers
 * [N * n_nodes]; newton_out / lin_out are host [N] or null (per-chain Newton and PCG
 * iteration totals).  On a batched problem every design's chains run in one batched
 * launch per kernel shape; U_in / F_out then hold design d's N x n_nodes_d rows after
 * those of design d - 1 (the layout of ppc_solve on a batch), newton_out / lin_out are
 * [n_designs * N].  Returns PPC_ERR_NEWTON / PPC_ERR_NONFINITE if a chain failed. */
int ppc_fine_sweep_device(ppc_handle* h, ppc_problem* pr, const ppc_params* p,
                          const double* U_in_dev, double* F_out_dev, int32_t* newton_out,
                          int32_t* lin_out, void* stream);

/* Size of the static device scratch of ppc_fine_sweep_noalloc, in MiB. */
#define PPC_NOALLOC_SCRATCH_MB 96

/* ppc_fine_sweep_device for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the same fine
 * sweep with the same kernels and results, but every per-sweep buffer (free-row copies of
 * U and F, base Jacobian, chain vectors, PCG vectors, Jacobian values, Brauer element
 * planes, chain counters) lives in one static device array of PPC_NOALLOC_SCRATCH_MB MiB
 * per GPU, held from the library's first ppc_create on that GPU until the process ends.
 * The call allocates no device or pinned memory and does not touch the problem's
 * workspace, so it may run between the problem's solves.  It still synchronises `stream`
 * once to read the chain counters (status, newton_out, lin_out).
 *   U_in_dev / F_out_dev  DEVICE [N * n_nodes], as ppc_fine_sweep_device
 *   newton_out / lin_out  host [N] or null
 * Every call on one GPU shares that GPU's scratch: calls that overlap in time on one GPU
 * (other host threads, other handles, other streams) race and must be serialised by the
 * caller.  Nothing in the scratch needs clearing between calls: each sweep writes every
 * value it reads.  PPC_ERR_ARG when N > 1024 or the sweep needs more than the scratch holds
 * (about N n (88 + 11 s) + N vals s + 8 vals bytes for n free nodes, vals ELL value
 * positions and s = 8 (FP64) or 4 (mixed); 40 chains of 7,081 free nodes in FP64 take
 * about 75 MB), before any device work. */
int ppc_fine_sweep_noalloc(ppc_handle* h, ppc_problem* pr, const ppc_params* p,
                           const double* U_in_dev, double* F_out_dev, int32_t* newton_out,
                           int32_t* lin_out, void* stream);

/* Per-chain counters of the last fine sweep run on this problem (by
 * ppc_fine_sweep_device, or the last sweep of a solve).  counts is host
 * [n_chains * 8], per chain: status, Newton iterations, PCG iterations, the largest
 * Newton count of one step, the largest PCG count of one Newton step, PCG solves that
 * stopped at max_lin, failing step (-1: none), residual evaluations.  n_chains must be
 * the N of that sweep; PPC_ERR_ARG for a batched problem, a null pointer, a different
 * N or no sweep yet.  Blocks until the counters are on the host. */
int ppc_fine_counts(const ppc_problem* pr, int32_t n_chains, int32_t* counts);

/* One coarse correction (Section 3, eqs. (11)-(14), in correction form): from the
 * samples U and jumps J (DEVICE [N * n_nodes]; J[n] = F_n - U_n mod N) compute
 * dU (DEVICE [N * n_nodes]) solving Q dU_n - C dU_{n-1} = Q J_n cyclically, with
 * C = M/dT, Q = C + Kbar(U) (eq. (10)).  With params->n_harm the harmonics from n_harm
 * on are those of J instead.  With params->coarse_mode = 1, dU = U^{k+1} - U^k of eq. (4)
 * with the nonlinear coarse step instead, F = U + J being the fine results (host-driven
 * Newton-GMRES; synchronises once per Krylov step).  cocg_out: host [N/2 + 1] or null (COCG
 * iterations per harmonic, summed over the Krylov steps in coarse_mode 1; 0 for the
 * harmonics not solved). */
int ppc_coarse_correction_device(ppc_handle* h, ppc_problem* pr, const ppc_params* p,
                                 const double* U_dev, const double* J_dev, double* dU_dev,
                                 int32_t* cocg_out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PPCMH_H */

// Internal declarations of the PP-PC library (not part of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ppcmh.h"

namespace ppc {

constexpr int kMaxHarmonicTerms = 16;   // terms of the excitation waveform i(t)
constexpr int kMaxMaterials = 64;   // validated bound of the material table
constexpr int kFineBlock = 1024;        // default fine-kernel workgroup
constexpr int kCocgBlock = 1024;
constexpr int kRowGroup = 8;            // lanes per CSR row in the vector SpMV
constexpr int kEllMaxWidth = 8;         // rows longer than this go to the ELL tail
constexpr size_t kLdsBudget = 160 * 1024 - 4096;   // dynamic LDS per workgroup (of 160 KB)

// ----------------------------------------------------------------------------------
// error plumbing: every internal failure throws ppc::Error, caught at the C-ABI
// ----------------------------------------------------------------------------------
struct Error {
    int code;
    std::string msg;
};

[[noreturn]] void fail(int code, const std::string& msg);
void hip_check(hipError_t e, const char* what);
#define PPC_HIP(call) ::ppc::hip_check((call), #call)

// Waveform of the imposed current, passed by value to kernels.
struct Wave {
    double f0;
    int n_h;
    int order[kMaxHarmonicTerms];
    double amp[kMaxHarmonicTerms];
    double phase[kMaxHarmonicTerms];
};

// Material laws, passed by value to kernels.
struct Laws {
    int n_mat;
    int law[kMaxMaterials];
    double nu[kMaxMaterials], k1[kMaxMaterials], k2[kMaxMaterials], k3[kMaxMaterials];
};

// Device-resident problem: pattern, maps and element geometry.  Element arrays are
// stored as planes (structure of arrays) of length n_tri.
struct DeviceMesh {
    int n_nodes = 0, n_tri = 0, n_free = 0, nnz = 0;
    int max_row = 0;           // longest CSR row
    // CSR pattern of the free block
    int* rowptr = nullptr;     // [n_free + 1]
    int* colidx = nullptr;     // [nnz]
    int* diag = nullptr;       // [n_free] slot of the diagonal entry
    // slot -> element contributions, each coded e*9 + a*3 + b
    int* slot_ptr = nullptr;   // [nnz + 1]
    int* slot_src = nullptr;   // [n_contrib]
    // free node -> incident (element, local vertex), coded e*3 + a
    int* node_ptr = nullptr;   // [n_free + 1]
    int* node_src = nullptr;   // [3 * n_tri] (only free vertices)
    int* efree = nullptr;      // [3][n_tri] free index of each vertex, -1 on Dirichlet
    int* free_node = nullptr;  // [n_free] mesh node of each free index
    int* mat = nullptr;        // [n_tri]
    double* xy = nullptr;      // [2 * n_nodes]
    int* tri = nullptr;        // [3 * n_tri]
    // geometry (set-up kernel)
    double* area = nullptr;    // [n_tri]
    double* k0 = nullptr;      // [6][n_tri]: K0 entries 00 01 02 11 12 22
    double* gx = nullptr;      // [3][n_tri] d(phi_a)/dx
    double* gy = nullptr;      // [3][n_tri] d(phi_a)/dy
    double* sigma = nullptr;   // [n_tri]
    double* js = nullptr;      // [n_tri]
    double* mval = nullptr;    // [nnz] conductivity mass M
    float* mval32 = nullptr;   // [nnz] FP32 copy for the mixed harmonic solves
    double* mdiag = nullptr;   // [n_free]
    double* fload = nullptr;   // [n_free] load per ampere F
    double fnorm = 0.0;        // ||F||_2
    // ELL copy of the pattern for the fine-sweep SpMV: rows of length <= ell_w are stored
    // column-major [ell_w][n_pad]; longer rows ("tail" rows) are stored whole in a
    // separate CSR block whose value positions follow the ELL block.
    int ell_w = 0;             // ELL width
    int n_tail = 0;            // rows stored in the tail
    int tail_nnz = 0;
    int n_vals = 0;            // value positions: ell_w * n_pad + tail_nnz
    int* ecol = nullptr;       // [ell_w][n_pad]; tail rows: ecol[0][i] = -1, ecol[1][i] = tail index
    unsigned short* ecol16 = nullptr;   // same columns as 16-bit indices (n < 65536), tail rows 0
    int* vslot = nullptr;      // [n_vals] CSR slot of each value position (-1: padding)
    double* mell = nullptr;    // [n_vals] conductivity mass M at each value position (padding 0)
    int* dpos = nullptr;       // [n_free] value position of the diagonal
    int* tail_row = nullptr;   // [n_tail]
    int* tail_ptr = nullptr;   // [n_tail + 1]
    int* tail_col = nullptr;   // [tail_nnz]
    size_t ell_pad = 0;        // n_pad used by the ELL arrays
    bool nonlinear = false;    // any element with a Brauer law
    int n_contrib = 0;
    // Brauer (nonlinear) elements in a compact numbering j, and the ELL value positions
    // and rows that their Jacobian and force contributions reach.  Everything else in
    // the fine-sweep Jacobian and residual is affine in the state (the base matrix).
    int n_nl = 0;              // Brauer elements
    int* nl_elem = nullptr;    // [n_nl] element of each j
    int* nl_efree = nullptr;   // [3][n_nl] free index of each vertex, -1 on Dirichlet
    int* nl_mat = nullptr;     // [n_nl]
    double* nl_area = nullptr; // [n_nl]
    double* nl_k0 = nullptr;   // [6][n_nl]
    int n_nlv = 0;             // ELL value positions with Brauer contributions
    int* nlv_val = nullptr;    // [n_nlv] value position
    int* nlv_ptr = nullptr;    // [n_nlv + 1]
    int* nlv_src = nullptr;    // codes j*9 + a*3 + b
    int* nlf_ptr = nullptr;    // [n_free + 1] per row: incident Brauer elements
    int* nlf_src = nullptr;    // codes j*3 + a
};

void mesh_free(DeviceMesh& d);

struct Workspace {
    int N = -1, precision = -1;
    // fine sweep
    double* fvec = nullptr;    // [N][kFineVec][n_pad] FP64 Newton vectors
    void* fpcg = nullptr;      // [N][kPcgVec][n_pad] PCG vectors (FP64 or FP32)
    void* fjac = nullptr;      // [N][nnz_pad] Jacobian values
    double* felem = nullptr;   // [N][8][nl_pad] Brauer element scratch
    double* jbase = nullptr;   // [vals_pad] base Jacobian M/dt + sum over linear elements
    double jbase_dt = 0.0;     // dt the base Jacobian was built for (0: none)
    int* fcount = nullptr;     // [N][8] counters per chain
    // PP-PC state (free layout [N][n_free])
    double* U = nullptr;
    double* F = nullptr;
    double* J = nullptr;
    double* R = nullptr;
    // coarse
    double* kbar = nullptr;    // [nnz]
    float* kbar32 = nullptr;   // [nnz] FP32 copy for the mixed harmonic solves
    double* nubar = nullptr;   // [3][n_tri]
    double2* rhat = nullptr;   // [2][H][n_free]: right-hand sides, then solutions
    double2* cwork = nullptr;  // [H][4][n_pad] COCG vectors r p q dinv
    double2* ckm = nullptr;    // [vals_pad] (Kbar, M) pairs in ELL order
    double2* sig = nullptr;    // [H] shifts sigma_p
    int* ccount = nullptr;     // [N][4] (PP-PC uses the first H rows, PP-IC one row per step)
    double* ic_e = nullptr;    // [n_free] PP-IC: U^{k+1}_{n-1} - U^k_{n-1} of the current step
    double* ic_un = nullptr;   // [n_free] PP-IC: U_N of the last propagation (next U_0)
    double2* twiddle = nullptr;// [N]
    double* partial = nullptr; // reduction partials
    double* scal = nullptr;    // small scalars
    double* host_scal = nullptr; // pinned host mirror
    int* host_fcount = nullptr;  // pinned [N][8] chain counters of the last sweep
    int* host_ccount = nullptr;  // pinned [N][4] coarse-solve counters
    // nonlinear periodic coarse problem (allocated on first use; layouts [N][n_free])
    double* nlc_jb = nullptr;    // [vals_pad] base Jacobian M/dT + linear elements
    double nlc_jb_dt = 0.0;      // step the nlc_jb was built for (0: none)
    double* nlc_jac = nullptr;   // [N][vals_pad] Jacobian of each row's coarse step
    double* nlc_vec = nullptr;   // [kNlcVec][N][n_free]: G(U^k), b, W, W trial, U, Phi, delta
    double* nlc_kry = nullptr;   // [2 kNlcKrylov + 1][N][n_free] Krylov basis V, then Z
    double* nlc_part = nullptr;  // reduction partials
    double* nlc_h = nullptr;     // [4][kNlcKrylov + 1] dot products and coefficients
    double* nlc_host = nullptr;  // pinned host mirror of nlc_h
    size_t n_pad = 0, nnz_pad = 0, ne_pad = 0, vals_pad = 0, nl_pad = 0;
};

void workspace_free(Workspace& w);

// nonlinear coarse problem: work vectors and the Krylov space of one Newton step
constexpr int kNlcVec = 7;
constexpr int kNlcKrylov = 30;

}  // namespace ppc

struct ppc_handle {
    int device = 0;
    hipStream_t stream = nullptr;
    hipEvent_t ev[8] = {};
    // side streams (default priority) for launches that may overlap on the device: the
    // kernel-shape groups of a batched fine sweep; fork / join events order them with the
    // main stream (and record the same dependencies under graph capture)
    static constexpr int kSide = 3;
    hipStream_t side[kSide] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kSide] = {};
    std::string last_error;
    int n_problems = 0;
};

struct ppc_problem {
    ppc_handle* h = nullptr;
    ppc::DeviceMesh mesh;
    ppc::Wave wave{};
    ppc::Laws laws{};
    ppc::Workspace ws;
    std::vector<int> free_of_node;   // host map node -> free index (-1 Dirichlet)
    std::vector<int> nl_elem;        // host list of Brauer elements
    double* lawtab = nullptr;        // device [n_mat][5]: law, nu, k1, k2, k3
    double* wavtab = nullptr;        // device [n_h][3]: order, amp, phase
    // register-row workgroup size chosen by ppc_autotune per precision (0: not tuned)
    int tuned_block[2] = {0, 0};
    // batched problem: one sub-problem per design (the fields above are unused then)
    std::vector<ppc_problem*> parts;
    bool batch = false;
};

namespace ppc {

// Arguments of one design's fine sweep (device pointers and sizes).
struct FineArgs {
    int n, N, m;
    double T, dt, fnorm;
    double tol_newton, tol_lin;
    int max_newton, max_lin;
    const int* rowptr;
    const int* colidx;
    const double* mval;
    const double* fload;
    const double* lawtab;   // [n_mat][5]: law, nu, k1, k2, k3
    const double* wavtab;   // [n_h][3]: order, amp, phase
    int n_h;
    double f0;
    const double* U;        // [N][n]
    double* F;              // [N][n]
    double* vec;            // [N][kFineVec][n_pad]
    void* pcg;              // [N][kPcgVec][n_pad] of S
    void* jac;              // [N][nnz_pad] of S
    double* elem;           // [N][8][nl_pad] Brauer element scratch
    int* count;             // [N][8]
    long n_pad, vals_pad, nl_pad;
    // state-independent base Jacobian and the Brauer part
    const double* jbase;    // [nvals]
    int n_nl, n_nlv;
    const int* nl_efree;
    const int* nl_mat;
    const double* nl_area;
    const double* nl_k0;
    const int* nlv_val;
    const int* nlv_ptr;
    const int* nlv_src;
    const int* nlf_ptr;
    const int* nlf_src;
    const double* mell;     // [nvals] M in the ELL value order
    // ELL pattern of the fine-sweep SpMV
    int W, ntail, nvals;
    int predictor;
    int lin_start;          // 0: Galerkin start of the PCG from the last corrections; 1: zero
    int lin_forcing;        // 1: adaptive PCG tolerance per Newton iteration (forcing terms)
    double* traj;            // [N][m+1][n] fine trajectory of each chain, or null
    // tolerance that follows the outer iteration: with adapt_scal set (the squared norms
    // ||J||^2, ||U||^2 of the previous iteration's jumps and iterate) each step's Newton
    // tolerance is max(tol_newton, min(kAdaptCap, tol_adapt * ||J|| / ||U||))
    const double* adapt_scal;
    double tol_adapt;
    long ell_pad;
    const int* ecol;
    const unsigned short* ecol16;
    const int* dpos;
    const int* tail_row;
    const int* tail_ptr;
    const int* tail_col;
};

// Adjoint backward sweep: chain c maps Lambda_{c+1} = lambda_{(c+1)m+1} to
// lambda_{cm+1} through J_j lambda_j = (M/dt) lambda_{j+1} + dP/du_j.
struct AdjArgs {
    const double* traj;      // [N][m+1][n] forward trajectory per chain
    const double* lam_in;    // [N][n] Lambda_c
    double* lam_out;         // [N][n] B_c(Lambda_{c+1})
    double* lam_all;         // [N][m][n] lambda_j of the sweep
    double tol_lin;          // relative tolerance of each adjoint solve
    double T;
};

// Kernel shape of a design's fine sweep: register rows R (0: memory path), workgroup,
// LDS residency LP of the memory path, dynamic LDS bytes.
struct FineShape {
    int R, block, LP;
    size_t lds;
};

// Batched fine sweep over several designs (one descriptor per design on the device).
struct FineBatch {
    FineArgs* d_args = nullptr;
    int2* d_work = nullptr;
    size_t work_cap = 0;
    int N = 0, precision = 0;
    std::vector<FineShape> shapes;
    std::vector<int> sizes;
    std::vector<int2> host_work;
    ppc_handle* h = nullptr;   // side streams and events for concurrent shape groups
    // the planned launches: spans of d_work and the kernel shape of each
    std::vector<std::pair<size_t, size_t>> spans;
    std::vector<FineShape> span_shapes;
    void release();
    ~FineBatch() { release(); }
};

// Arguments of one design's harmonic COCG solves.
struct CocgArgs {
    int n, H;
    const int* rowptr;
    const int* colidx;
    const double* kbar;
    const double* mval;
    const int* diag;
    const double2* sig;
    const double2* B;
    double2* X;
    double2* work;
    long n_pad;
    double tol;
    int max_it;
    int* count;
    int mixed;               // 1: complex-FP32 inner COCG refined by FP64 residuals
    const float* kbar32;
    const float* mval32;
    // ELL form (FP64, meshes whose search direction fits LDS)
    const double2* km;       // [n_vals] (Kbar, M) pair of each ELL value position
    const unsigned short* ecol16;
    const int* ecol;
    const int* dpos;
    long ell_pad;
    int W, ntail;
    const int* tail_row;
    const int* tail_ptr;
    const int* tail_col;
};

constexpr int kFineVec = 9;   // u, u_prev, R, R_trial, u_{j-2}, trial state, M u_prev / dt, u_{j-3}, u_{j-4}
constexpr int kHist = 3;      // Newton corrections kept for the Galerkin start of the PCG
constexpr double kAdaptCap = 1e-6;   // loosest Newton tolerance of an adaptive fine sweep
constexpr int kPcgVec = 5 + 2 * kHist;   // r, p, q, x, dinv, the corrections, their J products

// set-up (setup.hip)
void build_problem(ppc_problem* pr, const ppc_mesh* mesh, const ppc_material* mat,
                   const ppc_excitation* exc, hipStream_t s);
int validate_problem(const ppc_mesh* mesh, const ppc_material* mat, const ppc_excitation* exc,
                     std::string& msg);
int validate_params(const ppc_params* p, std::string& msg);

// Harmonics a coarse correction solves: all N/2 + 1, or the first params->n_harm (the
// others take the jumps' harmonics).  Excitation solves (the initial iterate) use all.
inline int solved_harmonics(const ppc_params* p, bool excitation) {
    const int H = p->N / 2 + 1;
    return (excitation || p->n_harm <= 0 || p->n_harm > H) ? H : p->n_harm;
}

// workspace sizing (api.hip)
void ensure_workspace(ppc_problem* pr, const ppc_params* p);

// fine sweep (fine.hip): F[n mod N] = F_n(U[n-1]) for all chains, one launch
void launch_fine_sweep(ppc_problem* pr, const ppc_params* p, const double* U, double* F,
                       hipStream_t s, const double* adapt_scal = nullptr);
void fine_batch_prepare(FineBatch& b, const std::vector<ppc_problem*>& parts, const ppc_params* p,
                        hipStream_t s, const double* adapt_scal = nullptr);
void fine_batch_launch(FineBatch& b, const std::vector<char>& active, hipStream_t s);
// the same in two parts: the work list of the active designs uploaded (synchronises), then
// the kernel launches alone (what a captured graph replays)
void fine_batch_plan(FineBatch& b, const std::vector<char>& active, hipStream_t s);
void fine_batch_run(const FineBatch& b, hipStream_t s);
FineArgs make_fine_args(ppc_problem* pr, const ppc_params* p, const double* U, double* F);
FineShape fine_shape(const ppc_problem* pr, const ppc_params* p);
void launch_fine_sweep_traj(ppc_problem* pr, const ppc_params* p, const double* U, double* F,
                            double* traj, hipStream_t s);
// The per-sweep buffers of one fine sweep (base Jacobian, chain vectors, PCG vectors,
// Jacobian values, Brauer element planes, chain counters) placed in one caller-provided
// device region instead of the problem's workspace.
struct FineScratch {
    double* jbase = nullptr;
    double* vec = nullptr;
    void* pcg = nullptr;
    void* jac = nullptr;
    double* elem = nullptr;
    int* count = nullptr;
    long n_pad = 0, vals_pad = 0, nl_pad = 0;
};
// Lays the buffers out from `base` (256-byte aligned regions) and returns the bytes they
// take; with base == nullptr only the size is computed.
size_t fine_scratch_layout(const ppc_problem* pr, const ppc_params* p, unsigned char* base, FineScratch* out);
// The fine sweep of launch_fine_sweep (same kernels and shapes) on those buffers: the base
// Jacobian is rebuilt into sc.jbase, nothing is allocated.
void launch_fine_sweep_in(ppc_problem* pr, const ppc_params* p, const double* U, double* F,
                          const FineScratch& sc, hipStream_t s);
// register-row workgroup sizes the library builds, and the shape one of them gives a mesh
// (R = 0 when its rows do not fit registers and LDS at that size)
constexpr int kRowBlocks[3] = {256, 512, 1024};
FineShape rows_shape(const ppc_problem* pr, const ppc_params* p, int block);
// Times one fine sweep per register-row workgroup size that fits the mesh (from U = 0 in the
// problem's own workspace, best of two after a warm-up); ms[i] for kRowBlocks[i], NaN when
// it does not fit.  Returns the fastest size, 0 when the mesh takes the memory path.
int autotune_fine(ppc_problem* pr, const ppc_params* p, double ms[3], hipEvent_t e0, hipEvent_t e1,
                  hipStream_t s);
// 256- and 512-thread register-row kernels (fine_blocks.hip)
void launch_fine_rows_small(const FineArgs& a, int N, const FineShape& sh, bool fp64, hipStream_t s);
void launch_fine_batch_rows_small(const FineArgs* args, const int2* work, int nblocks, const FineShape& sh,
                                  bool fp64, hipStream_t s);
void launch_adjoint_sweep(ppc_problem* pr, const ppc_params* p, const AdjArgs& b, hipStream_t s);

// adjoint helpers (adjoint.hip)
void launch_reverse_rows(int N, int n, const double* src, double* dst, hipStream_t s);
void launch_add_reversed(int N, int n, const double* dR, double* L, hipStream_t s);
void launch_loss(ppc_problem* pr, const ppc_params* p, const double* traj, double* part, double* out,
                 hipStream_t s);
void launch_gradients(ppc_problem* pr, const ppc_params* p, const double* traj, const double* lam_all,
                      double* dsig, double* dk_elem, double* dk_mat, int n_mat, hipStream_t s);

// coarse correction pieces (coarse.hip)
void launch_jumps(ppc_problem* pr, int N, const double* U, const double* F, double* J,
                  double* out3, hipStream_t s);
void launch_coarse(ppc_problem* pr, const ppc_params* p, const double* U, const double* J,
                   double* dU, bool accumulate, bool excitation_rhs, hipStream_t s);
void launch_coarse_pre(ppc_problem* pr, const ppc_params* p, const double* U, const double* J,
                       bool excitation_rhs, hipStream_t s);
CocgArgs make_cocg_args(ppc_problem* pr, const ppc_params* p);
void launch_cocg_batch(const std::vector<ppc_problem*>& parts, const std::vector<int>& list,
                       const ppc_params* p, int H, const CocgArgs* d_args, int2* d_work, std::vector<int2>& cw,
                       hipStream_t s);
// the same in two parts: the (design, harmonic) work list uploaded (synchronises), then
// the COCG launches alone
struct CocgBatchPlan {
    struct Span {
        int R;
        size_t lds;
        int begin, count;
    };
    std::vector<Span> spans;
    std::vector<int2> cw;
};
void cocg_batch_plan(const std::vector<ppc_problem*>& parts, const std::vector<int>& list, const ppc_params* p,
                     int H, int2* d_work, CocgBatchPlan& plan, hipStream_t s);
void cocg_batch_run(const CocgBatchPlan& plan, const CocgArgs* d_args, const int2* d_work, hipStream_t s,
                    ppc_handle* h = nullptr);

// The main stream s and the handle's side streams as lanes for independent work: lane(i)
// forks a side stream from s's work so far on first use; join() makes s wait for every
// lane used (stream-ordered, so it also holds under graph capture).
struct Lanes {
    ppc_handle* h;
    hipStream_t s;
    bool used[ppc_handle::kSide] = {};
    Lanes(ppc_handle* h_, hipStream_t s_);
    hipStream_t lane(int i);
    void join();
};
// PP-IC coarse propagation (eq. (5) with the update of eq. (4)): frozen coarse stiffness at
// the current iterate U, then U_0 = U_N of the last propagation and, for n = 1..N in order,
// U^{k+1}_n = F_n + Q^{-1} C (U^{k+1}_{n-1} - U^k_{n-1}), Q = C + Kbar, C = M/dT; the value
// at n = N is kept for the next iteration's U_0.  Counters of step n in ccount row n-1.
void launch_ic_propagation(ppc_problem* pr, const ppc_params* p, hipStream_t s);
// time stepping: the N samples of one chain's period trajectory, and per-sample squared
// norms of A - B and of A (out [N][2])
void launch_gather_samples(int n, int N, int m, const double* traj, double* U, hipStream_t s);
void launch_sample_change(int n, int N, const double* A, const double* B, double* out, hipStream_t s);
void launch_coarse_post(ppc_problem* pr, const ppc_params* p, double* dU, bool accumulate,
                        hipStream_t s);
void launch_to_nodal(const ppc_problem* pr, int N, const double* Ufree, double* Unodal,
                     hipStream_t s);
void launch_to_free(const ppc_problem* pr, int N, const double* Unodal, double* Ufree,
                    hipStream_t s);
void launch_safeguarded_update(ppc_problem* pr, int N, double cap, const double* dU, double* U,
                               double* out3, hipStream_t s);
void launch_max_b(ppc_problem* pr, int N, const double* U, double* out, hipStream_t s);

// The frozen block-cyclic coarse solve as an operator: set-up (Kbar at the samples Ulin,
// twiddles, shifts), then z = G^{-1} r over all N/2 + 1 harmonics (G of eq. (9) with Kbar;
// counters of harmonic p in ccount row p).
void launch_coarse_setup(ppc_problem* pr, const ppc_params* p, const double* Ulin, hipStream_t s);
void launch_coarse_apply(ppc_problem* pr, const ppc_params* p, const double* r, double* z, hipStream_t s);

// Nonlinear periodic coarse correction (eq. (4) with the nonlinear G of eq. (8)); see
// nlcoarse.hip.  out = U^{k+1} (accumulate, out may be U) or U^{k+1} - U^k.
struct NlcCounts {
    int newton = 0, krylov = 0;
    int64_t cocg_total = 0, step_newton = 0;
    int cocg_max = 0;
};
void launch_nonlinear_correction(ppc_problem* pr, const ppc_params* p, const double* U, const double* F,
                                 double* out, bool accumulate, NlcCounts& cnt, int32_t* cocg_out,
                                 hipStream_t s);
// y += x over L values
void launch_vec_add(long L, const double* x, double* y, hipStream_t s);

}  // namespace ppc

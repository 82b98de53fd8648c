// C-ABI entry points and the PP-PC driver (Section 2, eq. (4); Section 3).
//
// Driver per iteration k (all arithmetic in kernels; the host only sequences launches
// and reads three scalars and the per-chain counters):
//   fine sweep F_n(U^k_{n-1}) for every chain in one launch;
//   jumps J_n = F_n - U^k_{n mod N}, eps^k = ||J||_F / ||U^k||_F (the tolerance quantity
//     of Section 4 is not stated in the paper; this is the reading);
//   stop and return U^k if eps^k <= tol;
//   coarse correction U^{k+1} = U^k + dU (linearise, right-hand side, DFT along time,
//     COCG per harmonic, inverse DFT + update).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>

#include "internal.hpp"

namespace ppc {

void fail(int code, const std::string& msg) { throw Error{code, msg}; }

void hip_check(hipError_t e, const char* what) {
    if (e == hipSuccess) return;
    const int code = (e == hipErrorOutOfMemory) ? PPC_ERR_OOM : PPC_ERR_DEVICE;
    fail(code, std::string(what) + ": " + hipGetErrorString(e));
}

namespace {

thread_local std::string g_thread_error;

size_t pad64(size_t n) { return (n + 63) / 64 * 64; }

template <typename T>
T* dalloc(size_t n) {
    void* p = nullptr;
    if (n == 0) n = 1;
    const hipError_t e = hipMalloc(&p, n * sizeof(T));
    if (e != hipSuccess) fail(PPC_ERR_OOM, "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed");
    return static_cast<T*>(p);
}

void set_msg(char* msg, int32_t len, const std::string& s) {
    if (!msg || len <= 0) return;
    const size_t k = std::min((size_t)len - 1, s.size());
    std::memcpy(msg, s.data(), k);
    msg[k] = '\0';
}

template <typename Fn>
int guarded(ppc_handle* h, Fn&& fn) {
    std::string err;
    int code = PPC_OK;
    try {
        return fn();
    } catch (const Error& e) {
        code = e.code;
        err = e.msg;
    } catch (const std::bad_alloc&) {
        code = PPC_ERR_OOM;
        err = "host allocation failed";
    } catch (const std::exception& e) {
        code = PPC_ERR_ARG;
        err = e.what();
    } catch (...) {
        code = PPC_ERR_ARG;
        err = "unknown failure";
    }
    if (h) h->last_error = err;
    g_thread_error = err;
    return code;
}

__global__ void k_fill(long n, double v, double* __restrict__ x) {
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) x[k] = v;
}

void fill(double* x, long n, double v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill, dim3(1024), dim3(256), 0, s, n, v, x);
    PPC_HIP(hipGetLastError());
}

float elapsed(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    PPC_HIP(hipEventElapsedTime(&ms, a, b));
    return ms;
}

// Static device scratch of ppc_fine_sweep_noalloc: one copy per GPU the library runs on,
// held until the process ends.  Host code never uses the array's name as an address: the
// device address of each GPU's copy comes from hipGetSymbolAddress at ppc_create (with that
// device current) and is kept in g_scratch_dev.
constexpr size_t kScratchBytes = (size_t)PPC_NOALLOC_SCRATCH_MB << 20;
constexpr int kScratchDevices = 64;
constexpr int kNoAllocMaxChains = 1024;
__device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
unsigned char* g_scratch_dev[kScratchDevices] = {};

// The device address of this device's scratch copy; the device must be current.  Called
// once per device (later calls return the stored address).
unsigned char* scratch_address(int device) {
    if (device < 0 || device >= kScratchDevices) fail(PPC_ERR_DEVICE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) fail(PPC_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_dev[device] = static_cast<unsigned char*>(ptr);
    }
    return g_scratch_dev[device];
}

}  // namespace

void workspace_free(Workspace& w) {
    void* ptrs[] = {w.fvec, w.fpcg, w.fjac, w.felem, w.jbase, w.ckm, w.fcount, w.U, w.F, w.J, w.R, w.kbar, w.kbar32,
                    w.nubar, w.rhat, w.cwork, w.sig, w.ccount, w.twiddle, w.partial, w.scal, w.ic_e, w.ic_un,
                    w.nlc_jb, w.nlc_jac, w.nlc_vec, w.nlc_kry, w.nlc_part, w.nlc_h};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (w.host_scal) (void)hipHostFree(w.host_scal);
    if (w.host_fcount) (void)hipHostFree(w.host_fcount);
    if (w.host_ccount) (void)hipHostFree(w.host_ccount);
    if (w.nlc_host) (void)hipHostFree(w.nlc_host);
    w = Workspace{};
}

void ensure_workspace(ppc_problem* pr, const ppc_params* p) {
    Workspace& w = pr->ws;
    if (w.N == p->N) return;
    workspace_free(w);
    const DeviceMesh& d = pr->mesh;
    const size_t N = p->N, H = N / 2 + 1;
    w.n_pad = pad64(d.n_free);
    w.nnz_pad = pad64(d.nnz);
    w.ne_pad = pad64(d.n_tri);
    w.vals_pad = pad64(d.n_vals);
    w.fvec = dalloc<double>(N * kFineVec * w.n_pad);
    w.fpcg = dalloc<double>(N * kPcgVec * w.n_pad);     // sized for FP64, also used as FP32
    w.fjac = dalloc<double>(N * w.vals_pad);
    w.nl_pad = pad64(std::max(d.n_nl, 1));
    w.felem = dalloc<double>(N * 8 * w.nl_pad);
    w.jbase = dalloc<double>(w.vals_pad);
    w.jbase_dt = 0.0;
    w.fcount = dalloc<int>(N * 8);
    w.U = dalloc<double>(N * d.n_free);
    w.F = dalloc<double>(N * d.n_free);
    w.J = dalloc<double>(N * d.n_free);
    w.R = dalloc<double>(N * d.n_free);
    w.kbar = dalloc<double>(d.nnz);
    w.kbar32 = dalloc<float>(d.nnz);
    w.nubar = dalloc<double>(3 * (size_t)d.n_tri);
    w.rhat = dalloc<double2>(2 * H * d.n_free);
    w.cwork = dalloc<double2>(H * 4 * w.n_pad);
    w.ckm = dalloc<double2>(w.vals_pad);
    w.sig = dalloc<double2>(H);
    w.ccount = dalloc<int>(N * 4);
    w.ic_e = dalloc<double>(d.n_free);
    w.ic_un = dalloc<double>(d.n_free);
    w.twiddle = dalloc<double2>(N);
    w.partial = dalloc<double>(256 * 3);
    w.scal = dalloc<double>(16);
    void* hp = nullptr;
    PPC_HIP(hipHostMalloc(&hp, 16 * sizeof(double), hipHostMallocDefault));
    w.host_scal = static_cast<double*>(hp);
    PPC_HIP(hipHostMalloc(&hp, 8 * N * sizeof(int), hipHostMallocDefault));
    w.host_fcount = static_cast<int*>(hp);
    PPC_HIP(hipHostMalloc(&hp, 4 * N * sizeof(int), hipHostMallocDefault));
    w.host_ccount = static_cast<int*>(hp);
    w.N = p->N;
}

int autotune_fine(ppc_problem* pr, const ppc_params* p, double ms[3], hipEvent_t e0, hipEvent_t e1,
                  hipStream_t s) {
    ensure_workspace(pr, p);
    Workspace& w = pr->ws;
    const int n = pr->mesh.n_free;
    int best = 0;
    double best_ms = INFINITY;
    for (int i = 0; i < 3; ++i) {
        ms[i] = NAN;
        ppc_params q = *p;
        q.fine_block = kRowBlocks[i];
        if (q.block == kFineBlock || rows_shape(pr, &q, kRowBlocks[i]).R == 0) continue;
        double t = INFINITY;
        for (int rep = 0; rep < 3; ++rep) {
            fill(w.U, (long)p->N * n, 0.0, s);
            PPC_HIP(hipEventRecord(e0, s));
            launch_fine_sweep(pr, &q, w.U, w.F, s);
            PPC_HIP(hipEventRecord(e1, s));
            PPC_HIP(hipEventSynchronize(e1));
            float f = 0.0f;
            PPC_HIP(hipEventElapsedTime(&f, e0, e1));
            if (rep > 0) t = std::min(t, (double)f);
        }
        ms[i] = t;
        if (t < best_ms) {
            best_ms = t;
            best = kRowBlocks[i];
        }
    }
    return best;
}

namespace {

struct SweepCounts {
    int status = 0;
    int64_t newton = 0, lin = 0, resid = 0;
    int newton_max = 0, lin_max = 0, capped = 0;
    int fail_chain = -1, fail_step = -1;
};

// Chain counters [N][8] (status, Newton, PCG, Newton max, PCG max, capped, failing step,
// residual evaluations) summed over the chains.
SweepCounts parse_chain_counts(const int* c, int N, int32_t* newton_out, int32_t* lin_out) {
    SweepCounts r;
    for (int k = 0; k < N; ++k) {
        const int* q = c + 8 * k;
        if (q[0] != 0 && r.status == 0) {
            r.status = q[0];
            r.fail_chain = k;
            r.fail_step = q[6];
        }
        r.newton += q[1];
        r.lin += q[2];
        r.newton_max = std::max(r.newton_max, q[3]);
        r.lin_max = std::max(r.lin_max, q[4]);
        r.capped += q[5];
        r.resid += q[7];
        if (newton_out) newton_out[k] = q[1];
        if (lin_out) lin_out[k] = q[2];
    }
    return r;
}

SweepCounts read_chain_counts(ppc_problem* pr, int N, hipStream_t s, int32_t* newton_out,
                              int32_t* lin_out) {
    PPC_HIP(hipMemcpyAsync(pr->ws.host_fcount, pr->ws.fcount, 8 * (size_t)N * sizeof(int),
                           hipMemcpyDeviceToHost, s));
    PPC_HIP(hipStreamSynchronize(s));
    return parse_chain_counts(pr->ws.host_fcount, N, newton_out, lin_out);
}

void check_sweep(const SweepCounts& c) {
    if (c.status != 0)
        fail(c.status, "fine chain " + std::to_string(c.fail_chain + 1) + " failed at step " +
                           std::to_string(c.fail_step) +
                           (c.status == PPC_ERR_NONFINITE ? " (non-finite residual)" : " (Newton did not converge)"));
}

// Harmonic-solve counters [H][4] (status, iterations, converged, refinements).
int parse_cocg(const int* c, int H, int32_t* cocg_out, int64_t* total, int* mx) {
    int status = 0;
    for (int p = 0; p < H; ++p) {
        if (c[4 * p] != 0 && status == 0) status = c[4 * p];
        if (cocg_out) cocg_out[p] = c[4 * p + 1];
        if (total) *total += c[4 * p + 1];
        if (mx) *mx = std::max(*mx, c[4 * p + 1]);
    }
    if (status != 0)
        fail(status, status == PPC_ERR_BREAKDOWN ? "COCG breakdown in a harmonic solve" : "non-finite COCG residual");
    return 0;
}

int read_cocg(ppc_problem* pr, int H, hipStream_t s, int32_t* cocg_out, int64_t* total, int* mx) {
    PPC_HIP(hipMemcpyAsync(pr->ws.host_ccount, pr->ws.ccount, 4 * (size_t)H * sizeof(int),
                           hipMemcpyDeviceToHost, s));
    PPC_HIP(hipStreamSynchronize(s));
    return parse_cocg(pr->ws.host_ccount, H, cocg_out, total, mx);
}

// An instantiated HIP graph, destroyed with its owner.
struct GraphExec {
    hipGraphExec_t exec = nullptr;
    ~GraphExec() {
        if (exec) (void)hipGraphExecDestroy(exec);
    }
};

// Record the launches and copies that f enqueues on s into g.  The capture always ends,
// also when f throws, so the stream is never left capturing.
template <class F>
void capture_graph(GraphExec& g, hipStream_t s, F&& f) {
    PPC_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    try {
        f();
    } catch (...) {
        hipGraph_t dropped = nullptr;
        (void)hipStreamEndCapture(s, &dropped);
        if (dropped) (void)hipGraphDestroy(dropped);
        throw;
    }
    hipGraph_t graph = nullptr;
    PPC_HIP(hipStreamEndCapture(s, &graph));
    const hipError_t e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    PPC_HIP(e);
}

hipStream_t pick_stream(ppc_handle* h, void* stream) {
    return stream ? static_cast<hipStream_t>(stream) : h->stream;
}

void check_handle_problem(ppc_handle* h, ppc_problem* pr) {
    if (!h) fail(PPC_ERR_ARG, "null handle");
    if (!pr) fail(PPC_ERR_ARG, "null problem");
    if (pr->h != h) fail(PPC_ERR_ARG, "problem belongs to another handle");
}

void check_params(const ppc_params* p) {
    std::string msg;
    const int rc = validate_params(p, msg);
    if (rc != PPC_OK) fail(rc, msg);
}

// Parameters of the nested start's solve: max(1, m / 25) fine steps per subinterval, eps
// to 1e-2 (Newton to 1e-8 and harmonic solves to 1e-4 of their scales, well below that), from
// rest when the correction safeguard is on (strongly saturating designs) and from the
// automatic start otherwise.
ppc_params nested_params(const ppc_params* p) {
    ppc_params q = *p;
    q.m = std::max(1, p->m / 25);
    q.tol_ppc = std::max(p->tol_ppc, 1e-2);
    q.tol_newton = std::max(p->tol_newton, 1e-8);
    q.tol_cocg = std::max(p->tol_cocg, 1e-4);
    q.init_mode = p->b_cap > 0.0 ? 3 : 0;
    q.coarse_mode = 0;
    return q;
}

int solve_batch_device(ppc_handle* h, ppc_problem* bp, const ppc_params* p, const double* U_init_dev,
                       double* U_out_dev, double* resid_out, int32_t* iters_out, ppc_stats* st,
                       hipStream_t s);

int solve_device(ppc_handle* h, ppc_problem* pr, const ppc_params* p, const double* U_init_dev,
                 double* U_out_dev, double* resid_out, int32_t* iters_out, ppc_stats* st,
                 hipStream_t s) {
    PPC_HIP(hipSetDevice(h->device));
    ensure_workspace(pr, p);
    Workspace& w = pr->ws;
    const DeviceMesh& d = pr->mesh;
    const int N = p->N, H = N / 2 + 1, n = d.n_free;
    ppc_stats S{};
    S.n_free = d.n_free;
    S.nnz = d.nnz;
    S.n_tri = d.n_tri;
    hipEvent_t* ev = h->ev;
    double nested_ms = 0.0;
    PPC_HIP(hipEventRecord(ev[4], s));
    if (U_init_dev) {
        launch_to_free(pr, N, U_init_dev, w.U, s);
    } else {
        int mode = p->init_mode;
        if (mode == 0) mode = d.nonlinear ? 2 : 1;
        if (mode == 4) {
            // nested start: PP-PC of the same problem with max(1, m / 25) fine steps per
            // subinterval to eps <= 1e-2 from the automatic start; its samples are U^0
            const ppc_params q = nested_params(p);
            ppc_stats Sq{};
            (void)solve_device(h, pr, &q, nullptr, nullptr, nullptr, nullptr, &Sq, s);
            S.fine_launches += Sq.fine_launches;
            S.fine_ms += Sq.fine_ms;
            S.newton_total += Sq.newton_total;
            S.lin_total += Sq.lin_total;
            S.newton_max = std::max(S.newton_max, Sq.newton_max);
            S.lin_max = std::max(S.lin_max, Sq.lin_max);
            S.lin_capped += Sq.lin_capped;
            S.resid_total += Sq.resid_total;
            S.steps_total += Sq.steps_total;
            S.cocg_total += Sq.cocg_total;
            S.cocg_max = std::max(S.cocg_max, Sq.cocg_max);
            S.coarse_solves += Sq.coarse_solves;
            S.coarse_ms += Sq.coarse_ms;
            nested_ms = Sq.total_ms;
            PPC_HIP(hipEventRecord(ev[4], s));   // the nested solve reused the solve's events
        } else if (mode == 2) {
            fill(w.U, (long)N * n, 0.0, s);
        } else if (mode == 3) {
            // one fine sweep from rest: U^0_n = F_n(0)
            fill(w.U, (long)N * n, 0.0, s);
            PPC_HIP(hipEventRecord(ev[0], s));
            launch_fine_sweep(pr, p, w.U, w.F, s);
            PPC_HIP(hipEventRecord(ev[1], s));
            const SweepCounts c = read_chain_counts(pr, N, s, nullptr, nullptr);  // synchronises
            S.fine_launches++;
            S.fine_ms += elapsed(ev[0], ev[1]);
            S.newton_total += c.newton;
            S.lin_total += c.lin;
            S.newton_max = std::max(S.newton_max, c.newton_max);
            S.lin_max = std::max(S.lin_max, c.lin_max);
            S.lin_capped += c.capped;
            S.resid_total += c.resid;
            S.steps_total += (int64_t)N * p->m;
            check_sweep(c);
            PPC_HIP(hipMemcpyAsync(w.U, w.F, sizeof(double) * (size_t)N * n, hipMemcpyDeviceToDevice, s));
        } else {
            launch_coarse(pr, p, nullptr, nullptr, w.U, false, true, s);
            read_cocg(pr, H, s, nullptr, &S.cocg_total, &S.cocg_max);
            S.coarse_solves++;
        }
    }
    // Device work of one PP-PC iteration: the fine sweep with the jump norms and the
    // chain counters copied to pinned host memory, then (if not converged) the coarse
    // correction with its counters.  With params->graph each part is captured once, at
    // its second use, and replayed; the first iteration runs eagerly (it also sets the
    // kernels' attributes and the base Jacobian, which capture must not do).
    const bool use_graph = p->graph != 0;
    const bool ic = p->method == 1;
    const int n_solves = ic ? N : solved_harmonics(p, false);   // coarse solves (counter rows) per correction
    // PP-IC: the first propagation starts from U_N = U^0_0
    if (ic) PPC_HIP(hipMemcpyAsync(w.ic_un, w.U, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    GraphExec g_fine, g_coarse;
    // adaptive Newton tolerance: each sweep reads the squared norms ||J||^2, ||U||^2 that
    // the previous iteration's jump kernel left in w.scal; zero before the first sweep
    const double* adapt = p->tol_adapt > 0.0 ? w.scal : nullptr;
    if (adapt) PPC_HIP(hipMemsetAsync(w.scal, 0, 2 * sizeof(double), s));
    auto fine_ops = [&]() {
        launch_fine_sweep(pr, p, w.U, w.F, s, adapt);
        launch_jumps(pr, N, w.U, w.F, w.J, w.scal, s);
        PPC_HIP(hipMemcpyAsync(w.host_scal, w.scal, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
        PPC_HIP(hipMemcpyAsync(w.host_fcount, w.fcount, 8 * (size_t)N * sizeof(int), hipMemcpyDeviceToHost, s));
    };
    const bool nlc = p->coarse_mode == 1;
    NlcCounts nc;
    auto coarse_ops = [&]() {
        const double* lin = p->lin_point == 1 ? w.F : w.U;
        if (nlc) {
            // nonlinear coarse problem: host-driven Newton-Krylov, never captured
            launch_nonlinear_correction(pr, p, w.U, w.F, w.U, true, nc, nullptr, s);
            return;
        }
        if (ic) {
            launch_ic_propagation(pr, p, s);
        } else if (p->b_cap > 0.0) {
            // correction into w.R (free after the DFT), then the safeguarded update
            launch_coarse(pr, p, lin, w.J, w.R, false, false, s);
            launch_safeguarded_update(pr, N, p->b_cap, w.R, w.U, w.scal + 8, s);
            PPC_HIP(hipMemcpyAsync(w.host_scal + 8, w.scal + 8, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
        } else {
            launch_coarse(pr, p, lin, w.J, w.U, true, false, s);
        }
        PPC_HIP(hipMemcpyAsync(w.host_ccount, w.ccount, 4 * (size_t)n_solves * sizeof(int),
                               hipMemcpyDeviceToHost, s));
    };
    auto run = [&](GraphExec& g, int k, auto& ops) {
        if (!use_graph || k == 0) {
            ops();
            return;
        }
        if (!g.exec) capture_graph(g, s, ops);
        PPC_HIP(hipGraphLaunch(g.exec, s));
    };
    int status = PPC_NOT_CONVERGED;
    int k = 0;
    for (k = 0; k <= p->max_iters; ++k) {
        PPC_HIP(hipEventRecord(ev[0], s));
        run(g_fine, k, fine_ops);
        PPC_HIP(hipEventRecord(ev[1], s));
        S.fine_launches++;
        PPC_HIP(hipStreamSynchronize(s));
        const SweepCounts c = parse_chain_counts(w.host_fcount, N, nullptr, nullptr);
        S.fine_ms += elapsed(ev[0], ev[1]);
        S.newton_total += c.newton;
        S.lin_total += c.lin;
        S.newton_max = std::max(S.newton_max, c.newton_max);
        S.lin_max = std::max(S.lin_max, c.lin_max);
        S.lin_capped += c.capped;
        S.resid_total += c.resid;
        S.steps_total += (int64_t)N * p->m;
        check_sweep(c);
        const double jj = w.host_scal[0], uu = w.host_scal[1], j0 = w.host_scal[2];
        const double eps = uu > 0.0 ? std::sqrt(jj) / std::sqrt(uu) : (jj == 0.0 ? 0.0 : INFINITY);
        if (!std::isfinite(jj)) fail(PPC_ERR_NONFINITE, "non-finite jump norm");
        if (resid_out) resid_out[k] = eps;
        S.eps = eps;
        S.jump = std::sqrt(j0);
        if (p->progress) p->progress(p->m, k, eps, 1, p->progress_user);
        if (eps <= p->tol_ppc) {
            status = PPC_OK;
            break;
        }
        if (k == p->max_iters) break;
        PPC_HIP(hipEventRecord(ev[2], s));
        if (nlc)
            coarse_ops();
        else
            run(g_coarse, k, coarse_ops);
        PPC_HIP(hipEventRecord(ev[3], s));
        PPC_HIP(hipStreamSynchronize(s));
        if (!nlc) parse_cocg(w.host_ccount, n_solves, nullptr, &S.cocg_total, &S.cocg_max);
        if (!ic && p->b_cap > 0.0 && w.host_scal[8] < 1.0) S.damped++;
        S.coarse_ms += elapsed(ev[2], ev[3]);
        S.coarse_solves += ic ? N : (nlc ? 0 : 1);
    }
    if (nlc) {
        // one harmonic-solve launch per GMRES iteration
        S.cocg_total += nc.cocg_total;
        S.cocg_max = std::max(S.cocg_max, nc.cocg_max);
        S.coarse_solves += nc.krylov;
        S.coarse_newton = nc.newton;
        S.coarse_krylov = nc.krylov;
    }
    S.iterations = std::min(k, p->max_iters);
    if (U_out_dev) launch_to_nodal(pr, N, w.U, U_out_dev, s);
    if (d.nonlinear) {
        launch_max_b(pr, N, w.U, w.scal + 4, s);
        PPC_HIP(hipMemcpyAsync(w.host_scal + 4, w.scal + 4, sizeof(double), hipMemcpyDeviceToHost, s));
    }
    PPC_HIP(hipEventRecord(ev[5], s));
    PPC_HIP(hipStreamSynchronize(s));
    S.max_b_steel = d.nonlinear ? w.host_scal[4] : 0.0;
    S.total_ms = elapsed(ev[4], ev[5]) + nested_ms;
    S.status = status;
    if (iters_out) *iters_out = S.iterations;
    if (st) *st = S;
    return status;
}


// ---------------------------------------------------------------------------------------
// batched designs: every design runs the same PP-PC iteration; the fine sweeps of all
// active designs share launches (one per kernel shape), the harmonic solves of all active
// designs share one COCG launch, and each design stops at its own eps <= tol.
// ---------------------------------------------------------------------------------------
struct DevBuf {
    void* p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
};

// Pinned host array: the target of device-to-host copies that a captured graph replays.
template <typename T>
struct PinnedBuf {
    T* p = nullptr;
    explicit PinnedBuf(size_t n) {
        void* q = nullptr;
        PPC_HIP(hipHostMalloc(&q, std::max<size_t>(n, 1) * sizeof(T), hipHostMallocDefault));
        p = static_cast<T*>(q);
    }
    ~PinnedBuf() { if (p) (void)hipHostFree(p); }
    PinnedBuf(const PinnedBuf&) = delete;
    PinnedBuf& operator=(const PinnedBuf&) = delete;
};

int solve_batch_device(ppc_handle* h, ppc_problem* bp, const ppc_params* p, const double* U_init_dev,
                       double* U_out_dev, double* resid_out, int32_t* iters_out, ppc_stats* st,
                       hipStream_t s) {
    PPC_HIP(hipSetDevice(h->device));
    if (p->method != 0) fail(PPC_ERR_ARG, "PP-IC (method 1) runs single-design problems only");
    if (p->coarse_mode != 0) fail(PPC_ERR_ARG, "the nonlinear coarse problem (coarse_mode 1) runs single-design problems only");
    auto& parts = bp->parts;
    const int D = (int)parts.size();
    const int N = p->N, H = N / 2 + 1, R1 = p->max_iters + 1;
    std::vector<size_t> off(D + 1, 0);
    for (int d = 0; d < D; ++d) {
        ensure_workspace(parts[d], p);
        off[d + 1] = off[d] + (size_t)N * parts[d]->mesh.n_nodes;
    }
    ppc_stats S{};
    for (int d = 0; d < D; ++d) {
        S.n_free += parts[d]->mesh.n_free;
        S.nnz += parts[d]->mesh.nnz;
        S.n_tri += parts[d]->mesh.n_tri;
    }
    DevBuf scal, cargs, cwork;
    PPC_HIP(hipMalloc(&scal.p, sizeof(double) * 3 * D));
    PPC_HIP(hipMalloc(&cargs.p, sizeof(CocgArgs) * D));
    PPC_HIP(hipMalloc(&cwork.p, sizeof(int2) * (size_t)D * H));
    {
        std::vector<CocgArgs> ca(D);
        for (int d = 0; d < D; ++d) ca[d] = make_cocg_args(parts[d], p);
        PPC_HIP(hipMemcpyAsync(cargs.p, ca.data(), sizeof(CocgArgs) * D, hipMemcpyHostToDevice, s));
        PPC_HIP(hipStreamSynchronize(s));
    }
    std::vector<int> counts(8 * (size_t)N);
    std::vector<int> ccount(4 * (size_t)H);
    std::vector<int2> cw;
    hipEvent_t* ev = h->ev;
    PPC_HIP(hipEventRecord(ev[4], s));

    // harmonic solves of the listed designs (excitation: U^0 rows; else correction)
    auto coarse = [&](const std::vector<int>& list, bool excitation) {
        if (list.empty()) return;
        for (int d : list) {
            Workspace& w = parts[d]->ws;
            launch_coarse_pre(parts[d], p, excitation ? nullptr : (p->lin_point == 1 ? w.F : w.U),
                              excitation ? nullptr : w.J, excitation, s);
        }
        const int Hs = solved_harmonics(p, excitation);
        launch_cocg_batch(parts, list, p, Hs, static_cast<CocgArgs*>(cargs.p), static_cast<int2*>(cwork.p), cw, s);
        for (int d : list) {
            Workspace& w = parts[d]->ws;
            if (!excitation && p->b_cap > 0.0) {
                launch_coarse_post(parts[d], p, w.R, false, s);
                launch_safeguarded_update(parts[d], N, p->b_cap, w.R, w.U, w.scal + 8, s);
            } else {
                launch_coarse_post(parts[d], p, w.U, !excitation, s);
            }
        }
        for (int d : list) {
            PPC_HIP(hipMemcpyAsync(ccount.data(), parts[d]->ws.ccount, ccount.size() * sizeof(int),
                                   hipMemcpyDeviceToHost, s));
            PPC_HIP(hipStreamSynchronize(s));
            for (int q = 0; q < Hs; ++q) {
                if (ccount[4 * q] != 0)
                    fail(ccount[4 * q], "design " + std::to_string(d) + ": " +
                                            (ccount[4 * q] == PPC_ERR_BREAKDOWN ? "COCG breakdown" : "non-finite COCG residual"));
                S.cocg_total += ccount[4 * q + 1];
                S.cocg_max = std::max(S.cocg_max, ccount[4 * q + 1]);
            }
            if (!excitation && p->b_cap > 0.0) {
                double theta = 1.0;
                PPC_HIP(hipMemcpy(&theta, parts[d]->ws.scal + 8, sizeof(double), hipMemcpyDeviceToHost));
                if (theta < 1.0) S.damped++;
            }
        }
        S.coarse_solves++;
    };

    // chain counters of design d's last sweep (in counts) into the stats; fails on a
    // chain's status
    auto add_counts = [&](int d) {
        for (int c = 0; c < N; ++c) {
            const int* q = counts.data() + 8 * c;
            if (q[0] != 0)
                fail(q[0], "design " + std::to_string(d) + ", fine chain " + std::to_string(c + 1) +
                               " failed at step " + std::to_string(q[6]));
            S.newton_total += q[1];
            S.lin_total += q[2];
            S.newton_max = std::max(S.newton_max, q[3]);
            S.lin_max = std::max(S.lin_max, q[4]);
            S.lin_capped += q[5];
            S.resid_total += q[7];
        }
        S.steps_total += (int64_t)N * p->m;
    };
    auto take_counts = [&](int d) {
        PPC_HIP(hipMemcpy(counts.data(), parts[d]->ws.fcount, counts.size() * sizeof(int), hipMemcpyDeviceToHost));
        add_counts(d);
    };

    // initial iterate per design (the nested start: the whole batch solved on the coarser
    // fine grid first, which leaves every design's samples in its workspace)
    std::vector<int> coarse_init, fine_init;
    double nested_ms = 0.0;
    if (!U_init_dev && p->init_mode == 4) {
        const ppc_params q = nested_params(p);
        ppc_stats Sq{};
        (void)solve_batch_device(h, bp, &q, nullptr, nullptr, nullptr, nullptr, &Sq, s);
        S.fine_launches += Sq.fine_launches;
        S.fine_ms += Sq.fine_ms;
        S.newton_total += Sq.newton_total;
        S.lin_total += Sq.lin_total;
        S.newton_max = std::max(S.newton_max, Sq.newton_max);
        S.lin_max = std::max(S.lin_max, Sq.lin_max);
        S.lin_capped += Sq.lin_capped;
        S.resid_total += Sq.resid_total;
        S.steps_total += Sq.steps_total;
        S.cocg_total += Sq.cocg_total;
        S.cocg_max = std::max(S.cocg_max, Sq.cocg_max);
        S.coarse_solves += Sq.coarse_solves;
        S.coarse_ms += Sq.coarse_ms;
        S.damped += Sq.damped;
        nested_ms = Sq.total_ms;
        PPC_HIP(hipEventRecord(ev[4], s));   // the nested solve reused the solve's events
    }
    for (int d = 0; d < D; ++d) {
        Workspace& w = parts[d]->ws;
        const long cnt = (long)N * parts[d]->mesh.n_free;
        if (U_init_dev) {
            launch_to_free(parts[d], N, U_init_dev + off[d], w.U, s);
        } else {
            int mode = p->init_mode;
            if (mode == 4) continue;           // the nested solve left U^0 in place
            if (mode == 0) mode = parts[d]->mesh.nonlinear ? 2 : 1;
            if (mode == 2 || mode == 3) fill(w.U, cnt, 0.0, s);
            if (mode == 3) fine_init.push_back(d);
            if (mode == 1) coarse_init.push_back(d);
        }
    }
    coarse(coarse_init, true);

    // adaptive Newton tolerance: each design's sweeps read the squared norms that the
    // previous iteration's jump kernel left in scal (zero before the first sweep)
    if (p->tol_adapt > 0.0) PPC_HIP(hipMemsetAsync(scal.p, 0, sizeof(double) * 3 * D, s));
    FineBatch fb;
    fine_batch_prepare(fb, parts, p, s, static_cast<const double*>(scal.p));
    if (!fine_init.empty()) {
        // one fine sweep from rest for these designs: U^0_n = F_n(0)
        std::vector<char> from_rest(D, 0);
        for (int d : fine_init) from_rest[d] = 1;
        PPC_HIP(hipEventRecord(ev[0], s));
        fine_batch_launch(fb, from_rest, s);
        PPC_HIP(hipEventRecord(ev[1], s));
        PPC_HIP(hipStreamSynchronize(s));
        S.fine_launches++;
        S.fine_ms += elapsed(ev[0], ev[1]);
        for (int d : fine_init) {
            take_counts(d);
            Workspace& w = parts[d]->ws;
            PPC_HIP(hipMemcpyAsync(w.U, w.F, sizeof(double) * (size_t)N * parts[d]->mesh.n_free,
                                   hipMemcpyDeviceToDevice, s));
        }
    }
    // Device work of one iteration, as in the single-design solve: the fine sweep of the
    // active designs with their jump norms and chain counters copied to pinned memory, then
    // the corrections of the designs that go on with their counters.  With params->graph
    // each part is captured for the set of designs it serves (the first time that set
    // occurs after the first iteration) and replayed while the set is unchanged; the
    // work lists are uploaded eagerly when the set changes.
    const bool use_graph = p->graph != 0;
    const int Hs = solved_harmonics(p, false);
    PinnedBuf<double> hs_p(3 * (size_t)D), th_p((size_t)D);
    PinnedBuf<int> cnt_p(8 * (size_t)N * D), cc_p(4 * (size_t)H * D);
    std::vector<char> active(D, 1), fine_set, coarse_set;
    std::vector<int> corr;
    CocgBatchPlan cplan;
    GraphExec g_fine, g_coarse;
    auto fine_ops = [&]() {
        fine_batch_run(fb, s);
        for (int d = 0; d < D; ++d)
            if (active[d]) {
                Workspace& w = parts[d]->ws;
                launch_jumps(parts[d], N, w.U, w.F, w.J, static_cast<double*>(scal.p) + 3 * d, s);
                PPC_HIP(hipMemcpyAsync(cnt_p.p + 8 * (size_t)N * d, w.fcount, 8 * (size_t)N * sizeof(int),
                                       hipMemcpyDeviceToHost, s));
            }
        PPC_HIP(hipMemcpyAsync(hs_p.p, scal.p, sizeof(double) * 3 * D, hipMemcpyDeviceToHost, s));
    };
    // the designs' own kernels before and after the shared COCG launches run side by side
    // on the handle's lanes (each design's work stays on one lane, in order)
    auto coarse_ops = [&]() {
        {
            Lanes lanes(h, s);
            for (size_t i = 0; i < corr.size(); ++i) {
                Workspace& w = parts[corr[i]]->ws;
                launch_coarse_pre(parts[corr[i]], p, p->lin_point == 1 ? w.F : w.U, w.J, false, lanes.lane((int)i));
            }
            lanes.join();
        }
        cocg_batch_run(cplan, static_cast<CocgArgs*>(cargs.p), static_cast<int2*>(cwork.p), s, h);
        Lanes lanes(h, s);
        for (size_t i = 0; i < corr.size(); ++i) {
            const int d = corr[i];
            Workspace& w = parts[d]->ws;
            hipStream_t sd = lanes.lane((int)i);
            if (p->b_cap > 0.0) {
                launch_coarse_post(parts[d], p, w.R, false, sd);
                launch_safeguarded_update(parts[d], N, p->b_cap, w.R, w.U, w.scal + 8, sd);
                PPC_HIP(hipMemcpyAsync(th_p.p + d, w.scal + 8, sizeof(double), hipMemcpyDeviceToHost, sd));
            } else {
                launch_coarse_post(parts[d], p, w.U, true, sd);
            }
            PPC_HIP(hipMemcpyAsync(cc_p.p + 4 * (size_t)H * d, w.ccount, 4 * (size_t)Hs * sizeof(int),
                                   hipMemcpyDeviceToHost, sd));
        }
        lanes.join();
    };
    std::vector<int> iters(D, p->max_iters);
    int status = PPC_OK;
    int k = 0;
    for (k = 0; k <= p->max_iters; ++k) {
        PPC_HIP(hipEventRecord(ev[0], s));
        if (active != fine_set) {
            fine_batch_plan(fb, active, s);
            if (g_fine.exec) (void)hipGraphExecDestroy(g_fine.exec);
            g_fine.exec = nullptr;
            fine_set = active;
        }
        if (use_graph && k > 0) {
            if (!g_fine.exec) capture_graph(g_fine, s, fine_ops);
            PPC_HIP(hipGraphLaunch(g_fine.exec, s));
        } else {
            fine_ops();
        }
        PPC_HIP(hipEventRecord(ev[1], s));
        S.fine_launches++;
        PPC_HIP(hipStreamSynchronize(s));
        S.fine_ms += elapsed(ev[0], ev[1]);
        std::vector<int> next;
        double eps_k = 0.0;       // the largest eps of this iteration's designs
        for (int d = 0; d < D; ++d) {
            if (!active[d]) continue;
            std::copy(cnt_p.p + 8 * (size_t)N * d, cnt_p.p + 8 * (size_t)N * (d + 1), counts.begin());
            add_counts(d);
            const double jj = hs_p.p[3 * d], uu = hs_p.p[3 * d + 1];
            if (!std::isfinite(jj)) fail(PPC_ERR_NONFINITE, "design " + std::to_string(d) + ": non-finite jump norm");
            const double eps = uu > 0.0 ? std::sqrt(jj) / std::sqrt(uu) : (jj == 0.0 ? 0.0 : INFINITY);
            if (resid_out) resid_out[(size_t)d * R1 + k] = eps;
            S.eps = std::max(S.eps, eps);
            eps_k = std::max(eps_k, eps);
            if (eps <= p->tol_ppc) {
                active[d] = 0;
                iters[d] = k;
            } else if (k < p->max_iters) {
                next.push_back(d);
            }
        }
        if (p->progress) p->progress(p->m, k, eps_k, (int)next.size(), p->progress_user);
        if (next.empty()) break;
        PPC_HIP(hipEventRecord(ev[2], s));
        std::vector<char> cset(D, 0);
        for (int d : next) cset[d] = 1;
        if (cset != coarse_set) {
            corr = next;
            cocg_batch_plan(parts, corr, p, Hs, static_cast<int2*>(cwork.p), cplan, s);
            if (g_coarse.exec) (void)hipGraphExecDestroy(g_coarse.exec);
            g_coarse.exec = nullptr;
            coarse_set = cset;
        }
        if (use_graph && k > 0) {
            if (!g_coarse.exec) capture_graph(g_coarse, s, coarse_ops);
            PPC_HIP(hipGraphLaunch(g_coarse.exec, s));
        } else {
            coarse_ops();
        }
        PPC_HIP(hipEventRecord(ev[3], s));
        PPC_HIP(hipStreamSynchronize(s));
        S.coarse_ms += elapsed(ev[2], ev[3]);
        S.coarse_solves++;
        for (int d : corr) {
            const int* c = cc_p.p + 4 * (size_t)H * d;
            for (int q = 0; q < Hs; ++q) {
                if (c[4 * q] != 0)
                    fail(c[4 * q], "design " + std::to_string(d) + ": " +
                                       (c[4 * q] == PPC_ERR_BREAKDOWN ? "COCG breakdown" : "non-finite COCG residual"));
                S.cocg_total += c[4 * q + 1];
                S.cocg_max = std::max(S.cocg_max, c[4 * q + 1]);
            }
            if (p->b_cap > 0.0 && th_p.p[d] < 1.0) S.damped++;
        }
    }
    for (int d = 0; d < D; ++d)
        if (active[d]) status = PPC_NOT_CONVERGED;
    S.iterations = 0;
    for (int d = 0; d < D; ++d) {
        S.iterations = std::max(S.iterations, iters[d]);
        if (iters_out) iters_out[d] = iters[d];
        if (U_out_dev) launch_to_nodal(parts[d], N, parts[d]->ws.U, U_out_dev + off[d], s);
    }
    PPC_HIP(hipEventRecord(ev[5], s));
    PPC_HIP(hipStreamSynchronize(s));
    S.total_ms = elapsed(ev[4], ev[5]) + nested_ms;
    S.status = status;
    if (st) *st = S;
    return status;
}


// ---------------------------------------------------------------------------------------
// adjoint of the periodic steady state
// ---------------------------------------------------------------------------------------
// Classical time stepping on the device: one chain of the fine kernel per period (N m
// steps from u_start), the period's N samples gathered from its trajectory and compared
// with the previous period's.
int time_stepping_device(ppc_handle* h, ppc_problem* pr, const ppc_params* p, const double* u_start_dev,
                         const double* U_prev_dev, double* U_out_dev, int32_t* periods_out, ppc_stats* st,
                         hipStream_t s) {
    PPC_HIP(hipSetDevice(h->device));
    const DeviceMesh& d = pr->mesh;
    const int N = p->N, n = d.n_free;
    ppc_params q = *p;        // one chain over the whole period, same step size
    q.N = 1;
    q.m = p->N * p->m;
    ensure_workspace(pr, &q);
    Workspace& w = pr->ws;
    ppc_stats S{};
    S.n_free = d.n_free;
    S.nnz = d.nnz;
    S.n_tri = d.n_tri;
    DevBuf traj, cur, prev, nrm;
    PPC_HIP(hipMalloc(&traj.p, sizeof(double) * ((size_t)q.m + 1) * n));
    PPC_HIP(hipMalloc(&cur.p, sizeof(double) * (size_t)N * n));
    PPC_HIP(hipMalloc(&prev.p, sizeof(double) * (size_t)N * n));
    PPC_HIP(hipMalloc(&nrm.p, sizeof(double) * 2 * (size_t)N));
    double* Tr = static_cast<double*>(traj.p);
    double* C = static_cast<double*>(cur.p);
    double* P = static_cast<double*>(prev.p);
    hipEvent_t* ev = h->ev;
    PPC_HIP(hipEventRecord(ev[4], s));
    if (u_start_dev) launch_to_free(pr, 1, u_start_dev, w.U, s);
    else fill(w.U, n, 0.0, s);
    bool have_prev = false;
    if (U_prev_dev) {
        launch_to_free(pr, N, U_prev_dev, P, s);
        have_prev = true;
    }
    std::vector<double> hn(2 * (size_t)N);
    int status = PPC_NOT_CONVERGED, period = 0;
    for (period = 1; period <= p->max_iters; ++period) {
        PPC_HIP(hipEventRecord(ev[0], s));
        launch_fine_sweep_traj(pr, &q, w.U, w.F, Tr, s);
        PPC_HIP(hipEventRecord(ev[1], s));
        const SweepCounts c = read_chain_counts(pr, 1, s, nullptr, nullptr);   // synchronises
        S.fine_launches++;
        S.fine_ms += elapsed(ev[0], ev[1]);
        S.newton_total += c.newton;
        S.lin_total += c.lin;
        S.newton_max = std::max(S.newton_max, c.newton_max);
        S.lin_max = std::max(S.lin_max, c.lin_max);
        S.lin_capped += c.capped;
        S.resid_total += c.resid;
        S.steps_total += q.m;
        check_sweep(c);
        launch_gather_samples(n, N, p->m, Tr, C, s);
        PPC_HIP(hipMemcpyAsync(w.U, w.F, sizeof(double) * n, hipMemcpyDeviceToDevice, s));   // next start
        bool done = false;
        if (have_prev) {
            launch_sample_change(n, N, C, P, static_cast<double*>(nrm.p), s);
            PPC_HIP(hipMemcpyAsync(hn.data(), nrm.p, sizeof(double) * hn.size(), hipMemcpyDeviceToHost, s));
            PPC_HIP(hipStreamSynchronize(s));
            double change = 0.0, size = 0.0;
            for (int k = 0; k < N; ++k) {
                change = std::max(change, std::sqrt(hn[2 * k]));
                size = std::max(size, std::sqrt(hn[2 * k + 1]));
            }
            if (!std::isfinite(change)) fail(PPC_ERR_NONFINITE, "non-finite state in time stepping");
            S.eps = size > 0.0 ? change / size : (change == 0.0 ? 0.0 : INFINITY);
            done = change <= p->tol_ppc * size;
        }
        std::swap(C, P);          // P: this period's samples
        have_prev = true;
        if (done) {
            status = PPC_OK;
            break;
        }
    }
    S.iterations = std::min(period, p->max_iters);
    if (U_out_dev) launch_to_nodal(pr, N, P, U_out_dev, s);
    PPC_HIP(hipEventRecord(ev[5], s));
    PPC_HIP(hipStreamSynchronize(s));
    S.total_ms = elapsed(ev[4], ev[5]);
    S.status = status;
    if (periods_out) *periods_out = S.iterations;
    if (st) *st = S;
    return status;
}

int adjoint_device(ppc_handle* h, ppc_problem* pr, const ppc_params* p, const double* U_host, double* loss,
                   double* dsigma, double* dbrauer, int32_t* iters_out, ppc_stats* st, hipStream_t s) {
    PPC_HIP(hipSetDevice(h->device));
    ensure_workspace(pr, p);
    Workspace& w = pr->ws;
    const DeviceMesh& d = pr->mesh;
    const int N = p->N, m = p->m, n = d.n_free, H = N / 2 + 1;
    const int n_mat = pr->laws.n_mat;
    ppc_params p_full = *p;   // the adjoint's corrections solve every harmonic
    p_full.n_harm = 0;
    DevBuf traj, lam_all, Lam, FB, JR, dLR, part, out1, dsig, dke, dkm, Unod;
    PPC_HIP(hipMalloc(&traj.p, sizeof(double) * (size_t)N * (m + 1) * n));
    PPC_HIP(hipMalloc(&lam_all.p, sizeof(double) * (size_t)N * m * n));
    PPC_HIP(hipMalloc(&Lam.p, sizeof(double) * (size_t)N * n));
    PPC_HIP(hipMalloc(&FB.p, sizeof(double) * (size_t)N * n));
    PPC_HIP(hipMalloc(&JR.p, sizeof(double) * (size_t)N * n));
    PPC_HIP(hipMalloc(&dLR.p, sizeof(double) * (size_t)N * n));
    PPC_HIP(hipMalloc(&part.p, sizeof(double) * (size_t)N * m));
    PPC_HIP(hipMalloc(&out1.p, sizeof(double) * 4));
    PPC_HIP(hipMalloc(&dsig.p, sizeof(double) * (size_t)d.n_tri));
    PPC_HIP(hipMalloc(&dke.p, sizeof(double) * 3 * (size_t)d.n_tri));
    PPC_HIP(hipMalloc(&dkm.p, sizeof(double) * 3 * (size_t)n_mat));
    PPC_HIP(hipMalloc(&Unod.p, sizeof(double) * (size_t)N * d.n_nodes));
    double* dtraj = static_cast<double*>(traj.p);
    double* dlam = static_cast<double*>(lam_all.p);
    double* dL = static_cast<double*>(Lam.p);
    double* dFB = static_cast<double*>(FB.p);
    ppc_stats S{};
    S.n_free = d.n_free;
    S.nnz = d.nnz;
    S.n_tri = d.n_tri;
    hipEvent_t* ev = h->ev;
    PPC_HIP(hipEventRecord(ev[4], s));
    PPC_HIP(hipMemcpyAsync(Unod.p, U_host, sizeof(double) * (size_t)N * d.n_nodes, hipMemcpyHostToDevice, s));
    launch_to_free(pr, N, static_cast<double*>(Unod.p), w.U, s);
    // forward replay from the per-subinterval checkpoints U_{n-1}, storing every step
    launch_fine_sweep_traj(pr, p, w.U, w.F, dtraj, s);
    check_sweep(read_chain_counts(pr, N, s, nullptr, nullptr));
    S.fine_launches++;
    launch_loss(pr, p, dtraj, static_cast<double*>(part.p), static_cast<double*>(out1.p), s);
    if (!dsigma && !dbrauer) {
        // the loss alone: no adjoint iteration
        if (loss) PPC_HIP(hipMemcpyAsync(loss, out1.p, sizeof(double), hipMemcpyDeviceToHost, s));
        PPC_HIP(hipEventRecord(ev[5], s));
        PPC_HIP(hipStreamSynchronize(s));
        S.total_ms = elapsed(ev[4], ev[5]);
        S.status = PPC_OK;
        if (iters_out) *iters_out = 0;
        if (st) *st = S;
        return PPC_OK;
    }
    // backward PP-PC on the adjoint: Lambda_c = lambda_{cm+1}
    fill(dL, (long)N * n, 0.0, s);
    AdjArgs b{};
    b.traj = dtraj;
    b.lam_in = dL;
    b.lam_out = dFB;
    b.lam_all = dlam;
    b.tol_lin = 1e-12;
    b.T = p->T;
    int status = PPC_NOT_CONVERGED, k = 0;
    for (k = 0; k <= p->max_iters; ++k) {
        PPC_HIP(hipEventRecord(ev[0], s));
        launch_adjoint_sweep(pr, p, b, s);
        PPC_HIP(hipEventRecord(ev[1], s));
        S.fine_launches++;
        launch_jumps(pr, N, dL, dFB, w.J, w.scal, s);
        PPC_HIP(hipMemcpyAsync(w.host_scal, w.scal, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
        const SweepCounts c = read_chain_counts(pr, N, s, nullptr, nullptr);
        S.fine_ms += elapsed(ev[0], ev[1]);
        S.lin_total += c.lin;
        S.lin_max = std::max(S.lin_max, c.lin_max);
        S.lin_capped += c.capped;
        const double jj = w.host_scal[0], uu = w.host_scal[1];
        if (!std::isfinite(jj)) fail(PPC_ERR_NONFINITE, "non-finite adjoint jump norm");
        const double eps = uu > 0.0 ? std::sqrt(jj) / std::sqrt(uu) : (jj == 0.0 ? 0.0 : INFINITY);
        S.eps = eps;
        if (eps <= p->tol_ppc) {
            status = PPC_OK;
            break;
        }
        if (k == p->max_iters) break;
        // coarse correction of the time-reversed jumps (the backward cyclic system read
        // in reversed subinterval order is the forward one), K frozen at the samples U
        PPC_HIP(hipEventRecord(ev[2], s));
        launch_reverse_rows(N, n, w.J, static_cast<double*>(JR.p), s);
        launch_coarse(pr, &p_full, w.U, static_cast<double*>(JR.p), static_cast<double*>(dLR.p), false, false, s);
        launch_add_reversed(N, n, static_cast<double*>(dLR.p), dL, s);
        PPC_HIP(hipEventRecord(ev[3], s));
        read_cocg(pr, H, s, nullptr, &S.cocg_total, &S.cocg_max);
        S.coarse_ms += elapsed(ev[2], ev[3]);
        S.coarse_solves++;
    }
    S.iterations = std::min(k, p->max_iters);
    launch_gradients(pr, p, dtraj, dlam, static_cast<double*>(dsig.p), static_cast<double*>(dke.p),
                     static_cast<double*>(dkm.p), n_mat, s);
    if (loss) PPC_HIP(hipMemcpyAsync(loss, out1.p, sizeof(double), hipMemcpyDeviceToHost, s));
    if (dsigma) PPC_HIP(hipMemcpyAsync(dsigma, dsig.p, sizeof(double) * d.n_tri, hipMemcpyDeviceToHost, s));
    if (dbrauer) PPC_HIP(hipMemcpyAsync(dbrauer, dkm.p, sizeof(double) * 3 * n_mat, hipMemcpyDeviceToHost, s));
    PPC_HIP(hipEventRecord(ev[5], s));
    PPC_HIP(hipStreamSynchronize(s));
    S.total_ms = elapsed(ev[4], ev[5]);
    S.status = status;
    if (iters_out) *iters_out = S.iterations;
    if (st) *st = S;
    return status;
}

}  // namespace
}  // namespace ppc

using namespace ppc;

extern "C" {

int ppc_version(void) { return PPC_ABI_VERSION; }

int ppc_params_default(ppc_params* p) {
    if (!p) return PPC_ERR_ARG;
    std::memset(p, 0, sizeof(*p));
    p->T = 0.02;
    p->N = 10;
    p->m = 20;
    p->shift_mode = 0;
    p->lin_mode = 0;
    p->init_mode = 0;
    p->precision = 0;
    p->tol_ppc = 1e-12;
    p->max_iters = 60;
    p->tol_newton = 1e-13;
    p->max_newton = 50;
    p->tol_lin = 1e-8;
    p->max_lin = 20000;
    p->tol_cocg = 1e-10;
    p->max_cocg = 20000;
    p->block = 0;
    p->no_predictor = 0;
    p->lin_point = 1;
    p->coarse_precision = -1;
    p->graph = 1;
    p->method = 0;
    p->b_cap = 0.0;
    p->coarse_mode = 0;
    p->lin_start = 0;
    p->lin_forcing = 0;
    p->progress = nullptr;
    p->progress_user = nullptr;
    p->tol_adapt = 0.0;
    return PPC_OK;
}

const char* ppc_last_error(const ppc_handle* h) {
    return h ? h->last_error.c_str() : g_thread_error.c_str();
}

int ppc_validate(const ppc_mesh* mesh, const ppc_material* mat, const ppc_excitation* exc, char* msg,
                 int32_t msg_len) {
    std::string m;
    const int rc = validate_problem(mesh, mat, exc, m);
    set_msg(msg, msg_len, rc == PPC_OK ? std::string("ok") : m);
    if (rc != PPC_OK) g_thread_error = m;
    return rc;
}

int ppc_validate_params(const ppc_params* p, char* msg, int32_t msg_len) {
    std::string m;
    const int rc = validate_params(p, m);
    set_msg(msg, msg_len, rc == PPC_OK ? std::string("ok") : m);
    if (rc != PPC_OK) g_thread_error = m;
    return rc;
}

int ppc_create(int32_t device, ppc_handle** out) {
    return guarded(nullptr, [&]() -> int {
        if (!out) fail(PPC_ERR_ARG, "null output pointer");
        *out = nullptr;
        if (device < 0) fail(PPC_ERR_ARG, "negative device index");
        int count = 0;
        const hipError_t e = hipGetDeviceCount(&count);
        if (e != hipSuccess || count == 0) fail(PPC_ERR_DEVICE, "no usable GPU (hipGetDeviceCount)");
        if (device >= count) fail(PPC_ERR_ARG, "device index out of range");
        PPC_HIP(hipSetDevice(device));
        (void)scratch_address(device);
        auto* h = new ppc_handle();
        h->device = device;
        try {
            PPC_HIP(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
            for (auto& ev : h->ev) PPC_HIP(hipEventCreate(&ev));
            for (auto& st : h->side) PPC_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
            PPC_HIP(hipEventCreateWithFlags(&h->fork, hipEventDisableTiming));
            for (auto& ev : h->join) PPC_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        } catch (...) {
            ppc_destroy(h);
            throw;
        }
        *out = h;
        return PPC_OK;
    });
}

int ppc_destroy(ppc_handle* h) {
    if (!h) return PPC_OK;
    if (h->n_problems != 0) {
        h->last_error = "destroy the handle's problems first";
        return PPC_ERR_ARG;
    }
    (void)hipSetDevice(h->device);
    for (auto& ev : h->ev)
        if (ev) (void)hipEventDestroy(ev);
    for (auto& ev : h->join)
        if (ev) (void)hipEventDestroy(ev);
    if (h->fork) (void)hipEventDestroy(h->fork);
    for (auto& st : h->side)
        if (st) (void)hipStreamDestroy(st);
    if (h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
    return PPC_OK;
}

int ppc_problem_create(ppc_handle* h, const ppc_mesh* mesh, const ppc_material* mat,
                       const ppc_excitation* exc, ppc_problem** out) {
    return guarded(h, [&]() -> int {
        if (!out) fail(PPC_ERR_ARG, "null output pointer");
        *out = nullptr;
        if (!h) fail(PPC_ERR_ARG, "null handle");
        std::string msg;
        const int rc = validate_problem(mesh, mat, exc, msg);
        if (rc != PPC_OK) fail(rc, msg);
        PPC_HIP(hipSetDevice(h->device));
        auto* pr = new ppc_problem();
        pr->h = h;
        try {
            build_problem(pr, mesh, mat, exc, h->stream);
        } catch (...) {
            mesh_free(pr->mesh);
            if (pr->lawtab) (void)hipFree(pr->lawtab);
            if (pr->wavtab) (void)hipFree(pr->wavtab);
            delete pr;
            throw;
        }
        h->n_problems++;
        *out = pr;
        return PPC_OK;
    });
}

int ppc_problem_create_batch(ppc_handle* h, int32_t n_designs, const ppc_mesh* meshes,
                             const ppc_material* mats, const ppc_excitation* excs, ppc_problem** out) {
    return guarded(h, [&]() -> int {
        if (!out) fail(PPC_ERR_ARG, "null output pointer");
        *out = nullptr;
        if (!h) fail(PPC_ERR_ARG, "null handle");
        if (n_designs < 1 || !meshes || !mats || !excs) fail(PPC_ERR_ARG, "need n_designs >= 1 and non-null arrays");
        for (int d = 0; d < n_designs; ++d) {
            std::string msg;
            const int rc = validate_problem(&meshes[d], &mats[d], &excs[d], msg);
            if (rc != PPC_OK) fail(rc, "design " + std::to_string(d) + ": " + msg);
        }
        PPC_HIP(hipSetDevice(h->device));
        auto* bp = new ppc_problem();
        bp->h = h;
        bp->batch = true;
        try {
            for (int d = 0; d < n_designs; ++d) {
                auto* q = new ppc_problem();
                q->h = h;
                bp->parts.push_back(q);
                build_problem(q, &meshes[d], &mats[d], &excs[d], h->stream);
            }
        } catch (...) {
            for (auto* q : bp->parts) {
                q->h = nullptr;
                ppc_problem_destroy(q);
            }
            bp->parts.clear();
            delete bp;
            throw;
        }
        h->n_problems++;
        *out = bp;
        return PPC_OK;
    });
}

int ppc_batch_info(const ppc_problem* pr, int32_t* n_designs, int32_t* n_nodes, int32_t* n_free) {
    if (!pr) return PPC_ERR_ARG;
    if (!pr->batch) {
        if (n_designs) *n_designs = 1;
        if (n_nodes) n_nodes[0] = pr->mesh.n_nodes;
        if (n_free) n_free[0] = pr->mesh.n_free;
        return PPC_OK;
    }
    if (n_designs) *n_designs = (int32_t)pr->parts.size();
    for (size_t d = 0; d < pr->parts.size(); ++d) {
        if (n_nodes) n_nodes[d] = pr->parts[d]->mesh.n_nodes;
        if (n_free) n_free[d] = pr->parts[d]->mesh.n_free;
    }
    return PPC_OK;
}

int ppc_problem_destroy(ppc_problem* pr) {
    if (!pr) return PPC_OK;
    for (auto* q : pr->parts) {
        q->h = nullptr;
        ppc_problem_destroy(q);
    }
    pr->parts.clear();
    if (pr->h) (void)hipSetDevice(pr->h->device);
    workspace_free(pr->ws);
    mesh_free(pr->mesh);
    if (pr->lawtab) (void)hipFree(pr->lawtab);
    if (pr->wavtab) (void)hipFree(pr->wavtab);
    if (pr->h) pr->h->n_problems--;
    delete pr;
    return PPC_OK;
}

int ppc_fine_counts(const ppc_problem* pr, int32_t n_chains, int32_t* counts) {
    if (!pr || !counts || pr->batch || !pr->h) return PPC_ERR_ARG;
    if (pr->ws.N != n_chains || !pr->ws.fcount) return PPC_ERR_ARG;
    if (hipSetDevice(pr->h->device) != hipSuccess) return PPC_ERR_DEVICE;
    if (hipMemcpy(counts, pr->ws.fcount, sizeof(int32_t) * 8 * (size_t)n_chains, hipMemcpyDeviceToHost) !=
        hipSuccess)
        return PPC_ERR_DEVICE;
    return PPC_OK;
}
int ppc_problem_info(const ppc_problem* pr, int32_t* n_free, int32_t* nnz, int32_t* n_tri,
                     int32_t* n_nodes) {
    if (!pr) return PPC_ERR_ARG;
    if (pr->batch) {
        int32_t a = 0, b = 0, c = 0, e = 0;
        for (auto* q : pr->parts) {
            a += q->mesh.n_free;
            b += q->mesh.nnz;
            c += q->mesh.n_tri;
            e += q->mesh.n_nodes;
        }
        if (n_free) *n_free = a;
        if (nnz) *nnz = b;
        if (n_tri) *n_tri = c;
        if (n_nodes) *n_nodes = e;
        return PPC_OK;
    }
    if (n_free) *n_free = pr->mesh.n_free;
    if (nnz) *nnz = pr->mesh.nnz;
    if (n_tri) *n_tri = pr->mesh.n_tri;
    if (n_nodes) *n_nodes = pr->mesh.n_nodes;
    return PPC_OK;
}

int ppc_solve_device(ppc_handle* h, ppc_problem* pr, const ppc_params* p, const double* U_init_dev,
                     double* U_out_dev, double* resid_out, int32_t* iters_out, ppc_stats* stats,
                     void* stream) {
    return guarded(h, [&]() -> int {
        check_handle_problem(h, pr);
        check_params(p);
        if (!U_out_dev) fail(PPC_ERR_ARG, "null U_out");
        if (pr->batch)
            return solve_batch_device(h, pr, p, U_init_dev, U_out_dev, resid_out, iters_out, stats,
                                      pick_stream(h, stream));
        return solve_device(h, pr, p, U_init_dev, U_out_dev, resid_out, iters_out, stats,
                            pick_stream(h, stream));
    });
}

int ppc_solve(ppc_handle* h, ppc_problem* pr, const ppc_params* p, const double* U_init,
              double* U_out, double* resid_out, int32_t* iters_out, ppc_stats* stats) {
    return guarded(h, [&]() -> int {
        check_handle_problem(h, pr);
        check_params(p);
        if (!U_out) fail(PPC_ERR_ARG, "null U_out");
        PPC_HIP(hipSetDevice(h->device));
        size_t nodes = pr->mesh.n_nodes;
        if (pr->batch) {
            nodes = 0;
            for (auto* q : pr->parts) nodes += q->mesh.n_nodes;
        }
        const size_t cnt = (size_t)p->N * nodes;
        double* du = dalloc<double>(cnt);
        double* di = nullptr;
        int rc = PPC_OK;
        try {
            if (U_init) {
                di = dalloc<double>(cnt);
                PPC_HIP(hipMemcpyAsync(di, U_init, cnt * sizeof(double), hipMemcpyHostToDevice, h->stream));
            }
            rc = pr->batch ? solve_batch_device(h, pr, p, di, du, resid_out, iters_out, stats, h->stream)
                           : solve_device(h, pr, p, di, du, resid_out, iters_out, stats, h->stream);
            PPC_HIP(hipMemcpyAsync(U_out, du, cnt * sizeof(double), hipMemcpyDeviceToHost, h->stream));
            PPC_HIP(hipStreamSynchronize(h->stream));
        } catch (...) {
            (void)hipFree(du);
            if (di) (void)hipFree(di);
            throw;
        }
        (void)hipFree(du);
        if (di) (void)hipFree(di);
        return rc;
    });
}

int ppc_adjoint(ppc_handle* h, ppc_problem* pr, const ppc_params* p, const double* U_periodic,
                double* loss, double* dsigma, double* dbrauer, int32_t* iters_out, ppc_stats* stats) {
    return guarded(h, [&]() -> int {
        check_handle_problem(h, pr);
        check_params(p);
        if (!U_periodic) fail(PPC_ERR_ARG, "null U_periodic");
        if (pr->batch) fail(PPC_ERR_ARG, "the adjoint takes a single design");
        return adjoint_device(h, pr, p, U_periodic, loss, dsigma, dbrauer, iters_out, stats, h->stream);
    });
}

int ppc_fine_sweep_device(ppc_handle* h, ppc_problem* pr, const ppc_params* p, const double* U_in_dev,
                          double* F_out_dev, int32_t* newton_out, int32_t* lin_out, void* stream) {
    return guarded(h, [&]() -> int {
        check_handle_problem(h, pr);
        check_params(p);
        if (!U_in_dev || !F_out_dev) fail(PPC_ERR_ARG, "null U_in or F_out");
        PPC_HIP(hipSetDevice(h->device));
        hipStream_t s = pick_stream(h, stream);
        if (pr->batch) {
            // every design's chains in one batched launch per kernel shape; U / F in the
            // layout of the batched solve (design d's N x n_nodes_d rows after design d-1's)
            auto& parts = pr->parts;
            const int D = (int)parts.size(), N = p->N;
            std::vector<size_t> off(D + 1, 0);
            for (int d = 0; d < D; ++d) {
                ensure_workspace(parts[d], p);
                off[d + 1] = off[d] + (size_t)N * parts[d]->mesh.n_nodes;
                launch_to_free(parts[d], N, U_in_dev + off[d], parts[d]->ws.U, s);
            }
            FineBatch fb;
            fine_batch_prepare(fb, parts, p, s);
            fine_batch_launch(fb, std::vector<char>(D, 1), s);
            PPC_HIP(hipStreamSynchronize(s));
            for (int d = 0; d < D; ++d) {
                std::vector<int32_t> nw(N), ln(N);
                const SweepCounts c = read_chain_counts(parts[d], N, s, nw.data(), ln.data());
                if (c.status != 0)
                    fail(c.status, "design " + std::to_string(d) + ", fine chain " + std::to_string(c.fail_chain + 1) +
                                       " failed at step " + std::to_string(c.fail_step));
                for (int k = 0; k < N; ++k) {
                    if (newton_out) newton_out[(size_t)d * N + k] = nw[k];
                    if (lin_out) lin_out[(size_t)d * N + k] = ln[k];
                }
                launch_to_nodal(parts[d], N, parts[d]->ws.F, F_out_dev + off[d], s);
            }
            PPC_HIP(hipStreamSynchronize(s));
            return PPC_OK;
        }
        ensure_workspace(pr, p);
        launch_to_free(pr, p->N, U_in_dev, pr->ws.U, s);
        launch_fine_sweep(pr, p, pr->ws.U, pr->ws.F, s);
        const SweepCounts c = read_chain_counts(pr, p->N, s, newton_out, lin_out);
        check_sweep(c);
        launch_to_nodal(pr, p->N, pr->ws.F, F_out_dev, s);
        PPC_HIP(hipStreamSynchronize(s));
        return PPC_OK;
    });
}

int ppc_fine_sweep_noalloc(ppc_handle* h, ppc_problem* pr, const ppc_params* p, const double* U_in_dev,
                           double* F_out_dev, int32_t* newton_out, int32_t* lin_out, void* stream) {
    return guarded(h, [&]() -> int {
        check_handle_problem(h, pr);
        check_params(p);
        if (!U_in_dev || !F_out_dev) fail(PPC_ERR_ARG, "null U_in or F_out");
        if (pr->batch) fail(PPC_ERR_ARG, "single-design entry point called with a batch problem");
        if (p->N > kNoAllocMaxChains)
            fail(PPC_ERR_ARG, "N = " + std::to_string(p->N) + " exceeds the " + std::to_string(kNoAllocMaxChains) +
                                  " chains of the allocation-free fine sweep");
        const size_t L = (size_t)p->N * (size_t)pr->mesh.n_free;
        const size_t vecs = 2 * ((L * sizeof(double) + 255) / 256 * 256);     // U and F, free rows
        const size_t need = vecs + fine_scratch_layout(pr, p, nullptr, nullptr);
        if (need > kScratchBytes)
            fail(PPC_ERR_ARG, "the allocation-free fine sweep needs " + std::to_string(need) + " bytes of its " +
                                  std::to_string(kScratchBytes) + "-byte static scratch (N = " + std::to_string(p->N) +
                                  ", " + std::to_string(pr->mesh.n_free) + " free nodes)");
        PPC_HIP(hipSetDevice(h->device));
        hipStream_t s = pick_stream(h, stream);
        unsigned char* base = scratch_address(h->device);
        double* Uf = reinterpret_cast<double*>(base);
        double* Ff = reinterpret_cast<double*>(base + vecs / 2);
        FineScratch sc;
        (void)fine_scratch_layout(pr, p, base + vecs, &sc);
        launch_to_free(pr, p->N, U_in_dev, Uf, s);
        launch_fine_sweep_in(pr, p, Uf, Ff, sc, s);
        int host_count[8 * kNoAllocMaxChains];
        PPC_HIP(hipMemcpyAsync(host_count, sc.count, 8 * (size_t)p->N * sizeof(int), hipMemcpyDeviceToHost, s));
        PPC_HIP(hipStreamSynchronize(s));
        check_sweep(parse_chain_counts(host_count, p->N, newton_out, lin_out));
        launch_to_nodal(pr, p->N, Ff, F_out_dev, s);
        PPC_HIP(hipStreamSynchronize(s));
        return PPC_OK;
    });
}

int ppc_time_stepping_device(ppc_handle* h, ppc_problem* pr, const ppc_params* p, const double* u_start_dev,
                             const double* U_prev_dev, double* U_out_dev, int32_t* periods_out, ppc_stats* stats,
                             void* stream) {
    return guarded(h, [&]() -> int {
        check_handle_problem(h, pr);
        check_params(p);
        if (!U_out_dev) fail(PPC_ERR_ARG, "null U_out");
        if (pr->batch) fail(PPC_ERR_ARG, "single-design entry point called with a batch problem");
        if ((long)p->N * p->m > 1000000) fail(PPC_ERR_ARG, "N m above 1e6 steps per period");
        return time_stepping_device(h, pr, p, u_start_dev, U_prev_dev, U_out_dev, periods_out, stats,
                                    pick_stream(h, stream));
    });
}

int ppc_autotune(ppc_handle* h, ppc_problem* pr, const ppc_params* p, int32_t* block_out, double* ms_out) {
    return guarded(h, [&]() -> int {
        check_handle_problem(h, pr);
        check_params(p);
        if (p->fine_block != 0) fail(PPC_ERR_ARG, "autotune with fine_block forced");
        PPC_HIP(hipSetDevice(h->device));
        hipStream_t s = h->stream;
        const int slot = p->precision != 0 ? 1 : 0;
        if (!pr->batch) {
            double ms[3];
            const int b = autotune_fine(pr, p, ms, h->ev[6], h->ev[7], s);
            pr->tuned_block[slot] = b;
            if (block_out) block_out[0] = b;
            if (ms_out) std::copy(ms, ms + 3, ms_out);
            return PPC_OK;
        }
        // The batched sweep is what runs, so it is what is timed: policy b puts every design
        // at b threads, or at the next larger size its rows fit (designs of one size class
        // thereby share a size).  A design timed alone owns its CUs, which the batch's
        // workgroups share, so single-design timings would not rank sizes for the batch.
        const int D = (int)pr->parts.size();
        for (auto* q : pr->parts) ensure_workspace(q, p);
        auto policy = [&](int b) {
            std::vector<int> out(D, 0);
            for (int d = 0; d < D; ++d)
                for (int rb : kRowBlocks)
                    if (rb >= b && rows_shape(pr->parts[d], p, rb).R > 0) {
                        out[d] = rb;
                        break;
                    }
            return out;
        };
        const std::vector<char> active(D, 1);
        std::vector<std::vector<int>> assign;
        double ms[3];
        int best = -1;
        for (int i = 0; i < 3; ++i) {
            assign.push_back(policy(kRowBlocks[i]));
            ms[i] = NAN;
            int same = -1;
            for (int j = 0; j < i; ++j)
                if (assign[j] == assign[i]) same = j;
            if (same >= 0) {
                ms[i] = ms[same];
                continue;
            }
            for (int d = 0; d < D; ++d) pr->parts[d]->tuned_block[slot] = assign[i][d];
            FineBatch fb;
            fine_batch_prepare(fb, pr->parts, p, s);
            double t = INFINITY;
            for (int rep = 0; rep < 3; ++rep) {
                for (auto* q : pr->parts) fill(q->ws.U, (long)p->N * q->mesh.n_free, 0.0, s);
                PPC_HIP(hipEventRecord(h->ev[6], s));
                fine_batch_launch(fb, active, s);
                PPC_HIP(hipEventRecord(h->ev[7], s));
                PPC_HIP(hipEventSynchronize(h->ev[7]));
                if (rep > 0) t = std::min(t, (double)elapsed(h->ev[6], h->ev[7]));
            }
            ms[i] = t;
            if (best < 0 || t < ms[best]) best = i;
        }
        for (int d = 0; d < D; ++d) {
            pr->parts[d]->tuned_block[slot] = assign[best][d];
            if (block_out) block_out[d] = assign[best][d];
            if (ms_out) std::copy(ms, ms + 3, ms_out + 3 * (size_t)d);
        }
        return PPC_OK;
    });
}

int ppc_coarse_correction_device(ppc_handle* h, ppc_problem* pr, const ppc_params* p, const double* U_dev,
                                 const double* J_dev, double* dU_dev, int32_t* cocg_out, void* stream) {
    return guarded(h, [&]() -> int {
        check_handle_problem(h, pr);
        check_params(p);
        if (!U_dev || !J_dev || !dU_dev) fail(PPC_ERR_ARG, "null U, J or dU");
        if (pr->batch) fail(PPC_ERR_ARG, "single-design entry point called with a batch problem");
        PPC_HIP(hipSetDevice(h->device));
        hipStream_t s = pick_stream(h, stream);
        ensure_workspace(pr, p);
        launch_to_free(pr, p->N, U_dev, pr->ws.U, s);
        launch_to_free(pr, p->N, J_dev, pr->ws.J, s);
        if (p->coarse_mode == 1) {
            // F = U + J, then the nonlinear correction (U^{k+1} - U^k) into R
            Workspace& w = pr->ws;
            const long L = (long)p->N * pr->mesh.n_free;
            PPC_HIP(hipMemcpyAsync(w.F, w.U, sizeof(double) * L, hipMemcpyDeviceToDevice, s));
            launch_vec_add(L, w.J, w.F, s);
            NlcCounts nc;
            launch_nonlinear_correction(pr, p, w.U, w.F, w.R, false, nc, cocg_out, s);
            launch_to_nodal(pr, p->N, w.R, dU_dev, s);
            PPC_HIP(hipStreamSynchronize(s));
            return PPC_OK;
        }
        launch_coarse(pr, p, pr->ws.U, pr->ws.J, pr->ws.F, false, false, s);
        const int Hs = solved_harmonics(p, false);
        read_cocg(pr, Hs, s, cocg_out, nullptr, nullptr);
        if (cocg_out)
            for (int q = Hs; q < p->N / 2 + 1; ++q) cocg_out[q] = 0;
        launch_to_nodal(pr, p->N, pr->ws.F, dU_dev, s);
        PPC_HIP(hipStreamSynchronize(s));
        return PPC_OK;
    });
}

}  // extern "C"

// Nonlinear periodic coarse problem: the correction of eq. (4) with the coarse propagator
// G of eq. (8) taken on the nonlinear problem, instead of the frozen linearisation.
//
// Eq. (4) asks for U^{k+1}_n = G(U^{k+1}_{n-1}) + b_n cyclically, b_n = F_n(U^k_{n-1}) -
// G(U^k_{n-1}).  With W_n = U^{k+1}_n - b_n = G(U^{k+1}_{n-1}) every row is one implicit-Euler
// step of size dT = T/N:
//     Phi_n(W) = C (W_n - U_{n-1}) + K(W_n) W_n - i(T_n) F = 0,   U = W + b,  C = M/dT,
// a block-cyclic nonlinear system whose Jacobian has C + dK(W_n)W_n/dW_n on the diagonal and
// -C below it (row 0 couples to row N-1).  Newton's method solves it from W = G(U^k), where
// Phi_n = -C J_{n-1}.  Each Newton step solves the Jacobian system by flexible GMRES,
// preconditioned by the frozen block-cyclic solve (the same Kbar, DFT and per-harmonic COCG as
// the frozen correction): when the Jacobian blocks stay close to C + Kbar the preconditioned
// operator is close to the identity.
//
// Layout: every vector is [N][n_free] in row order n = 0..N-1 (row 0 is the step that ends
// at T_N).  One workgroup per row evaluates the step residual and assembles that row's
// Jacobian with the fine sweep's device functions (base values M/dT plus the linear
// elements, then the Brauer elements).  The Krylov vectors are dense [N][n_free] arrays; the
// Gram-Schmidt coefficients and norms return to the host once per Krylov step.
#include "fine_chain.hpp"

namespace ppc {
namespace {

constexpr int kNlcBlock = 512;
constexpr int kDotBlocks = 256;
constexpr int kDotThreads = 256;
// vectors of nlc_vec
enum { NV_G = 0, NV_B = 1, NV_W = 2, NV_WT = 3, NV_U = 4, NV_PHI = 5, NV_D = 6 };

// Row r = (c + 1) mod N of chain c: Phi_r at W_r with U_{r-1} = Uc[c] and the current at
// T_{c+1}; the row's Jacobian values (jac + r vals_pad); part[c], part[N + c] = ||Phi_r||^2,
// ||C U_{r-1}||^2.
__global__ __launch_bounds__(kNlcBlock) void k_nlc_residual(FineArgs a, const double* __restrict__ W,
                                                            const double* __restrict__ Uc,
                                                            double* __restrict__ Phi, double* __restrict__ jac,
                                                            double* __restrict__ part) {
    __shared__ double sh[64];
    const int c = blockIdx.x;
    const int N = a.N, n = a.n;
    const int r = (c + 1) % N;
    const long NP = a.n_pad;
    const double dT = a.T / N;
    const double* ut = W + (long)r * n;
    const double* up = Uc + (long)c * n;
    double* cp = a.vec + ((long)c * kFineVec + V_CP) * NP;
    double* el = a.elem + (long)c * 8 * a.nl_pad;
    double* jv = jac + (long)r * a.vals_pad;
    double v[2];
    v[1] = mass_prev(a, up, 1.0 / dT, cp);
    nl_element_pass(a, ut, el);
    init_jac<double>(a, jv);
    __syncthreads();
    const double cur = current((double)(c + 1) * dT, a.f0, a.n_h, a.wavtab);
    v[0] = resid_rows(a, ut, cp, el, cur, Phi + (long)r * n);
    assemble_nl<double>(a, el, jv);
    int ph = 0;
    block_sum<double, 2>(v, sh, ph);
    if (threadIdx.x == 0) {
        part[c] = v[0];
        part[N + c] = v[1];
    }
}

__device__ inline double mass_row(const FineArgs& a, const double* __restrict__ x, int i) {
    double acc = 0.0;
    for (int k = a.rowptr[i]; k < a.rowptr[i + 1]; ++k) acc += a.mval[k] * x[a.colidx[k]];
    return acc;
}

// Y_r = Jac_r X_r - C X_{r-1} (grid.y = r): ELL rows one thread each; the long (tail) rows,
// one thread each, in the first block of every row.
__global__ void k_nlc_jv(FineArgs a, const double* __restrict__ jac, const double* __restrict__ X,
                         double* __restrict__ Y, double inv_dT) {
    const int r = blockIdx.y, N = a.N, n = a.n;
    const int rp = (r + N - 1) % N;
    const double* x = X + (long)r * n;
    const double* xp = X + (long)rp * n;
    const double* jv = jac + (long)r * a.vals_pad;
    double* y = Y + (long)r * n;
    const long NP = a.ell_pad;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && a.ecol[i] >= 0) {
        double acc = 0.0;
        for (int w = 0; w < a.W; ++w) acc += jv[w * NP + i] * x[a.ecol[w * NP + i]];
        y[i] = acc - inv_dT * mass_row(a, xp, i);
    }
    if (blockIdx.x == 0) {
        const long base = (long)a.W * NP;
        for (int t = threadIdx.x; t < a.ntail; t += blockDim.x) {
            const int row = a.tail_row[t];
            double acc = 0.0;
            for (int j = a.tail_ptr[t]; j < a.tail_ptr[t + 1]; ++j) acc += jv[base + j] * x[a.tail_col[j]];
            y[row] = acc - inv_dT * mass_row(a, xp, row);
        }
    }
}

// part[j * gridDim.x + b] = block b's share of V_j . w for j = blockIdx.y
__global__ __launch_bounds__(kDotThreads) void k_nlc_dots(long L, const double* __restrict__ V, long ld,
                                                          const double* __restrict__ w, double* __restrict__ part) {
    __shared__ double sh[64];
    const double* v = V + (long)blockIdx.y * ld;
    double acc = 0.0;
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < L; k += (long)gridDim.x * blockDim.x)
        acc += v[k] * w[k];
    double t[1] = {acc};
    int ph = 0;
    block_sum<double, 1>(t, sh, ph);
    if (threadIdx.x == 0) part[(long)blockIdx.y * gridDim.x + blockIdx.x] = t[0];
}

// out[j] = sum over b < nb of part[j * nb + b], j < nv (fixed order)
__global__ void k_nlc_sum(int nb, int nv, const double* __restrict__ part, double* __restrict__ out) {
    for (int j = threadIdx.x; j < nv; j += blockDim.x) {
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += part[(long)j * nb + b];
        out[j] = s;
    }
}

// w -= sum over j < nv of h[j] V_j
__global__ void k_nlc_subtract(long L, int nv, const double* __restrict__ V, long ld,
                               const double* __restrict__ h, double* __restrict__ w) {
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < L; k += (long)gridDim.x * blockDim.x) {
        double acc = w[k];
        for (int j = 0; j < nv; ++j) acc -= h[j] * V[(long)j * ld + k];
        w[k] = acc;
    }
}

// out = alpha x + beta y (y may be null: out = alpha x); out may be x or y
__global__ void k_nlc_axpby(long L, double alpha, const double* x, double beta, const double* y, double* out) {
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < L; k += (long)gridDim.x * blockDim.x)
        out[k] = y ? alpha * x[k] + beta * y[k] : alpha * x[k];
}

// out = W + b (accumulate) or W + b - U
__global__ void k_nlc_finish(long L, const double* __restrict__ W, const double* __restrict__ b,
                             const double* __restrict__ U, double* __restrict__ out, int accumulate) {
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < L; k += (long)gridDim.x * blockDim.x)
        out[k] = accumulate ? W[k] + b[k] : (W[k] + b[k]) - U[k];
}

// One implicit-Euler step of size dT = T/N from every sample, G[(c + 1) mod N] = G(U[c]) (the
// coarse propagator of eq. (8) on the full K(u)): the fine sweep with m = 1 and no predictor.
// For its duration the workspace's base Jacobian is the coarse one (nlc_jb, built for dT when
// needed), so the fine sweep's own base Jacobian stays as it is.
void coarse_step_sweep(ppc_problem* pr, const ppc_params* p, const double* U, double* G, hipStream_t s) {
    struct Swap {
        Workspace& w;
        explicit Swap(Workspace& w_) : w(w_) { flip(); }
        ~Swap() { flip(); }
        void flip() {
            std::swap(w.jbase, w.nlc_jb);
            std::swap(w.jbase_dt, w.nlc_jb_dt);
        }
    } swap(pr->ws);
    ppc_params q = *p;
    q.m = 1;
    q.no_predictor = 1;
    launch_fine_sweep(pr, &q, U, G, s);
}

dim3 vec_grid(long L) { return dim3((unsigned)std::max(1L, std::min((L + 255) / 256, 4096L))); }

void ensure_nlc(ppc_problem* pr, const ppc_params* p) {
    Workspace& w = pr->ws;
    if (w.nlc_host) return;                 // allocated last: the set is complete
    for (double** ptr : {&w.nlc_jb, &w.nlc_jac, &w.nlc_vec, &w.nlc_kry, &w.nlc_part, &w.nlc_h})
        if (*ptr) {                         // a set left partial by an allocation failure
            (void)hipFree(*ptr);
            *ptr = nullptr;
        }
    w.nlc_jb_dt = 0.0;
    const size_t L = (size_t)p->N * pr->mesh.n_free;
    auto alloc = [](double** ptr, size_t count) {
        if (hipMalloc(reinterpret_cast<void**>(ptr), std::max<size_t>(count, 1) * sizeof(double)) != hipSuccess)
            fail(PPC_ERR_OOM, "hipMalloc of " + std::to_string(count * sizeof(double)) +
                                  " bytes for the nonlinear coarse problem failed");
    };
    alloc(&w.nlc_jb, w.vals_pad);
    alloc(&w.nlc_jac, (size_t)p->N * w.vals_pad);
    alloc(&w.nlc_vec, kNlcVec * L);
    alloc(&w.nlc_kry, (2 * kNlcKrylov + 1) * L);
    alloc(&w.nlc_part, (size_t)std::max(2 * p->N, (kNlcKrylov + 1) * kDotBlocks));
    alloc(&w.nlc_h, 4 * (kNlcKrylov + 1));
    void* hp = nullptr;
    PPC_HIP(hipHostMalloc(&hp, 4 * (kNlcKrylov + 1) * sizeof(double), hipHostMallocDefault));
    w.nlc_host = static_cast<double*>(hp);
}

}  // namespace

void launch_vec_add(long L, const double* x, double* y, hipStream_t s) {
    hipLaunchKernelGGL(k_nlc_axpby, vec_grid(L), dim3(256), 0, s, L, 1.0, x, 1.0, y, y);
    PPC_HIP(hipGetLastError());
}

void launch_nonlinear_correction(ppc_problem* pr, const ppc_params* p, const double* U, const double* F,
                                 double* out, bool accumulate, NlcCounts& cnt, int32_t* cocg_out,
                                 hipStream_t s) {
    ensure_nlc(pr, p);
    Workspace& w = pr->ws;
    const int N = p->N, n = pr->mesh.n_free, H = N / 2 + 1;
    const long L = (long)N * n;
    const double dT = p->T / N;
    double* vec = w.nlc_vec;
    double* G = vec + NV_G * L;
    double* B = vec + NV_B * L;
    double* Wc = vec + NV_W * L;
    double* Wt = vec + NV_WT * L;
    double* Uc = vec + NV_U * L;
    double* Phi = vec + NV_PHI * L;
    double* D = vec + NV_D * L;
    double* V = w.nlc_kry;                            // V_0 .. V_kNlcKrylov
    double* Z = w.nlc_kry + (long)(kNlcKrylov + 1) * L;  // Z_0 .. Z_{kNlcKrylov-1}
    double* hd = w.nlc_h;                             // [4][kNlcKrylov + 1]
    const int K1 = kNlcKrylov + 1;
    const dim3 vg = vec_grid(L);
    if (cocg_out)
        for (int q = 0; q < H; ++q) cocg_out[q] = 0;

    // G(U^k) and b = F - G(U^k); W starts at G(U^k)
    coarse_step_sweep(pr, p, U, G, s);
    PPC_HIP(hipMemcpyAsync(w.host_fcount, w.fcount, 8 * (size_t)N * sizeof(int), hipMemcpyDeviceToHost, s));
    PPC_HIP(hipStreamSynchronize(s));
    for (int c = 0; c < N; ++c) {
        const int* q = w.host_fcount + 8 * c;
        if (q[0] != 0)
            fail(q[0], "coarse step " + std::to_string(c + 1) + " of the nonlinear coarse problem failed" +
                           (q[0] == PPC_ERR_NONFINITE ? " (non-finite residual)" : " (Newton did not converge)"));
        cnt.step_newton += q[1];
    }
    hipLaunchKernelGGL(k_nlc_axpby, vg, dim3(256), 0, s, L, 1.0, F, -1.0, G, B);
    PPC_HIP(hipMemcpyAsync(Wc, G, sizeof(double) * L, hipMemcpyDeviceToDevice, s));
    launch_coarse_setup(pr, p, p->lin_point == 1 ? F : U, s);

    // The coarse step's sweep arguments with the base Jacobian for dT.
    ppc_params q1 = *p;
    q1.m = 1;
    FineArgs a = make_fine_args(pr, &q1, nullptr, nullptr);
    a.jbase = w.nlc_jb;

    double scale_c = 0.0;   // ||C F||_F at the start: sets the rounding floor of Phi
    auto residual = [&](const double* Wx) -> double {
        hipLaunchKernelGGL(k_nlc_axpby, vg, dim3(256), 0, s, L, 1.0, Wx, 1.0, B, Uc);
        hipLaunchKernelGGL(k_nlc_residual, dim3(N), dim3(kNlcBlock), 0, s, a, Wx, Uc, Phi, w.nlc_jac,
                           w.nlc_part);
        hipLaunchKernelGGL(k_nlc_sum, dim3(1), dim3(64), 0, s, N, 2, w.nlc_part, hd);
        PPC_HIP(hipGetLastError());
        double h2[2];
        PPC_HIP(hipMemcpyAsync(w.nlc_host, hd, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        PPC_HIP(hipStreamSynchronize(s));
        h2[0] = w.nlc_host[0];
        h2[1] = w.nlc_host[1];
        if (scale_c == 0.0) scale_c = std::sqrt(h2[1]);
        return std::sqrt(h2[0]);    // +inf or NaN when the state overflows the B-H law
    };
    // the dot products V_j . x for j < nv into hd + off (device)
    auto dots = [&](const double* Vb, int nv, const double* x, int off) {
        hipLaunchKernelGGL(k_nlc_dots, dim3(kDotBlocks, nv), dim3(kDotThreads), 0, s, L, Vb, L, x, w.nlc_part);
        hipLaunchKernelGGL(k_nlc_sum, dim3(1), dim3(64), 0, s, kDotBlocks, nv, w.nlc_part, hd + off);
    };

    double rn = residual(Wc);
    if (!std::isfinite(rn)) fail(PPC_ERR_NONFINITE, "non-finite residual in the nonlinear coarse problem");
    const double rn0 = rn;
    const double target = std::max(p->tol_cocg * rn0, 1e-14 * scale_c);
    std::vector<double> Hm((size_t)K1 * kNlcKrylov), g(K1), cs(kNlcKrylov), sn(kNlcKrylov), y(kNlcKrylov);
    std::vector<double> hh(4 * K1);
    constexpr int kMaxNewton = 30;
    bool at_floor = false;
    for (int it = 0; it < kMaxNewton && rn > target; ++it) {
        // flexible GMRES on Jac d = -Phi from d = 0, right-preconditioned by the frozen solve
        const double gm_target = std::max(1e-3 * rn, 0.5 * target);
        hipLaunchKernelGGL(k_nlc_axpby, vg, dim3(256), 0, s, L, -1.0 / rn, Phi, 0.0, nullptr, V);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = rn;
        int used = 0;
        for (int j = 0; j < kNlcKrylov; ++j) {
            double* vj = V + (long)j * L;
            double* zj = Z + (long)j * L;
            double* wv = V + (long)(j + 1) * L;
            launch_coarse_apply(pr, p, vj, zj, s);
            PPC_HIP(hipMemcpyAsync(w.host_ccount, w.ccount, 4 * (size_t)H * sizeof(int), hipMemcpyDeviceToHost, s));
            hipLaunchKernelGGL(k_nlc_jv, dim3((n + 255) / 256, N), dim3(256), 0, s, a, w.nlc_jac, zj, wv, 1.0 / dT);
            // classical Gram-Schmidt twice against V_0..V_j, then ||w||^2
            dots(V, j + 1, wv, 0);
            hipLaunchKernelGGL(k_nlc_subtract, vg, dim3(256), 0, s, L, j + 1, V, L, hd, wv);
            dots(V, j + 1, wv, K1);
            hipLaunchKernelGGL(k_nlc_subtract, vg, dim3(256), 0, s, L, j + 1, V, L, hd + K1, wv);
            dots(wv, 1, wv, 2 * K1);
            PPC_HIP(hipGetLastError());
            PPC_HIP(hipMemcpyAsync(w.nlc_host, hd, 3 * K1 * sizeof(double), hipMemcpyDeviceToHost, s));
            PPC_HIP(hipStreamSynchronize(s));
            std::copy(w.nlc_host, w.nlc_host + 3 * K1, hh.begin());
            // a breakdown or a non-finite residual in a harmonic solve of the preconditioner
            // would carry NaN into the Krylov basis: report it as the frozen correction does
            for (int q = 0; q < H; ++q) {
                const int st = w.host_ccount[4 * q];
                if (st != 0)
                    fail(st, std::string(st == PPC_ERR_BREAKDOWN ? "COCG breakdown" : "non-finite COCG residual") +
                                 " in harmonic " + std::to_string(q) +
                                 " of the nonlinear coarse problem's preconditioner");
            }
            for (int q = 0; q < H; ++q) {
                const int its = w.host_ccount[4 * q + 1];
                cnt.cocg_total += its;
                cnt.cocg_max = std::max(cnt.cocg_max, its);
                if (cocg_out) cocg_out[q] += its;
            }
            cnt.krylov++;
            double* col = Hm.data() + (size_t)j * K1;
            for (int i = 0; i <= j; ++i) col[i] = hh[i] + hh[K1 + i];
            const double hn = std::sqrt(std::max(hh[2 * K1], 0.0));
            col[j + 1] = hn;
            for (int i = 0; i < j; ++i) {       // earlier rotations
                const double t = cs[i] * col[i] + sn[i] * col[i + 1];
                col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
                col[i] = t;
            }
            const double den = std::hypot(col[j], col[j + 1]);
            cs[j] = den > 0.0 ? col[j] / den : 1.0;
            sn[j] = den > 0.0 ? col[j + 1] / den : 0.0;
            col[j] = den;
            col[j + 1] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            used = j + 1;
            if (std::fabs(g[j + 1]) <= gm_target || hn == 0.0) break;
            hipLaunchKernelGGL(k_nlc_axpby, vg, dim3(256), 0, s, L, 1.0 / hn, wv, 0.0, nullptr, wv);
        }
        for (int i = used - 1; i >= 0; --i) {   // H y = g (upper triangular)
            double t = g[i];
            for (int k = i + 1; k < used; ++k) t -= Hm[(size_t)k * K1 + i] * y[k];
            const double dg = Hm[(size_t)i * K1 + i];
            y[i] = dg != 0.0 ? t / dg : 0.0;
        }
        for (int i = 0; i < used; ++i) w.nlc_host[3 * K1 + i] = -y[i];
        PPC_HIP(hipMemcpyAsync(hd + 3 * K1, w.nlc_host + 3 * K1, used * sizeof(double), hipMemcpyHostToDevice, s));
        PPC_HIP(hipMemsetAsync(D, 0, sizeof(double) * L, s));
        hipLaunchKernelGGL(k_nlc_subtract, vg, dim3(256), 0, s, L, used, Z, L, hd + 3 * K1, D);
        // backtracking on ||Phi||
        double lam = 1.0, rt = 0.0;
        bool accepted = false;
        while (lam >= std::ldexp(1.0, -20)) {
            hipLaunchKernelGGL(k_nlc_axpby, vg, dim3(256), 0, s, L, 1.0, Wc, lam, D, Wt);
            rt = residual(Wt);
            if (std::isfinite(rt) && rt <= (1.0 - 1e-4 * lam) * rn) {   // a non-finite trial is a rejected one
                accepted = true;
                break;
            }
            lam *= 0.5;
        }
        cnt.newton++;
        if (!accepted) {
            if (rn <= 1e-11 * scale_c) {        // no decrease representable: rounding floor
                at_floor = true;
                break;
            }
            fail(PPC_ERR_NEWTON, "nonlinear coarse problem: line search failed");
        }
        std::swap(Wc, Wt);
        rn = rt;
    }
    if (rn > target && !at_floor)
        fail(PPC_ERR_NEWTON, "nonlinear coarse problem: no convergence in " + std::to_string(kMaxNewton) +
                                 " Newton steps (||Phi|| = " + std::to_string(rn) + ", target " +
                                 std::to_string(target) + ")");
    hipLaunchKernelGGL(k_nlc_finish, vg, dim3(256), 0, s, L, Wc, B, U, out, accumulate ? 1 : 0);
    PPC_HIP(hipGetLastError());
}

}  // namespace ppc

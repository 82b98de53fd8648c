// Fine sweep host side: kernel shapes, launchers, the base Jacobian and batched launches.
// The device code (Section 2, eqs. (2)-(3)) is in fine_chain.hpp.
#include "fine_chain.hpp"

namespace ppc {

namespace {


// Register rows (R rows per thread, the smallest with R rows_block >= n, in workgroups of
// rows_block threads) when p, r, the FP32 diagonal and the tail sums fit in
// LDS; otherwise (or with block_req = 1024) the streaming memory path with 1024 threads,
// p in LDS when it fits there beside the tail sums (LP = 1).
FineShape pick_shape(int n, size_t n_pad, int n_tail, size_t elem, int block_req, int rows_block) {
    // tail-row sums: one per tail row and history vector (the Galerkin start's products)
    const size_t tail = (size_t)kHist * std::max(n_tail, 1) * elem;
    if (block_req != kFineBlock) {
        // 1024 threads take any R up to 8 (no padded rows beyond the next 1024), and up to
        // 12 in FP32 (in FP64 the LDS runs out first); the smaller workgroups powers of two
        const int rmax = (rows_block == kFineBlock && elem == sizeof(float)) ? 12 : 8;
        for (int R = 1; R <= rmax; ++R) {
            if ((long)R * rows_block < n) continue;
            if (rows_block != kFineBlock && (R & (R - 1)) != 0) continue;
            const size_t lds = 2 * n_pad * elem + n_pad * sizeof(float) + tail;
            if (lds <= kLdsBudget) return {R, rows_block, 0, lds};
            break;
        }
    }
    if (n_pad * elem + tail <= kLdsBudget) return {0, kFineBlock, 1, n_pad * elem + tail};
    return {0, kFineBlock, 0, tail};
}

template <typename S, int R, int BLOCK, int LP>
void launch_shape(const FineArgs& a, int N, size_t lds, hipStream_t s) {
    static bool attr_set = false;
    if (!attr_set) {
        PPC_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fine_sweep<S, R, BLOCK, LP>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBudget));
        attr_set = true;
    }
    hipLaunchKernelGGL((k_fine_sweep<S, R, BLOCK, LP>), dim3(N), dim3(BLOCK), lds, s, a);
}

// R = 9..12 rows per thread at 1024 threads: FP32 only (an FP64 mesh that needs them does
// not fit LDS and takes the memory path)
template <typename S>
void launch_wide(const FineArgs& a, int N, const FineShape& sh, hipStream_t s) {
    if constexpr (sizeof(S) == 4) {
        switch (sh.R) {
            case 9: launch_shape<S, 9, kFineBlock, 0>(a, N, sh.lds, s); return;
            case 10: launch_shape<S, 10, kFineBlock, 0>(a, N, sh.lds, s); return;
            case 11: launch_shape<S, 11, kFineBlock, 0>(a, N, sh.lds, s); return;
            case 12: launch_shape<S, 12, kFineBlock, 0>(a, N, sh.lds, s); return;
            default: break;
        }
    }
    fail(PPC_ERR_ARG, "no fine kernel with " + std::to_string(sh.R) + " rows per thread");
}

template <typename S>
void launch_typed(const FineArgs& a, int N, const FineShape& sh, hipStream_t s) {
    if (sh.R > 0 && sh.block != kFineBlock) launch_fine_rows_small(a, N, sh, sizeof(S) == 8, s);
    else if (sh.R == 1) launch_shape<S, 1, kFineBlock, 0>(a, N, sh.lds, s);
    else if (sh.R == 2) launch_shape<S, 2, kFineBlock, 0>(a, N, sh.lds, s);
    else if (sh.R == 3) launch_shape<S, 3, kFineBlock, 0>(a, N, sh.lds, s);
    else if (sh.R == 4) launch_shape<S, 4, kFineBlock, 0>(a, N, sh.lds, s);
    else if (sh.R == 5) launch_shape<S, 5, kFineBlock, 0>(a, N, sh.lds, s);
    else if (sh.R == 6) launch_shape<S, 6, kFineBlock, 0>(a, N, sh.lds, s);
    else if (sh.R == 7) launch_shape<S, 7, kFineBlock, 0>(a, N, sh.lds, s);
    else if (sh.R == 8) launch_shape<S, 8, kFineBlock, 0>(a, N, sh.lds, s);
    else if (sh.R > 8) launch_wide<S>(a, N, sh, s);
    else if (sh.LP == 1) launch_shape<S, 0, kFineBlock, 1>(a, N, sh.lds, s);
    else launch_shape<S, 0, kFineBlock, 0>(a, N, sh.lds, s);
}

}  // namespace

// Base Jacobian Jb of a sweep: value position v takes M_s / dt of its CSR slot s plus
// nu K0_ab of every linear element contribution of s (slot order); padding takes 0.
__global__ void k_jbase(int nvals, int ne, const int* __restrict__ vslot, const int* __restrict__ slot_ptr,
                        const int* __restrict__ slot_src, const int* __restrict__ mat,
                        const double* __restrict__ lawtab, const double* __restrict__ k0,
                        const double* __restrict__ mval, double inv_dt, double* __restrict__ jb) {
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < nvals; v += gridDim.x * blockDim.x) {
        const int s = vslot[v];
        double acc = 0.0;
        if (s >= 0) {
            acc = mval[s] * inv_dt;
            for (int k = slot_ptr[s]; k < slot_ptr[s + 1]; ++k) {
                const int code = slot_src[k];
                const int e = code / 9, ab = code - 9 * e;
                const double* L = lawtab + 5 * mat[e];
                if (L[0] != 0.0) continue;        // Brauer: added per Newton iteration
                const int qa = ab / 3, qb = ab - 3 * qa;
                const int lo = qa < qb ? qa : qb, hi = qa < qb ? qb : qa;
                const int kidx = lo == 0 ? hi : (lo == 1 ? 2 + hi : 5);
                acc += L[1] * k0[(long)kidx * ne + e];
            }
        }
        jb[v] = acc;
    }
}

// (Re)build the base Jacobian when the step size changed since the last build.
void ensure_jbase(ppc_problem* pr, const ppc_params* p, hipStream_t s) {
    Workspace& w = pr->ws;
    const DeviceMesh& d = pr->mesh;
    const double dt = p->T / (double)(p->N * p->m);
    if (w.jbase_dt == dt) return;
    const int nb = std::max(1, std::min((d.n_vals + 255) / 256, 4096));
    hipLaunchKernelGGL(k_jbase, dim3(nb), dim3(256), 0, s, d.n_vals, d.n_tri, d.vslot, d.slot_ptr, d.slot_src,
                       d.mat, pr->lawtab, d.k0, d.mval, 1.0 / dt, w.jbase);
    PPC_HIP(hipGetLastError());
    w.jbase_dt = dt;
}

FineArgs make_fine_args(ppc_problem* pr, const ppc_params* p, const double* U, double* F) {
    const DeviceMesh& d = pr->mesh;
    Workspace& w = pr->ws;
    FineArgs a{};
    a.n = d.n_free;
    a.N = p->N;
    a.m = p->m;
    a.T = p->T;
    a.dt = p->T / (double)(p->N * p->m);
    a.fnorm = d.fnorm;
    a.tol_newton = p->tol_newton;
    a.tol_lin = p->tol_lin;
    a.max_newton = p->max_newton;
    a.max_lin = p->max_lin;
    a.rowptr = d.rowptr;
    a.colidx = d.colidx;
    a.mval = d.mval;
    a.mell = d.mell;
    a.fload = d.fload;
    a.lawtab = pr->lawtab;
    a.wavtab = pr->wavtab;
    a.n_h = pr->wave.n_h;
    a.f0 = pr->wave.f0;
    a.U = U;
    a.F = F;
    a.vec = w.fvec;
    a.pcg = w.fpcg;
    a.jac = w.fjac;
    a.elem = w.felem;
    a.nl_pad = (long)w.nl_pad;
    a.jbase = w.jbase;
    a.n_nl = d.n_nl;
    a.n_nlv = d.n_nlv;
    a.nl_efree = d.nl_efree;
    a.nl_mat = d.nl_mat;
    a.nl_area = d.nl_area;
    a.nl_k0 = d.nl_k0;
    a.nlv_val = d.nlv_val;
    a.nlv_ptr = d.nlv_ptr;
    a.nlv_src = d.nlv_src;
    a.nlf_ptr = d.nlf_ptr;
    a.nlf_src = d.nlf_src;
    a.count = w.fcount;
    a.n_pad = (long)w.n_pad;
    a.vals_pad = (long)w.vals_pad;
    a.W = d.ell_w;
    a.ntail = d.n_tail;
    a.nvals = d.n_vals;
    a.ell_pad = (long)d.ell_pad;
    a.ecol = d.ecol;
    a.ecol16 = d.ecol16;
    a.dpos = d.dpos;
    a.tail_row = d.tail_row;
    a.tail_ptr = d.tail_ptr;
    a.tail_col = d.tail_col;
    a.predictor = p->no_predictor == 0 ? 1 : 0;
    // 0 picks by precision: the Galerkin start pays in FP64 PCG, where solves run long
    // enough for the saved iterations to outweigh its three Jacobian products, and
    // costs time in FP32 PCG, whose looser solves save fewer iterations
    a.lin_start = p->lin_start == 1 || (p->lin_start == 0 && p->precision != 0) ? 1 : 0;
    a.lin_forcing = p->lin_forcing;
    a.traj = nullptr;
    a.adapt_scal = nullptr;
    a.tol_adapt = p->tol_adapt;
    return a;
}

FineShape rows_shape(const ppc_problem* pr, const ppc_params* p, int rows_block) {
    const size_t elem = p->precision == 0 ? sizeof(double) : sizeof(float);
    // the register-row SpMV reads 16-bit columns (built for n < 65536; R B <= 8192 rows)
    const int block = pr->mesh.ecol16 ? p->block : kFineBlock;
    const size_t n_pad = ((size_t)pr->mesh.n_free + 63) / 64 * 64;   // the workspace's row padding
    return pick_shape(pr->mesh.n_free, n_pad, pr->mesh.n_tail, elem, block, rows_block);
}

// Register-row workgroup size: params->fine_block when set, else the tuned size of this
// precision, else 1024.  A forced size whose rows do not fit is an argument error.
FineShape fine_shape(const ppc_problem* pr, const ppc_params* p) {
    const int tuned = pr->tuned_block[p->precision != 0 ? 1 : 0];
    const int rb = p->fine_block ? p->fine_block : (tuned ? tuned : kFineBlock);
    const FineShape sh = rows_shape(pr, p, rb);
    if (p->fine_block && sh.R == 0)
        fail(PPC_ERR_ARG, "fine_block " + std::to_string(p->fine_block) + ": the mesh's " +
                              std::to_string(pr->mesh.n_free) + " rows do not fit register rows at that size");
    return sh;
}


void launch_fine_sweep(ppc_problem* pr, const ppc_params* p, const double* U, double* F,
                       hipStream_t s, const double* adapt_scal) {
    ensure_jbase(pr, p, s);
    FineArgs a = make_fine_args(pr, p, U, F);
    if (p->tol_adapt > 0.0) a.adapt_scal = adapt_scal;
    const FineShape sh = fine_shape(pr, p);
    if (p->precision == 0)
        launch_typed<double>(a, p->N, sh, s);
    else
        launch_typed<float>(a, p->N, sh, s);
    PPC_HIP(hipGetLastError());
}

void launch_fine_sweep_traj(ppc_problem* pr, const ppc_params* p, const double* U, double* F,
                            double* traj, hipStream_t s) {
    ensure_jbase(pr, p, s);
    FineArgs a = make_fine_args(pr, p, U, F);
    a.traj = traj;
    const FineShape sh = fine_shape(pr, p);
    if (p->precision == 0)
        launch_typed<double>(a, p->N, sh, s);
    else
        launch_typed<float>(a, p->N, sh, s);
    PPC_HIP(hipGetLastError());
}

size_t fine_scratch_layout(const ppc_problem* pr, const ppc_params* p, unsigned char* base, FineScratch* out) {
    const DeviceMesh& d = pr->mesh;
    const size_t N = (size_t)p->N;
    const size_t s = p->precision == 0 ? sizeof(double) : sizeof(float);
    auto pad = [](size_t x, size_t q) { return (x + q - 1) / q * q; };
    FineScratch sc;
    sc.n_pad = (long)pad((size_t)d.n_free, 64);
    sc.vals_pad = (long)pad((size_t)d.n_vals, 64);
    sc.nl_pad = (long)pad((size_t)std::max(d.n_nl, 1), 64);
    size_t off = 0;
    auto take = [&](size_t bytes) -> unsigned char* {
        unsigned char* q = base ? base + off : nullptr;
        off += pad(std::max<size_t>(bytes, 1), 256);
        return q;
    };
    sc.jbase = reinterpret_cast<double*>(take((size_t)sc.vals_pad * sizeof(double)));
    sc.vec = reinterpret_cast<double*>(take(N * kFineVec * (size_t)sc.n_pad * sizeof(double)));
    sc.pcg = take(N * kPcgVec * (size_t)sc.n_pad * s);
    sc.jac = take(N * (size_t)sc.vals_pad * s);
    sc.elem = reinterpret_cast<double*>(take(N * 8 * (size_t)sc.nl_pad * sizeof(double)));
    sc.count = reinterpret_cast<int*>(take(N * 8 * sizeof(int)));
    if (out) *out = sc;
    return off;
}

void launch_fine_sweep_in(ppc_problem* pr, const ppc_params* p, const double* U, double* F,
                          const FineScratch& sc, hipStream_t s) {
    const DeviceMesh& d = pr->mesh;
    const double dt = p->T / (double)(p->N * p->m);
    const int nb = std::max(1, std::min((d.n_vals + 255) / 256, 4096));
    hipLaunchKernelGGL(k_jbase, dim3(nb), dim3(256), 0, s, d.n_vals, d.n_tri, d.vslot, d.slot_ptr, d.slot_src,
                       d.mat, pr->lawtab, d.k0, d.mval, 1.0 / dt, sc.jbase);
    FineArgs a = make_fine_args(pr, p, U, F);
    a.vec = sc.vec;
    a.pcg = sc.pcg;
    a.jac = sc.jac;
    a.elem = sc.elem;
    a.nl_pad = sc.nl_pad;
    a.jbase = sc.jbase;
    a.count = sc.count;
    a.n_pad = sc.n_pad;
    a.vals_pad = sc.vals_pad;
    const FineShape sh = fine_shape(pr, p);
    if (p->precision == 0)
        launch_typed<double>(a, p->N, sh, s);
    else
        launch_typed<float>(a, p->N, sh, s);
    PPC_HIP(hipGetLastError());
}

namespace {

template <int R, int LP>
void launch_adj_shape(const FineArgs& a, const AdjArgs& b, size_t lds, hipStream_t s) {
    static bool attr_set = false;
    if (!attr_set) {
        PPC_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_adjoint_sweep<double, R, kFineBlock, LP>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBudget));
        attr_set = true;
    }
    hipLaunchKernelGGL((k_adjoint_sweep<double, R, kFineBlock, LP>), dim3(a.N), dim3(kFineBlock), lds, s, a, b);
}

}  // namespace

// The adjoint solves are FP64 whatever the forward precision.
void launch_adjoint_sweep(ppc_problem* pr, const ppc_params* p, const AdjArgs& b, hipStream_t s) {
    ensure_jbase(pr, p, s);
    const FineArgs a = make_fine_args(pr, p, nullptr, nullptr);
    const FineShape sh = pick_shape(pr->mesh.n_free, pr->ws.n_pad, pr->mesh.n_tail, sizeof(double), p->block,
                                    kFineBlock);
    if (sh.R == 1) launch_adj_shape<1, 0>(a, b, sh.lds, s);
    else if (sh.R == 2) launch_adj_shape<2, 0>(a, b, sh.lds, s);
    else if (sh.R == 3) launch_adj_shape<3, 0>(a, b, sh.lds, s);
    else if (sh.R == 4) launch_adj_shape<4, 0>(a, b, sh.lds, s);
    else if (sh.R == 5) launch_adj_shape<5, 0>(a, b, sh.lds, s);
    else if (sh.R == 6) launch_adj_shape<6, 0>(a, b, sh.lds, s);
    else if (sh.R == 7) launch_adj_shape<7, 0>(a, b, sh.lds, s);
    else if (sh.R == 8) launch_adj_shape<8, 0>(a, b, sh.lds, s);
    else if (sh.LP == 1) launch_adj_shape<0, 1>(a, b, sh.lds, s);
    else launch_adj_shape<0, 0>(a, b, sh.lds, s);
    PPC_HIP(hipGetLastError());
}

namespace {

template <typename S, int R, int LP>
void launch_batch_shape(const FineArgs* args, const int2* work, int nblocks, size_t lds, hipStream_t s) {
    static bool attr_set = false;
    if (!attr_set) {
        PPC_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fine_sweep_batch<S, R, kFineBlock, LP>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBudget));
        attr_set = true;
    }
    hipLaunchKernelGGL((k_fine_sweep_batch<S, R, kFineBlock, LP>), dim3(nblocks), dim3(kFineBlock), lds, s,
                       args, work);
}

template <typename S>
void launch_batch_wide(const FineArgs* args, const int2* work, int nblocks, const FineShape& sh, hipStream_t s) {
    if constexpr (sizeof(S) == 4) {
        switch (sh.R) {
            case 9: launch_batch_shape<S, 9, 0>(args, work, nblocks, sh.lds, s); return;
            case 10: launch_batch_shape<S, 10, 0>(args, work, nblocks, sh.lds, s); return;
            case 11: launch_batch_shape<S, 11, 0>(args, work, nblocks, sh.lds, s); return;
            case 12: launch_batch_shape<S, 12, 0>(args, work, nblocks, sh.lds, s); return;
            default: break;
        }
    }
    fail(PPC_ERR_ARG, "no fine kernel with " + std::to_string(sh.R) + " rows per thread");
}

template <typename S>
void launch_batch_typed(const FineArgs* args, const int2* work, int nblocks, const FineShape& sh,
                        hipStream_t s) {
    if (sh.R > 0 && sh.block != kFineBlock) launch_fine_batch_rows_small(args, work, nblocks, sh, sizeof(S) == 8, s);
    else if (sh.R == 1) launch_batch_shape<S, 1, 0>(args, work, nblocks, sh.lds, s);
    else if (sh.R == 2) launch_batch_shape<S, 2, 0>(args, work, nblocks, sh.lds, s);
    else if (sh.R == 3) launch_batch_shape<S, 3, 0>(args, work, nblocks, sh.lds, s);
    else if (sh.R == 4) launch_batch_shape<S, 4, 0>(args, work, nblocks, sh.lds, s);
    else if (sh.R == 5) launch_batch_shape<S, 5, 0>(args, work, nblocks, sh.lds, s);
    else if (sh.R == 6) launch_batch_shape<S, 6, 0>(args, work, nblocks, sh.lds, s);
    else if (sh.R == 7) launch_batch_shape<S, 7, 0>(args, work, nblocks, sh.lds, s);
    else if (sh.R == 8) launch_batch_shape<S, 8, 0>(args, work, nblocks, sh.lds, s);
    else if (sh.R > 8) launch_batch_wide<S>(args, work, nblocks, sh, s);
    else if (sh.LP == 1) launch_batch_shape<S, 0, 1>(args, work, nblocks, sh.lds, s);
    else launch_batch_shape<S, 0, 0>(args, work, nblocks, sh.lds, s);
}

int shape_key(const FineShape& sh) { return sh.block * 256 + sh.R * 16 + sh.LP; }

}  // namespace

void FineBatch::release() {
    if (d_args) (void)hipFree(d_args);
    if (d_work) (void)hipFree(d_work);
    d_args = nullptr;
    d_work = nullptr;
    work_cap = 0;
}

// Upload one FineArgs per design (U / F are each design's own state arrays).  With
// adapt_scal and params->tol_adapt, design d's sweeps read its jump norms at adapt_scal + 3 d.
void fine_batch_prepare(FineBatch& b, const std::vector<ppc_problem*>& parts, const ppc_params* p,
                        hipStream_t s, const double* adapt_scal) {
    const int D = (int)parts.size();
    std::vector<FineArgs> host(D);
    b.shapes.resize(D);
    b.sizes.clear();
    for (int d = 0; d < D; ++d) {
        ensure_jbase(parts[d], p, s);
        host[d] = make_fine_args(parts[d], p, parts[d]->ws.U, parts[d]->ws.F);
        if (adapt_scal && p->tol_adapt > 0.0) host[d].adapt_scal = adapt_scal + 3 * d;
        b.shapes[d] = fine_shape(parts[d], p);
        b.sizes.push_back(parts[d]->mesh.n_free);
    }
    b.h = D > 0 ? parts[0]->h : nullptr;
    if (b.d_args) (void)hipFree(b.d_args);
    PPC_HIP(hipMalloc(&b.d_args, sizeof(FineArgs) * D));
    PPC_HIP(hipMemcpyAsync(b.d_args, host.data(), sizeof(FineArgs) * D, hipMemcpyHostToDevice, s));
    PPC_HIP(hipStreamSynchronize(s));
    b.N = p->N;
    b.precision = p->precision;
}

// Work list of the active designs' chains, longest designs first, grouped by kernel shape,
// uploaded to d_work; synchronises so that the host list may change afterwards.
void fine_batch_plan(FineBatch& b, const std::vector<char>& active, hipStream_t s) {
    const int D = (int)b.shapes.size();
    std::vector<int> order;
    for (int d = 0; d < D; ++d)
        if (active[d]) order.push_back(d);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return b.sizes[x] > b.sizes[y]; });
    std::vector<int> keys;
    for (int d : order) {
        const int k = shape_key(b.shapes[d]);
        if (std::find(keys.begin(), keys.end(), k) == keys.end()) keys.push_back(k);
    }
    std::vector<int2> work;
    b.spans.clear();
    b.span_shapes.clear();
    for (int k : keys) {
        const size_t start = work.size();
        FineShape sh{};
        for (int d : order) {
            if (shape_key(b.shapes[d]) != k) continue;
            if (b.shapes[d].lds >= sh.lds) sh = b.shapes[d];
            for (int c = 0; c < b.N; ++c) work.push_back(make_int2(d, c));
        }
        b.spans.emplace_back(start, work.size() - start);
        b.span_shapes.push_back(sh);
    }
    if (work.empty()) return;
    if (work.size() > b.work_cap) {
        if (b.d_work) (void)hipFree(b.d_work);
        PPC_HIP(hipMalloc(&b.d_work, sizeof(int2) * work.size()));
        b.work_cap = work.size();
    }
    b.host_work = work;
    PPC_HIP(hipMemcpyAsync(b.d_work, b.host_work.data(), sizeof(int2) * work.size(), hipMemcpyHostToDevice, s));
    PPC_HIP(hipStreamSynchronize(s));
}

// One launch per kernel shape over the planned work list.  Several shapes run side by side:
// group g goes to the main stream (g = 0) or a side stream, which waits for the main
// stream's work so far and which the main stream waits for at the end, so every group can
// fill the CUs the others leave free.
void fine_batch_run(const FineBatch& b, hipStream_t s) {
    const size_t G = b.spans.size();
    Lanes lanes(G > 1 ? b.h : nullptr, s);
    for (size_t g = 0; g < G; ++g) {
        hipStream_t sg = lanes.lane((int)g);
        const int2* w = b.d_work + b.spans[g].first;
        const int nb = (int)b.spans[g].second;
        if (b.precision == 0)
            launch_batch_typed<double>(b.d_args, w, nb, b.span_shapes[g], sg);
        else
            launch_batch_typed<float>(b.d_args, w, nb, b.span_shapes[g], sg);
    }
    lanes.join();
    PPC_HIP(hipGetLastError());
}

void fine_batch_launch(FineBatch& b, const std::vector<char>& active, hipStream_t s) {
    fine_batch_plan(b, active, s);
    fine_batch_run(b, s);
}

}  // namespace ppc

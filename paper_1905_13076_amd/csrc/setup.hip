// Problem set-up: validation, sparsity pattern and element maps on the host, element
// geometry / conductivity mass / load on the device.
//
// Discretisation of eq. (1) (Section 2) with linear triangles: per element the edge
// coefficients b_a = y_{a+1} - y_{a+2}, c_a = x_{a+2} - x_{a+1} (cyclic), area
// A = |b_0 c_1 - b_1 c_0| / 2, unit curl-curl matrix K0_ab = (b_a b_b + c_a c_b)/(4A),
// conductivity mass sigma A/12 (1 + delta_ab) and load js A/3.  Dirichlet nodes
// (A = 0) are eliminated; the free nodes keep ascending node order.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "internal.hpp"

namespace ppc {

namespace {

bool finite(double v) { return std::isfinite(v); }

int find_root(std::vector<int>& p, int x) {
    while (p[x] != x) {
        p[x] = p[p[x]];
        x = p[x];
    }
    return x;
}

}  // namespace

int validate_problem(const ppc_mesh* mesh, const ppc_material* mat, const ppc_excitation* exc,
                     std::string& msg) {
    if (!mesh || !mat || !exc) { msg = "null mesh, material or excitation"; return PPC_ERR_ARG; }
    if (mesh->n_nodes < 3 || mesh->n_tri < 1) { msg = "need n_nodes >= 3 and n_tri >= 1"; return PPC_ERR_ARG; }
    if (!mesh->xy || !mesh->tri) { msg = "null xy or tri"; return PPC_ERR_ARG; }
    if (mesh->n_dir < 1 || !mesh->dir) { msg = "no Dirichlet node: K would be singular"; return PPC_ERR_MESH; }
    const int nn = mesh->n_nodes, ne = mesh->n_tri;
    if ((int64_t)ne * 9 > (int64_t)INT32_MAX / 2) { msg = "mesh too large for int32 slot codes"; return PPC_ERR_ARG; }
    for (int i = 0; i < 2 * nn; ++i)
        if (!finite(mesh->xy[i])) { msg = "non-finite node coordinate"; return PPC_ERR_ARG; }
    std::vector<int> touched(nn, 0);
    for (int e = 0; e < ne; ++e) {
        const int* t = mesh->tri + 3 * e;
        for (int a = 0; a < 3; ++a)
            if (t[a] < 0 || t[a] >= nn) { msg = "triangle " + std::to_string(e) + " has an out-of-range node"; return PPC_ERR_MESH; }
        if (t[0] == t[1] || t[1] == t[2] || t[0] == t[2]) { msg = "triangle " + std::to_string(e) + " repeats a node"; return PPC_ERR_MESH; }
        double x[3], y[3];
        for (int a = 0; a < 3; ++a) { x[a] = mesh->xy[2 * t[a]]; y[a] = mesh->xy[2 * t[a] + 1]; }
        const double b0 = y[1] - y[2], b1 = y[2] - y[0];
        const double c0 = x[2] - x[1], c1 = x[0] - x[2];
        const double a2 = std::fabs(b0 * c1 - b1 * c0);
        double h2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            const double dx = x[(a + 1) % 3] - x[a], dy = y[(a + 1) % 3] - y[a];
            h2 = std::max(h2, dx * dx + dy * dy);
        }
        if (!(a2 > 1e-12 * h2)) { msg = "triangle " + std::to_string(e) + " is degenerate"; return PPC_ERR_MESH; }
        for (int a = 0; a < 3; ++a) touched[t[a]] = 1;
    }
    for (int i = 0; i < nn; ++i)
        if (!touched[i]) { msg = "node " + std::to_string(i) + " belongs to no triangle"; return PPC_ERR_MESH; }
    std::vector<char> isdir(nn, 0);
    for (int k = 0; k < mesh->n_dir; ++k) {
        const int d = mesh->dir[k];
        if (d < 0 || d >= nn) { msg = "Dirichlet index out of range"; return PPC_ERR_MESH; }
        isdir[d] = 1;
    }
    int n_free = 0;
    for (int i = 0; i < nn; ++i) n_free += !isdir[i];
    if (n_free == 0) { msg = "every node is a Dirichlet node: nothing to solve"; return PPC_ERR_MESH; }
    // every connected component must hold a Dirichlet node, else K is singular
    std::vector<int> par(nn);
    std::iota(par.begin(), par.end(), 0);
    for (int e = 0; e < ne; ++e) {
        const int* t = mesh->tri + 3 * e;
        for (int a = 1; a < 3; ++a) {
            const int r0 = find_root(par, t[0]), r1 = find_root(par, t[a]);
            if (r0 != r1) par[r1] = r0;
        }
    }
    std::vector<char> comp_dir(nn, 0);
    for (int i = 0; i < nn; ++i)
        if (isdir[i]) comp_dir[find_root(par, i)] = 1;
    for (int i = 0; i < nn; ++i)
        if (!comp_dir[find_root(par, i)]) { msg = "a connected part of the mesh has no Dirichlet node"; return PPC_ERR_MESH; }
    // materials
    if (!mat->sigma || !mat->mat_id || !mat->table) { msg = "null material array"; return PPC_ERR_ARG; }
    if (mat->n_mat < 1 || mat->n_mat > kMaxMaterials) { msg = "n_mat must be in [1, 64]"; return PPC_ERR_ARG; }
    for (int k = 0; k < mat->n_mat; ++k) {
        const ppc_law& L = mat->table[k];
        if (L.law == PPC_LAW_LINEAR) {
            if (!finite(L.nu) || !(L.nu > 0.0)) { msg = "linear law needs a finite nu > 0"; return PPC_ERR_ARG; }
        } else if (L.law == PPC_LAW_BRAUER) {
            if (!finite(L.k1) || !finite(L.k2) || !finite(L.k3) || L.k1 < 0.0 || L.k2 < 0.0 || !(L.k3 > 0.0)) {
                msg = "Brauer law needs finite k1 >= 0, k2 >= 0, k3 > 0";
                return PPC_ERR_ARG;
            }
        } else {
            msg = "unknown law " + std::to_string(L.law);
            return PPC_ERR_ARG;
        }
    }
    for (int e = 0; e < ne; ++e) {
        if (!finite(mat->sigma[e]) || mat->sigma[e] < 0.0) { msg = "sigma must be finite and >= 0"; return PPC_ERR_ARG; }
        if (mat->mat_id[e] < 0 || mat->mat_id[e] >= mat->n_mat) { msg = "mat_id out of range"; return PPC_ERR_ARG; }
    }
    // excitation
    if (!exc->js) { msg = "null js"; return PPC_ERR_ARG; }
    for (int e = 0; e < ne; ++e)
        if (!finite(exc->js[e])) { msg = "non-finite js"; return PPC_ERR_ARG; }
    if (!finite(exc->f0) || exc->f0 < 0.0) { msg = "f0 must be finite and >= 0"; return PPC_ERR_ARG; }
    if (exc->n_h < 0 || exc->n_h > kMaxHarmonicTerms) { msg = "n_h must be in [0, 16]"; return PPC_ERR_ARG; }
    if (exc->n_h > 0 && (!exc->order || !exc->amp || !exc->phase)) { msg = "null waveform array"; return PPC_ERR_ARG; }
    for (int k = 0; k < exc->n_h; ++k)
        if (exc->order[k] < 0 || !finite(exc->amp[k]) || !finite(exc->phase[k])) {
            msg = "waveform terms need order >= 0 and finite amp, phase";
            return PPC_ERR_ARG;
        }
    return PPC_OK;
}

int validate_params(const ppc_params* p, std::string& msg) {
    if (!p) { msg = "null params"; return PPC_ERR_ARG; }
    if (!finite(p->T) || !(p->T > 0.0)) { msg = "T must be finite and > 0"; return PPC_ERR_ARG; }
    if (p->N < 2 || (p->N % 2) != 0) { msg = "N must be even and >= 2"; return PPC_ERR_ARG; }
    if (p->N > 4096) { msg = "N must be <= 4096"; return PPC_ERR_ARG; }
    if (p->m < 1) { msg = "m must be >= 1"; return PPC_ERR_ARG; }
    if (p->shift_mode < 0 || p->shift_mode > 1) { msg = "shift_mode must be 0 or 1"; return PPC_ERR_ARG; }
    if (p->lin_mode < 0 || p->lin_mode > 1) { msg = "lin_mode must be 0 or 1"; return PPC_ERR_ARG; }
    if (p->init_mode < 0 || p->init_mode > 4) { msg = "init_mode must be 0, 1, 2, 3 or 4"; return PPC_ERR_ARG; }
    if (p->precision < 0 || p->precision > 1) { msg = "precision must be 0 or 1"; return PPC_ERR_ARG; }
    if (p->graph < 0 || p->graph > 1) { msg = "graph must be 0 or 1"; return PPC_ERR_ARG; }
    if (p->method < 0 || p->method > 1) { msg = "method must be 0 (PP-PC) or 1 (PP-IC)"; return PPC_ERR_ARG; }
    if (p->method == 1 && p->b_cap > 0.0) { msg = "b_cap applies to PP-PC only"; return PPC_ERR_ARG; }
    if (p->n_harm < 0 || p->n_harm > p->N / 2 + 1) { msg = "n_harm must be 0 (all) or 1..N/2+1"; return PPC_ERR_ARG; }
    if (p->method == 1 && p->n_harm != 0) { msg = "n_harm applies to PP-PC only"; return PPC_ERR_ARG; }
    if (p->fine_block != 0 && p->fine_block != 256 && p->fine_block != 512 && p->fine_block != 1024) {
        msg = "fine_block must be 0, 256, 512 or 1024";
        return PPC_ERR_ARG;
    }
    if (p->fine_block != 0 && p->block == 1024) {
        msg = "fine_block selects register rows; block 1024 forces the memory path";
        return PPC_ERR_ARG;
    }
    if (!(p->b_cap >= 0.0) || !std::isfinite(p->b_cap)) { msg = "b_cap must be finite and >= 0"; return PPC_ERR_ARG; }
    if (p->coarse_mode < 0 || p->coarse_mode > 1) {
        msg = "coarse_mode must be 0 (frozen) or 1 (nonlinear)";
        return PPC_ERR_ARG;
    }
    if (p->coarse_mode == 1 && (p->method != 0 || p->n_harm != 0 || p->b_cap > 0.0)) {
        msg = "coarse_mode 1 applies to PP-PC with all harmonics and without b_cap";
        return PPC_ERR_ARG;
    }
    if (p->coarse_precision < -1 || p->coarse_precision > 1) {
        msg = "coarse_precision must be -1, 0 or 1";
        return PPC_ERR_ARG;
    }
    if (!finite(p->tol_ppc) || p->tol_ppc < 0.0) { msg = "tol_ppc must be finite and >= 0"; return PPC_ERR_ARG; }
    if (p->max_iters < 0 || p->max_iters > 100000) { msg = "max_iters out of range"; return PPC_ERR_ARG; }
    if (!finite(p->tol_newton) || !(p->tol_newton > 0.0)) { msg = "tol_newton must be > 0"; return PPC_ERR_ARG; }
    if (p->max_newton < 1) { msg = "max_newton must be >= 1"; return PPC_ERR_ARG; }
    if (!finite(p->tol_lin) || !(p->tol_lin > 0.0) || p->tol_lin >= 1.0) { msg = "tol_lin must be in (0, 1)"; return PPC_ERR_ARG; }
    if (p->max_lin < 1) { msg = "max_lin must be >= 1"; return PPC_ERR_ARG; }
    if (!finite(p->tol_cocg) || !(p->tol_cocg > 0.0) || p->tol_cocg >= 1.0) { msg = "tol_cocg must be in (0, 1)"; return PPC_ERR_ARG; }
    if (p->max_cocg < 1) { msg = "max_cocg must be >= 1"; return PPC_ERR_ARG; }
    if (p->no_predictor < 0 || p->no_predictor > 1) { msg = "no_predictor must be 0 or 1"; return PPC_ERR_ARG; }
    if (p->lin_start < 0 || p->lin_start > 2) { msg = "lin_start must be 0, 1 or 2"; return PPC_ERR_ARG; }
    if (p->lin_forcing < 0 || p->lin_forcing > 1) { msg = "lin_forcing must be 0 or 1"; return PPC_ERR_ARG; }
    if (!finite(p->tol_adapt) || p->tol_adapt < 0.0 || p->tol_adapt >= 1.0) {
        msg = "tol_adapt must be in [0, 1)";
        return PPC_ERR_ARG;
    }
    if (p->lin_point < 0 || p->lin_point > 1) { msg = "lin_point must be 0 or 1"; return PPC_ERR_ARG; }
    if (p->block != 0 && (p->block < 64 || p->block > 1024 || (p->block % 64) != 0)) {
        msg = "block must be 0 or a multiple of 64 in [64, 1024]";
        return PPC_ERR_ARG;
    }
    return PPC_OK;
}

// ------------------------------------------------------------------------------------
// set-up kernels (a1): geometry, conductivity mass, load
// ------------------------------------------------------------------------------------
__global__ void k_geometry(int ne, const double* __restrict__ xy, const int* __restrict__ tri,
                           double* __restrict__ area, double* __restrict__ k0,
                           double* __restrict__ gx, double* __restrict__ gy) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += gridDim.x * blockDim.x) {
        double x[3], y[3];
        for (int a = 0; a < 3; ++a) {
            const int v = tri[3 * e + a];
            x[a] = xy[2 * v];
            y[a] = xy[2 * v + 1];
        }
        double b[3], c[3];
        for (int a = 0; a < 3; ++a) {
            b[a] = y[(a + 1) % 3] - y[(a + 2) % 3];
            c[a] = x[(a + 2) % 3] - x[(a + 1) % 3];
        }
        const double a2s = b[0] * c[1] - b[1] * c[0];   // twice the signed area
        const double A = 0.5 * fabs(a2s);
        area[e] = A;
        const double s = 1.0 / (4.0 * A);
        k0[0 * ne + e] = (b[0] * b[0] + c[0] * c[0]) * s;
        k0[1 * ne + e] = (b[0] * b[1] + c[0] * c[1]) * s;
        k0[2 * ne + e] = (b[0] * b[2] + c[0] * c[2]) * s;
        k0[3 * ne + e] = (b[1] * b[1] + c[1] * c[1]) * s;
        k0[4 * ne + e] = (b[1] * b[2] + c[1] * c[2]) * s;
        k0[5 * ne + e] = (b[2] * b[2] + c[2] * c[2]) * s;
        for (int a = 0; a < 3; ++a) {
            gx[a * ne + e] = b[a] / a2s;
            gy[a * ne + e] = c[a] / a2s;
        }
    }
}

// compact copies of the area and K0 of the Brauer elements
__global__ void k_gather_nl(int nnl, int ne, const int* __restrict__ nl_elem,
                            const double* __restrict__ area, const double* __restrict__ k0,
                            double* __restrict__ nl_area, double* __restrict__ nl_k0) {
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < nnl; j += gridDim.x * blockDim.x) {
        const int e = nl_elem[j];
        nl_area[j] = area[e];
        for (int q = 0; q < 6; ++q) nl_k0[(size_t)q * nnl + j] = k0[(size_t)q * ne + e];
    }
}

// M_s = sum over contributions (e, a, b) of sigma_e A_e / 12 (1 + delta_ab)
__global__ void k_mass(int nnz, const int* __restrict__ slot_ptr, const int* __restrict__ slot_src,
                       const double* __restrict__ sigma, const double* __restrict__ area,
                       double* __restrict__ mval) {
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < nnz; s += gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int k = slot_ptr[s]; k < slot_ptr[s + 1]; ++k) {
            const int code = slot_src[k];
            const int e = code / 9, ab = code % 9;
            const double w = ((ab / 3) == (ab % 3)) ? 2.0 : 1.0;
            acc += sigma[e] * area[e] * (w / 12.0);
        }
        mval[s] = acc;
    }
}

// F_i = sum over incident (e, a) of js_e A_e / 3; also the mass diagonal
__global__ void k_load(int n, const int* __restrict__ node_ptr, const int* __restrict__ node_src,
                       const double* __restrict__ js, const double* __restrict__ area,
                       const int* __restrict__ diag, const double* __restrict__ mval,
                       double* __restrict__ fload, double* __restrict__ mdiag) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int k = node_ptr[i]; k < node_ptr[i + 1]; ++k) {
            const int e = node_src[k] / 3;
            acc += js[e] * area[e] / 3.0;
        }
        fload[i] = acc;
        mdiag[i] = mval[diag[i]];
    }
}

// M at each ELL value position: mell_v = M_{vslot_v} (0 for padding)
__global__ void k_mell(int nvals, const int* __restrict__ vslot, const double* __restrict__ mval,
                       double* __restrict__ mell) {
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < nvals; v += gridDim.x * blockDim.x) {
        const int s = vslot[v];
        mell[v] = s >= 0 ? mval[s] : 0.0;
    }
}

__global__ void k_to_f32(int n, const double* __restrict__ x, float* __restrict__ y) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) y[i] = (float)x[i];
}

// ||x||_2 over one block, fixed summation order
__global__ void k_norm2(int n, const double* __restrict__ x, double* __restrict__ out) {
    __shared__ double red[1024];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc += x[i] * x[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sqrt(red[0]);
}

namespace {

template <typename T>
T* dalloc(size_t n) {
    void* p = nullptr;
    if (n == 0) n = 1;
    const hipError_t e = hipMalloc(&p, n * sizeof(T));
    if (e != hipSuccess) fail(PPC_ERR_OOM, "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed");
    return static_cast<T*>(p);
}

template <typename T>
T* upload(const std::vector<T>& v, hipStream_t s) {
    T* d = dalloc<T>(v.size());
    if (!v.empty()) PPC_HIP(hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return d;
}

int grid_for(int n, int block) {
    const int g = (n + block - 1) / block;
    return std::max(1, std::min(g, 4096));
}

}  // namespace

void build_problem(ppc_problem* pr, const ppc_mesh* mesh, const ppc_material* mat,
                   const ppc_excitation* exc, hipStream_t s) {
    DeviceMesh& d = pr->mesh;
    const int nn = mesh->n_nodes, ne = mesh->n_tri;
    d.n_nodes = nn;
    d.n_tri = ne;
    // free numbering: non-Dirichlet nodes in ascending order
    std::vector<char> isdir(nn, 0);
    for (int k = 0; k < mesh->n_dir; ++k) isdir[mesh->dir[k]] = 1;
    pr->free_of_node.assign(nn, -1);
    std::vector<int> free_node;
    for (int i = 0; i < nn; ++i)
        if (!isdir[i]) {
            pr->free_of_node[i] = (int)free_node.size();
            free_node.push_back(i);
        }
    const int n = (int)free_node.size();
    d.n_free = n;
    // vertex -> free index planes
    std::vector<int> efree(3 * (size_t)ne);
    for (int e = 0; e < ne; ++e)
        for (int a = 0; a < 3; ++a) efree[(size_t)a * ne + e] = pr->free_of_node[mesh->tri[3 * e + a]];
    // CSR pattern among free nodes
    std::vector<std::vector<int>> cols(n);
    for (int e = 0; e < ne; ++e)
        for (int a = 0; a < 3; ++a) {
            const int i = efree[(size_t)a * ne + e];
            if (i < 0) continue;
            for (int b = 0; b < 3; ++b) {
                const int j = efree[(size_t)b * ne + e];
                if (j >= 0) cols[i].push_back(j);
            }
        }
    std::vector<int> rowptr(n + 1, 0), colidx;
    int max_row = 0;
    for (int i = 0; i < n; ++i) {
        auto& c = cols[i];
        std::sort(c.begin(), c.end());
        c.erase(std::unique(c.begin(), c.end()), c.end());
        rowptr[i + 1] = rowptr[i] + (int)c.size();
        max_row = std::max(max_row, (int)c.size());
    }
    colidx.reserve(rowptr[n]);
    for (int i = 0; i < n; ++i) colidx.insert(colidx.end(), cols[i].begin(), cols[i].end());
    cols.clear();
    cols.shrink_to_fit();
    const int nnz = rowptr[n];
    d.nnz = nnz;
    d.max_row = max_row;
    auto slot_of = [&](int i, int j) {
        const int* b = colidx.data() + rowptr[i];
        const int* e = colidx.data() + rowptr[i + 1];
        const int* p = std::lower_bound(b, e, j);
        return (int)(p - colidx.data());
    };
    std::vector<int> diag(n);
    for (int i = 0; i < n; ++i) diag[i] = slot_of(i, i);
    // slot -> contributions (counting sort by slot)
    std::vector<int> slot_ptr(nnz + 1, 0), code_slot;
    std::vector<int> codes;
    codes.reserve(9 * (size_t)ne);
    code_slot.reserve(9 * (size_t)ne);
    for (int e = 0; e < ne; ++e)
        for (int a = 0; a < 3; ++a) {
            const int i = efree[(size_t)a * ne + e];
            if (i < 0) continue;
            for (int b = 0; b < 3; ++b) {
                const int j = efree[(size_t)b * ne + e];
                if (j < 0) continue;
                const int sl = slot_of(i, j);
                codes.push_back(e * 9 + a * 3 + b);
                code_slot.push_back(sl);
                slot_ptr[sl + 1]++;
            }
        }
    for (int k = 0; k < nnz; ++k) slot_ptr[k + 1] += slot_ptr[k];
    std::vector<int> slot_src(codes.size());
    {
        std::vector<int> fillp(slot_ptr.begin(), slot_ptr.end() - 1);
        for (size_t k = 0; k < codes.size(); ++k) slot_src[fillp[code_slot[k]]++] = codes[k];
    }
    d.n_contrib = (int)codes.size();
    // ELL layout for the fine sweep
    const size_t NP = (n + 63) / 64 * 64;
    int W = 1;
    bool has_long = false;
    for (int i = 0; i < n; ++i) {
        const int len = rowptr[i + 1] - rowptr[i];
        if (len <= kEllMaxWidth) W = std::max(W, len);
        else has_long = true;
    }
    if (has_long) W = std::max(W, 2);   // slot 1 of a tail row holds its tail index
    std::vector<int> ecol((size_t)W * NP, 0), tail_row, tail_ptr(1, 0), tail_col, dpos(n);
    std::vector<int> vslot((size_t)W * NP, -1);
    for (int i = 0; i < n; ++i) {
        const int len = rowptr[i + 1] - rowptr[i];
        if (len <= W) {
            for (int k = 0; k < W; ++k) {
                const size_t v = (size_t)k * NP + i;
                if (k < len) {
                    ecol[v] = colidx[rowptr[i] + k];
                    vslot[v] = rowptr[i] + k;
                    if (ecol[v] == i) dpos[i] = (int)v;
                } else {
                    ecol[v] = i;   // padding: zero value times the row's own entry
                }
            }
        } else {
            ecol[i] = -1;
            ecol[NP + i] = (int)tail_row.size();
            tail_row.push_back(i);
            for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) tail_col.push_back(colidx[k]);
            tail_ptr.push_back((int)tail_col.size());
        }
    }
    const size_t tail_base = (size_t)W * NP;
    for (size_t t = 0; t < tail_row.size(); ++t) {
        const int i = tail_row[t];
        for (int k = tail_ptr[t]; k < tail_ptr[t + 1]; ++k) {
            const int slot = rowptr[i] + (k - tail_ptr[t]);
            vslot.push_back(slot);
            if (colidx[slot] == i) dpos[i] = (int)(tail_base + k);
        }
    }
    d.ell_w = W;
    d.ell_pad = NP;
    d.n_tail = (int)tail_row.size();
    d.tail_nnz = (int)tail_col.size();
    d.n_vals = (int)vslot.size();
    // free node -> incident vertices
    std::vector<int> node_ptr(n + 1, 0);
    for (int e = 0; e < ne; ++e)
        for (int a = 0; a < 3; ++a) {
            const int i = efree[(size_t)a * ne + e];
            if (i >= 0) node_ptr[i + 1]++;
        }
    for (int i = 0; i < n; ++i) node_ptr[i + 1] += node_ptr[i];
    std::vector<int> node_src(node_ptr[n]);
    {
        std::vector<int> fillp(node_ptr.begin(), node_ptr.end() - 1);
        for (int e = 0; e < ne; ++e)
            for (int a = 0; a < 3; ++a) {
                const int i = efree[(size_t)a * ne + e];
                if (i >= 0) node_src[fillp[i]++] = e * 3 + a;
            }
    }
    // materials and waveform
    Laws& L = pr->laws;
    L.n_mat = mat->n_mat;
    for (int k = 0; k < mat->n_mat; ++k) {
        L.law[k] = mat->table[k].law;
        L.nu[k] = mat->table[k].nu;
        L.k1[k] = mat->table[k].k1;
        L.k2[k] = mat->table[k].k2;
        L.k3[k] = mat->table[k].k3;
    }
    pr->nl_elem.clear();
    for (int e = 0; e < ne; ++e)
        if (L.law[mat->mat_id[e]] == PPC_LAW_BRAUER) pr->nl_elem.push_back(e);
    d.nonlinear = !pr->nl_elem.empty();
    // Brauer elements in a compact numbering j; the ELL value positions whose slot holds a
    // Brauer contribution (codes j*9 + a*3 + b, slot order); per row, the incident
    // Brauer elements (codes j*3 + a, node order).
    const int nnl = (int)pr->nl_elem.size();
    std::vector<int> nl_of_elem(ne, -1), nl_efree(3 * (size_t)nnl), nl_mat(nnl);
    for (int j = 0; j < nnl; ++j) {
        const int e = pr->nl_elem[j];
        nl_of_elem[e] = j;
        for (int a = 0; a < 3; ++a) nl_efree[(size_t)a * nnl + j] = efree[(size_t)a * ne + e];
        nl_mat[j] = mat->mat_id[e];
    }
    std::vector<int> nlv_val, nlv_ptr(1, 0), nlv_src;
    for (size_t v = 0; v < vslot.size(); ++v) {
        const int sl = vslot[v];
        if (sl < 0) continue;
        const size_t before = nlv_src.size();
        for (int k = slot_ptr[sl]; k < slot_ptr[sl + 1]; ++k) {
            const int j = nl_of_elem[slot_src[k] / 9];
            if (j >= 0) nlv_src.push_back(j * 9 + slot_src[k] % 9);
        }
        if (nlv_src.size() > before) {
            nlv_val.push_back((int)v);
            nlv_ptr.push_back((int)nlv_src.size());
        }
    }
    std::vector<int> nlf_ptr(n + 1, 0), nlf_src;
    for (int i = 0; i < n; ++i) {
        for (int k = node_ptr[i]; k < node_ptr[i + 1]; ++k) {
            const int j = nl_of_elem[node_src[k] / 3];
            if (j >= 0) nlf_src.push_back(j * 3 + node_src[k] % 3);
        }
        nlf_ptr[i + 1] = (int)nlf_src.size();
    }
    d.n_nl = nnl;
    d.n_nlv = (int)nlv_val.size();
    {
        std::vector<double> lt(5 * (size_t)mat->n_mat);
        for (int k = 0; k < mat->n_mat; ++k) {
            lt[5 * k + 0] = (double)L.law[k];
            lt[5 * k + 1] = L.nu[k];
            lt[5 * k + 2] = L.k1[k];
            lt[5 * k + 3] = L.k2[k];
            lt[5 * k + 4] = L.k3[k];
        }
        pr->lawtab = upload(lt, s);
        std::vector<double> wt(3 * (size_t)std::max(1, exc->n_h), 0.0);
        for (int k = 0; k < exc->n_h; ++k) {
            wt[3 * k + 0] = (double)exc->order[k];
            wt[3 * k + 1] = exc->amp[k];
            wt[3 * k + 2] = exc->phase[k];
        }
        pr->wavtab = upload(wt, s);
    }
    Wave& wave = pr->wave;
    wave.f0 = exc->f0;
    wave.n_h = exc->n_h;
    for (int k = 0; k < exc->n_h; ++k) {
        wave.order[k] = exc->order[k];
        wave.amp[k] = exc->amp[k];
        wave.phase[k] = exc->phase[k];
    }
    // upload
    d.rowptr = upload(rowptr, s);
    d.colidx = upload(colidx, s);
    d.diag = upload(diag, s);
    d.slot_ptr = upload(slot_ptr, s);
    d.slot_src = upload(slot_src, s);
    d.node_ptr = upload(node_ptr, s);
    d.node_src = upload(node_src, s);
    d.efree = upload(efree, s);
    d.ecol = upload(ecol, s);
    if (n < 65536) {
        std::vector<unsigned short> e16(ecol.size());
        for (size_t v = 0; v < ecol.size(); ++v) e16[v] = (unsigned short)(ecol[v] < 0 ? 0 : ecol[v]);
        d.ecol16 = upload(e16, s);
    }
    d.vslot = upload(vslot, s);
    d.dpos = upload(dpos, s);
    d.tail_row = upload(tail_row, s);
    d.tail_ptr = upload(tail_ptr, s);
    d.tail_col = upload(tail_col, s);
    d.free_node = upload(free_node, s);
    d.nl_elem = upload(pr->nl_elem, s);
    d.nl_efree = upload(nl_efree, s);
    d.nl_mat = upload(nl_mat, s);
    d.nlv_val = upload(nlv_val, s);
    d.nlv_ptr = upload(nlv_ptr, s);
    d.nlv_src = upload(nlv_src, s);
    d.nlf_ptr = upload(nlf_ptr, s);
    d.nlf_src = upload(nlf_src, s);
    d.mat = upload(std::vector<int>(mat->mat_id, mat->mat_id + ne), s);
    d.xy = upload(std::vector<double>(mesh->xy, mesh->xy + 2 * (size_t)nn), s);
    d.tri = upload(std::vector<int>(mesh->tri, mesh->tri + 3 * (size_t)ne), s);
    d.sigma = upload(std::vector<double>(mat->sigma, mat->sigma + ne), s);
    d.js = upload(std::vector<double>(exc->js, exc->js + ne), s);
    d.area = dalloc<double>(ne);
    d.k0 = dalloc<double>(6 * (size_t)ne);
    d.gx = dalloc<double>(3 * (size_t)ne);
    d.gy = dalloc<double>(3 * (size_t)ne);
    d.nl_area = dalloc<double>(nnl);
    d.nl_k0 = dalloc<double>(6 * (size_t)nnl);
    d.mval = dalloc<double>(nnz);
    d.mdiag = dalloc<double>(n);
    d.fload = dalloc<double>(n);
    double* fn = dalloc<double>(1);
    hipLaunchKernelGGL(k_geometry, dim3(grid_for(ne, 256)), dim3(256), 0, s, ne, d.xy, d.tri, d.area,
                       d.k0, d.gx, d.gy);
    if (nnl > 0)
        hipLaunchKernelGGL(k_gather_nl, dim3(grid_for(nnl, 256)), dim3(256), 0, s, nnl, ne, d.nl_elem,
                           d.area, d.k0, d.nl_area, d.nl_k0);
    hipLaunchKernelGGL(k_mass, dim3(grid_for(nnz, 256)), dim3(256), 0, s, nnz, d.slot_ptr, d.slot_src,
                       d.sigma, d.area, d.mval);
    hipLaunchKernelGGL(k_load, dim3(grid_for(n, 256)), dim3(256), 0, s, n, d.node_ptr, d.node_src,
                       d.js, d.area, d.diag, d.mval, d.fload, d.mdiag);
    d.mval32 = dalloc<float>(nnz);
    hipLaunchKernelGGL(k_to_f32, dim3(grid_for(nnz, 256)), dim3(256), 0, s, nnz, d.mval, d.mval32);
    d.mell = dalloc<double>((size_t)d.n_vals);
    hipLaunchKernelGGL(k_mell, dim3(grid_for(d.n_vals, 256)), dim3(256), 0, s, d.n_vals, d.vslot, d.mval, d.mell);
    hipLaunchKernelGGL(k_norm2, dim3(1), dim3(1024), 0, s, n, d.fload, fn);
    PPC_HIP(hipGetLastError());
    PPC_HIP(hipMemcpyAsync(&d.fnorm, fn, sizeof(double), hipMemcpyDeviceToHost, s));
    PPC_HIP(hipStreamSynchronize(s));
    PPC_HIP(hipFree(fn));
}

void mesh_free(DeviceMesh& d) {
    void* ptrs[] = {d.rowptr, d.colidx, d.diag, d.slot_ptr, d.slot_src, d.node_ptr, d.node_src,
                    d.efree, d.free_node, d.mat, d.xy, d.tri, d.area, d.k0, d.gx, d.gy,
                    d.sigma, d.js, d.mval, d.mval32, d.mdiag, d.fload, d.ecol, d.ecol16, d.vslot, d.mell, d.dpos,
                    d.tail_row, d.tail_ptr, d.tail_col, d.nl_elem, d.nl_efree, d.nl_mat, d.nl_area,
                    d.nl_k0, d.nlv_val, d.nlv_ptr, d.nlv_src, d.nlf_ptr, d.nlf_src};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    d = DeviceMesh{};
}

}  // namespace ppc

// Adjoint of the periodic steady state: loss, gradients and the time-reversal helpers.
//
// Loss (the period-averaged eddy-current loss, the exact element integral of
// sigma (dA/dt)^2 over the periodic fine trajectory of eq. (1) discretised by implicit
// Euler):  P = 1/(T dt) sum_j du_j^T M du_j,  du_j = u_j - u_{j-1}.
// Adjoint: J_j lambda_j = (M/dt) lambda_{j+1} + dP/du_j (cyclic), solved by the backward
// fine sweep (fine.hip) inside a PP-PC iteration whose coarse correction is the forward
// one (Section 3, eqs. (11)-(14)) applied to the time-reversed jumps: reversing the
// subinterval index turns the backward cyclic coarse system into the forward one.
// Gradients: dP/dtheta = dP/dtheta|_u - sum_j lambda_j^T dR_j/dtheta for every element
// conductivity and the Brauer constants of every material.
#include <cmath>

#include "internal.hpp"

namespace ppc {

namespace {

__device__ inline double block_reduce_256(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    return red[0];
}

}  // namespace

// dst[r] = src[N-1-r]
__global__ void k_reverse_rows(int N, int n, const double* __restrict__ src, double* __restrict__ dst) {
    const long total = (long)N * n;
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < total; k += (long)gridDim.x * blockDim.x) {
        const long r = k / n;
        const long i = k - r * n;
        dst[k] = src[(N - 1 - r) * n + i];
    }
}

// L[c] += dR[N-1-c]
__global__ void k_add_reversed(int N, int n, const double* __restrict__ dR, double* __restrict__ L) {
    const long total = (long)N * n;
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < total; k += (long)gridDim.x * blockDim.x) {
        const long c = k / n;
        const long i = k - c * n;
        L[k] += dR[(N - 1 - c) * n + i];
    }
}

// one block per fine step (c, jl): du^T M du, du = traj[c][jl] - traj[c][jl-1]
__global__ void k_loss_steps(int n, int m, const int* __restrict__ rowptr, const int* __restrict__ colidx,
                             const double* __restrict__ mval, const double* __restrict__ traj,
                             double* __restrict__ part) {
    __shared__ double red[256];
    const int b = blockIdx.x;
    const int c = b / m, jl = b % m + 1;
    const double* u1 = traj + ((long)c * (m + 1) + jl) * n;
    const double* u0 = u1 - n;
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        double mu = 0.0;
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            const int j = colidx[k];
            mu += mval[k] * (u1[j] - u0[j]);
        }
        acc += (u1[i] - u0[i]) * mu;
    }
    const double s = block_reduce_256(acc, red);
    if (threadIdx.x == 0) part[b] = s;
}

__global__ void k_sum_scaled(int nb, const double* __restrict__ part, double scale, double* __restrict__ out) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) acc += part[b];
    const double s = block_reduce_256(acc, red);
    if (threadIdx.x == 0) out[0] = s * scale;
}

// Per element: dP/dsigma_e and the Brauer partials -sum_j dnu/dk lambda_e . w_e.
__global__ void k_grad_elem(int ne, int n, int N, int m, double T, double dt,
                            const int* __restrict__ efree, const double* __restrict__ area,
                            const double* __restrict__ k0, const int* __restrict__ mat,
                            const double* __restrict__ lawtab, const double* __restrict__ traj,
                            const double* __restrict__ lam, double* __restrict__ dsig,
                            double* __restrict__ dk) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += gridDim.x * blockDim.x) {
        int g[3];
        for (int q = 0; q < 3; ++q) g[q] = efree[q * ne + e];
        const double A = area[e];
        const double* L = lawtab + 5 * mat[e];
        const bool brauer = L[0] != 0.0;
        const double k00 = k0[e], k01 = k0[ne + e], k02 = k0[2 * ne + e];
        const double k11 = k0[3 * ne + e], k12 = k0[4 * ne + e], k22 = k0[5 * ne + e];
        double s_sig = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        for (int c = 0; c < N; ++c) {
            const double* Tc = traj + (long)c * (m + 1) * n;
            for (int jl = 1; jl <= m; ++jl) {
                const double* u1 = Tc + (long)jl * n;
                const double* u0 = u1 - n;
                const double* lj = lam + ((long)c * m + (jl - 1)) * n;
                double uv[3], de[3], le[3];
                for (int q = 0; q < 3; ++q) {
                    const int gq = g[q];
                    uv[q] = gq >= 0 ? u1[gq] : 0.0;
                    de[q] = gq >= 0 ? u1[gq] - u0[gq] : 0.0;
                    le[q] = gq >= 0 ? lj[gq] : 0.0;
                }
                const double sd = de[0] + de[1] + de[2];
                double dMd = 0.0, lMd = 0.0;
                for (int q = 0; q < 3; ++q) {
                    const double md = A / 12.0 * (de[q] + sd);
                    dMd += de[q] * md;
                    lMd += le[q] * md;
                }
                s_sig += dMd / (T * dt) - lMd / dt;
                if (brauer) {
                    const double w0 = k00 * uv[0] + k01 * uv[1] + k02 * uv[2];
                    const double w1 = k01 * uv[0] + k11 * uv[1] + k12 * uv[2];
                    const double w2 = k02 * uv[0] + k12 * uv[1] + k22 * uv[2];
                    const double b2 = (uv[0] * w0 + uv[1] * w1 + uv[2] * w2) / A;
                    const double ex = exp(L[3] * b2);
                    const double lw = le[0] * w0 + le[1] * w1 + le[2] * w2;
                    s1 -= ex * lw;
                    s2 -= L[2] * b2 * ex * lw;
                    s3 -= lw;
                }
            }
        }
        dsig[e] = s_sig;
        dk[e] = s1;
        dk[ne + e] = s2;
        dk[2 * ne + e] = s3;
    }
}

// one block per material: dk_mat[mid][q] = sum over its Brauer elements (fixed order)
__global__ void k_grad_mat(int ne, const int* __restrict__ mat, const double* __restrict__ lawtab,
                           const double* __restrict__ dk, double* __restrict__ out) {
    __shared__ double red[256];
    const int mid = blockIdx.x;
    const bool brauer = lawtab[5 * mid] != 0.0;
    for (int q = 0; q < 3; ++q) {
        double acc = 0.0;
        if (brauer)
            for (int e = threadIdx.x; e < ne; e += blockDim.x)
                if (mat[e] == mid) acc += dk[q * ne + e];
        const double s = block_reduce_256(acc, red);
        if (threadIdx.x == 0) out[3 * mid + q] = s;
        __syncthreads();
    }
}

void launch_reverse_rows(int N, int n, const double* src, double* dst, hipStream_t s) {
    hipLaunchKernelGGL(k_reverse_rows, dim3(1024), dim3(256), 0, s, N, n, src, dst);
    PPC_HIP(hipGetLastError());
}

void launch_add_reversed(int N, int n, const double* dR, double* L, hipStream_t s) {
    hipLaunchKernelGGL(k_add_reversed, dim3(1024), dim3(256), 0, s, N, n, dR, L);
    PPC_HIP(hipGetLastError());
}

void launch_loss(ppc_problem* pr, const ppc_params* p, const double* traj, double* part, double* out,
                 hipStream_t s) {
    const DeviceMesh& d = pr->mesh;
    const int nb = p->N * p->m;
    const double dt = p->T / (double)(p->N * p->m);
    hipLaunchKernelGGL(k_loss_steps, dim3(nb), dim3(256), 0, s, d.n_free, p->m, d.rowptr, d.colidx, d.mval,
                       traj, part);
    hipLaunchKernelGGL(k_sum_scaled, dim3(1), dim3(256), 0, s, nb, part, 1.0 / (p->T * dt), out);
    PPC_HIP(hipGetLastError());
}

void launch_gradients(ppc_problem* pr, const ppc_params* p, const double* traj, const double* lam_all,
                      double* dsig, double* dk_elem, double* dk_mat, int n_mat, hipStream_t s) {
    const DeviceMesh& d = pr->mesh;
    const double dt = p->T / (double)(p->N * p->m);
    const int g = std::max(1, std::min((d.n_tri + 255) / 256, 4096));
    hipLaunchKernelGGL(k_grad_elem, dim3(g), dim3(256), 0, s, d.n_tri, d.n_free, p->N, p->m, p->T, dt, d.efree,
                       d.area, d.k0, d.mat, pr->lawtab, traj, lam_all, dsig, dk_elem);
    hipLaunchKernelGGL(k_grad_mat, dim3(n_mat), dim3(256), 0, s, d.n_tri, d.mat, pr->lawtab, dk_elem, dk_mat);
    PPC_HIP(hipGetLastError());
}

}  // namespace ppc

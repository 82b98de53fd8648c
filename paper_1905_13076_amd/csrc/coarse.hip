// Coarse periodic correction (Section 3) and the per-iteration jumps (Section 2).
//
// In the linear case eq. (4) with the implicit-Euler coarse propagator of eq. (8) is
// the block-cyclic system G U^{k+1} = r^k of eq. (9); since r^k = G U^k + Q J^k with
// the jumps J_n = F_n - U_n (n mod N), the new iterate is U^{k+1} = U^k + dU with
//     Q dU_n - C dU_{n-1} = Q J_n    (cyclic in n),   C = M/dT,  Q = C + Kbar  (eq. (10)).
// The DFT along time (eqs. (11)-(13)) turns G into the blocks Kbar + sigma_p M with
// sigma_p = (1 - exp(-i w_p dT))/dT, w_p = 2 pi p / T, one independent complex-symmetric
// system per harmonic p = 0..N/2 (the negative harmonics are the conjugates); the
// inverse transform (eq. (14)) returns dU.  For a nonlinear problem the paper defers
// the treatment of the coarse matrices; here Kbar is frozen at the time average over
// the coarse samples of the differential reluctivity (or of the chord reluctivity).
//
// Kernels: jumps + norms (two-level fixed-order reduction), linearisation per element,
// Kbar by slot gather, coarse right-hand side R_n = Q J_n (the matrix read once per
// row for all samples), DFT along time with a twiddle table, one workgroup per
// harmonic running Jacobi-preconditioned COCG in complex FP64 (van der Vorst and
// Melissen's conjugate-orthogonal CG for complex symmetric matrices), and the inverse
// DFT fused with the update U += dU.
#include <cmath>

#include "internal.hpp"
#include "wave.hpp"

namespace ppc {

namespace {
constexpr int kRedBlocks = 256;

__device__ inline double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cdiv(double2 a, double2 b) {
    const double s = fabs(b.x) > fabs(b.y) ? fabs(b.x) : fabs(b.y);
    const double bx = b.x / s, by = b.y / s;
    const double d = bx * bx + by * by;
    return make_double2((a.x * bx + a.y * by) / d / s, (a.y * bx - a.x * by) / d / s);
}

template <int K>
__device__ inline void block_sum_d(double (&v)[K], double* lds, int& phase) {
#pragma unroll
    for (int k = 0; k < K; ++k)
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    double* buf = lds + phase * 16 * K;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) buf[w * K + k] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (int j = 0; j < nw; ++j) s += buf[j * K + k];
        v[k] = s;
    }
    phase ^= 1;
}
}  // namespace

// J = F - U over [N][n]; per-block partial sums of ||J||^2, ||U||^2, ||J_0||^2
__global__ void k_jumps(long total, int n, const double* __restrict__ U, const double* __restrict__ F,
                        double* __restrict__ J, double* __restrict__ part) {
    __shared__ double lds[2 * 16 * 3];
    int ph = 0;
    double v[3] = {0.0, 0.0, 0.0};
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < total; k += (long)gridDim.x * blockDim.x) {
        const double j = F[k] - U[k];
        if (J) J[k] = j;
        v[0] += j * j;
        v[1] += U[k] * U[k];
        if (k < n) v[2] += j * j;
    }
    block_sum_d<3>(v, lds, ph);
    if (threadIdx.x == 0)
        for (int q = 0; q < 3; ++q) part[3 * blockIdx.x + q] = v[q];
}

__global__ void k_sum_partials(int nb, int K, const double* __restrict__ part, double* __restrict__ out) {
    if (threadIdx.x < K) {
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += part[K * b + threadIdx.x];
        out[threadIdx.x] = s;
    }
}

// Per element: time average over the samples of nu I + 2 nu' g g^T (lin_mode 0) or of
// nu I (lin_mode 1), g = grad A_h.  U null means one sample u = 0.
__global__ void k_linearise(int ne, int n, int nsamp, const double* __restrict__ U,
                            const int* __restrict__ efree, const double* __restrict__ gx,
                            const double* __restrict__ gy, const double* __restrict__ area,
                            const double* __restrict__ k0, const int* __restrict__ mat,
                            const double* __restrict__ lawtab, int lin_mode,
                            double* __restrict__ nub) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += gridDim.x * blockDim.x) {
        int g[3];
        double ax[3], ay[3];
        for (int q = 0; q < 3; ++q) {
            g[q] = efree[q * ne + e];
            ax[q] = gx[q * ne + e];
            ay[q] = gy[q * ne + e];
        }
        const double* L = lawtab + 5 * mat[e];
        const bool brauer = L[0] != 0.0;
        double sxx = 0.0, sxy = 0.0, syy = 0.0;
        const int ns = U ? nsamp : 1;
        for (int s = 0; s < ns; ++s) {
            double uv[3];
            for (int q = 0; q < 3; ++q) uv[q] = (U && g[q] >= 0) ? U[(long)s * n + g[q]] : 0.0;
            double nu, dnu = 0.0, gxx = 0.0, gyy = 0.0;
            if (lin_mode == 0) {
                gxx = ax[0] * uv[0] + ax[1] * uv[1] + ax[2] * uv[2];
                gyy = ay[0] * uv[0] + ay[1] * uv[1] + ay[2] * uv[2];
                const double b2 = gxx * gxx + gyy * gyy;
                if (brauer) {
                    const double ex = exp(L[3] * b2);
                    nu = L[2] * ex + L[4];
                    dnu = L[2] * L[3] * ex;
                } else {
                    nu = L[1];
                }
            } else {
                // chord: nu at b2 = u.(K0 u)/A
                const double k00 = k0[e], k01 = k0[ne + e], k02 = k0[2 * ne + e];
                const double k11 = k0[3 * ne + e], k12 = k0[4 * ne + e], k22 = k0[5 * ne + e];
                const double w0 = k00 * uv[0] + k01 * uv[1] + k02 * uv[2];
                const double w1 = k01 * uv[0] + k11 * uv[1] + k12 * uv[2];
                const double w2 = k02 * uv[0] + k12 * uv[1] + k22 * uv[2];
                const double b2 = (uv[0] * w0 + uv[1] * w1 + uv[2] * w2) / area[e];
                nu = brauer ? L[2] * exp(L[3] * b2) + L[4] : L[1];
            }
            sxx += nu + 2.0 * dnu * gxx * gxx;
            sxy += 2.0 * dnu * gxx * gyy;
            syy += nu + 2.0 * dnu * gyy * gyy;
        }
        nub[e] = sxx / ns;
        nub[ne + e] = sxy / ns;
        nub[2 * ne + e] = syy / ns;
    }
}

// Kbar_s = sum over contributions (e, a, b) of A_e g_a^T nubar_e g_b
__global__ void k_kbar(int nnz, int ne, const int* __restrict__ slot_ptr, const int* __restrict__ slot_src,
                       const double* __restrict__ area, const double* __restrict__ gx,
                       const double* __restrict__ gy, const double* __restrict__ nub,
                       double* __restrict__ kbar, float* __restrict__ kbar32) {
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < nnz; s += gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int k = slot_ptr[s]; k < slot_ptr[s + 1]; ++k) {
            const int code = slot_src[k];
            const int e = code / 9, ab = code - 9 * e;
            const int qa = ab / 3, qb = ab - 3 * qa;
            const double xa = gx[qa * ne + e], ya = gy[qa * ne + e];
            const double xb = gx[qb * ne + e], yb = gy[qb * ne + e];
            acc += area[e] * (nub[e] * xa * xb + nub[ne + e] * (xa * yb + ya * xb) + nub[2 * ne + e] * ya * yb);
        }
        kbar[s] = acc;
        kbar32[s] = (float)acc;
    }
}

// R[s][i] = sum_k (M_k / dT + Kbar_k) J[s][col_k]
__global__ void k_coarse_rhs(int n, int N, const int* __restrict__ rowptr, const int* __restrict__ colidx,
                             const double* __restrict__ mval, const double* __restrict__ kbar,
                             double inv_dT, const double* __restrict__ J, double* __restrict__ R) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (i >= n || s >= N) return;
    const double* Js = J + (long)s * n;
    double acc = 0.0;
    for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) acc += (mval[k] * inv_dT + kbar[k]) * Js[colidx[k]];
    R[(long)s * n + i] = acc;
}

// Time stepping: samples U[j mod N] = traj[j m] (the state at T_j), j = 1..N, of one
// chain's trajectory over a whole period ([N m + 1][n], row 0 the start).
__global__ void k_gather_samples(int n, int N, int m, const double* __restrict__ traj, double* __restrict__ U) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y + 1;
    if (i >= n) return;
    U[(long)(j % N) * n + i] = traj[(long)j * m * n + i];
}

// Per sample s (one workgroup each): out[2s] = ||A_s - B_s||^2, out[2s+1] = ||A_s||^2.
__global__ void k_sample_change(int n, const double* __restrict__ A, const double* __restrict__ B,
                                double* __restrict__ out) {
    __shared__ double red[2][256];
    const int s = blockIdx.x;
    const double* a = A + (long)s * n;
    const double* b = B + (long)s * n;
    double dd = 0.0, aa = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double d = a[i] - b[i];
        dd += d * d;
        aa += a[i] * a[i];
    }
    red[0][threadIdx.x] = dd;
    red[1][threadIdx.x] = aa;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[2 * s] = red[0][0];
        out[2 * s + 1] = red[1][0];
    }
}

void launch_gather_samples(int n, int N, int m, const double* traj, double* U, hipStream_t s) {
    hipLaunchKernelGGL(k_gather_samples, dim3((n + 255) / 256, N), dim3(256), 0, s, n, N, m, traj, U);
    PPC_HIP(hipGetLastError());
}

void launch_sample_change(int n, int N, const double* A, const double* B, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_sample_change, dim3(N), dim3(256), 0, s, n, A, B, out);
    PPC_HIP(hipGetLastError());
}

// PP-IC start of a propagation (eq. (5)): e = U_N - U^k_0, then U_0 = U_N; thread 0 also
// sets the single shift 1/dT of the propagation's solves.
__global__ void k_ic_start(int n, double inv_dT, const double* __restrict__ un, double* __restrict__ u0,
                           double* __restrict__ e, double2* __restrict__ sig) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) sig[0] = make_double2(inv_dT, 0.0);
    if (i >= n) return;
    const double v = un[i];
    e[i] = v - u0[i];
    u0[i] = v;
}

// PP-IC right-hand side C e = M e / dT, as a complex vector with zero imaginary part
__global__ void k_ic_rhs(int n, const int* __restrict__ rowptr, const int* __restrict__ colidx,
                         const double* __restrict__ mval, double inv_dT, const double* __restrict__ e,
                         double2* __restrict__ b) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) acc += mval[k] * e[colidx[k]];
    b[i] = make_double2(acc * inv_dT, 0.0);
}

// PP-IC step: v = F_n + x (x = Q^{-1} C e); rows n < N: e = v - U^k_n and U_n = v; row N
// (u == null): U_N = v, the next iteration's U_0.
__global__ void k_ic_update(int n, const double2* __restrict__ x, const double* __restrict__ f,
                            double* __restrict__ u, double* __restrict__ e, double* __restrict__ un) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double v = f[i] + x[i].x;
    if (u) {
        e[i] = v - u[i];
        u[i] = v;
    } else {
        un[i] = v;
    }
}

// R[s][i] = i(T_s) F_i with row 0 carrying T_N = T (the coarse excitation rows of eq. (9))
__global__ void k_excitation_rows(int n, int N, double T, const double* __restrict__ fload,
                                  const double* __restrict__ wav, int n_h, double f0,
                                  double* __restrict__ R) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (i >= n || s >= N) return;
    const double t = s == 0 ? T : s * (T / N);
    double cur = 0.0;
    for (int h = 0; h < n_h; ++h) cur = cur + wav[3 * h + 1] * sin(2.0 * M_PI * wav[3 * h] * f0 * t + wav[3 * h + 2]);
    R[(long)s * n + i] = cur * fload[i];
}

__global__ void k_twiddle(int N, double2* __restrict__ tw) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    double s, c;
    sincospi(2.0 * k / N, &s, &c);
    tw[k] = make_double2(c, -s);   // exp(-2 pi i k / N)
}

// Rhat[p][i] = sum_s R[s][i] exp(-2 pi i p s / N) for harmonics p = p0 + blockIdx.y
__global__ void k_dft(int n, int N, int p0, const double* __restrict__ R, const double2* __restrict__ tw,
                      double2* __restrict__ Rh) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int p = p0 + blockIdx.y;
    if (i >= n) return;
    double re = 0.0, im = 0.0;
    for (int s = 0; s < N; ++s) {
        const double r = R[(long)s * n + i];
        const double2 w = tw[(int)(((long)p * s) % N)];
        re += r * w.x;
        im += r * w.y;
    }
    Rh[(long)p * n + i] = make_double2(re, im);
}

// One workgroup per harmonic p: (Kbar + sigma_p M) x = b by Jacobi-preconditioned COCG.
__device__ __forceinline__ void cocg_body(const CocgArgs& a, const int p, double* lds) {
    const int n = a.n;
    const int* __restrict__ rowptr = a.rowptr;
    const int* __restrict__ colidx = a.colidx;
    const double* __restrict__ kbar = a.kbar;
    const double* __restrict__ mval = a.mval;
    const int* __restrict__ diag = a.diag;
    const double2* __restrict__ sig = a.sig;
    const double2* __restrict__ B = a.B;
    double2* __restrict__ X = a.X;
    double2* __restrict__ work = a.work;
    const long n_pad = a.n_pad;
    const double tol = a.tol;
    const int max_it = a.max_it;
    int* __restrict__ count = a.count;
    int ph = 0;
    const double2 sg = sig[p];
    const double2* b = B + (long)p * n;
    double2* x = X + (long)p * n;
    double2* r = work + ((long)p * 4 + 0) * n_pad;
    double2* pv = work + ((long)p * 4 + 1) * n_pad;
    double2* q = work + ((long)p * 4 + 2) * n_pad;
    double2* dv = work + ((long)p * 4 + 3) * n_pad;
    double v[3] = {0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int d = diag[i];
        const double2 D = make_double2(kbar[d] + sg.x * mval[d], sg.y * mval[d]);
        const double2 di = cdiv(make_double2(1.0, 0.0), D);
        dv[i] = di;
        const double2 ri = b[i];
        const double2 zi = cmul(di, ri);
        r[i] = ri;
        pv[i] = zi;
        x[i] = make_double2(0.0, 0.0);
        const double2 rz = cmul(ri, zi);
        v[0] += rz.x;
        v[1] += rz.y;
        v[2] += ri.x * ri.x + ri.y * ri.y;
    }
    block_sum_d<3>(v, lds, ph);
    double2 rho = make_double2(v[0], v[1]);
    const double bn2 = v[2];
    double rr = bn2;
    const double target2 = tol * tol * bn2;
    int k = 0, status = 0;
    constexpr int G = kRowGroup;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int sub = lane % G, grp = lane / G;
    constexpr int RPW = 64 / G;
    while (rr > target2 && k < max_it) {
        // q = (Kbar + sigma M) p ;  mu = p^T q
        double m2[2] = {0.0, 0.0};
        for (int base = wave * RPW; base < n; base += nw * RPW) {
            const int i = base + grp;
            double ax = 0.0, ay = 0.0, bx = 0.0, by = 0.0;
            if (i < n) {
                const int k1 = rowptr[i + 1];
                for (int kk = rowptr[i] + sub; kk < k1; kk += G) {
                    const double2 pc = pv[colidx[kk]];
                    const double kv = kbar[kk], mv = mval[kk];
                    ax += kv * pc.x;
                    ay += kv * pc.y;
                    bx += mv * pc.x;
                    by += mv * pc.y;
                }
            }
#pragma unroll
            for (int off = G / 2; off > 0; off >>= 1) {
                ax += __shfl_xor(ax, off);
                ay += __shfl_xor(ay, off);
                bx += __shfl_xor(bx, off);
                by += __shfl_xor(by, off);
            }
            if (i < n && sub == 0) {
                const double2 qi = make_double2(ax + sg.x * bx - sg.y * by, ay + sg.x * by + sg.y * bx);
                q[i] = qi;
                const double2 pq = cmul(pv[i], qi);
                m2[0] += pq.x;
                m2[1] += pq.y;
            }
        }
        block_sum_d<2>(m2, lds, ph);
        const double2 mu = make_double2(m2[0], m2[1]);
        if (mu.x == 0.0 && mu.y == 0.0) { status = PPC_ERR_BREAKDOWN; break; }
        const double2 alpha = cdiv(rho, mu);
        double v2[3] = {0.0, 0.0, 0.0};
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const double2 pi = pv[i], qi = q[i];
            const double2 ap = cmul(alpha, pi), aq = cmul(alpha, qi);
            double2 xi = x[i];
            xi.x += ap.x;
            xi.y += ap.y;
            x[i] = xi;
            double2 ri = r[i];
            ri.x -= aq.x;
            ri.y -= aq.y;
            r[i] = ri;
            const double2 rz = cmul(ri, cmul(dv[i], ri));
            v2[0] += rz.x;
            v2[1] += rz.y;
            v2[2] += ri.x * ri.x + ri.y * ri.y;
        }
        block_sum_d<3>(v2, lds, ph);
        const double2 rho_new = make_double2(v2[0], v2[1]);
        rr = v2[2];
        ++k;
        if (rr <= target2) break;
        if (rho_new.x == 0.0 && rho_new.y == 0.0) { status = PPC_ERR_BREAKDOWN; break; }
        if (!isfinite(rr)) { status = PPC_ERR_NONFINITE; break; }
        const double2 beta = cdiv(rho_new, rho);
        rho = rho_new;
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const double2 zi = cmul(dv[i], r[i]);
            const double2 bp = cmul(beta, pv[i]);
            pv[i] = make_double2(zi.x + bp.x, zi.y + bp.y);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        count[4 * p + 0] = status;
        count[4 * p + 1] = k;
        count[4 * p + 2] = (rr <= target2) ? 1 : 0;
    }
}

// (Kbar, M) pairs in ELL order: position v takes CSR slot vslot[v] (padding: 0)
__global__ void k_km(int nvals, const int* __restrict__ vslot, const double* __restrict__ kbar,
                     const double* __restrict__ mval, double2* __restrict__ km) {
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < nvals; v += gridDim.x * blockDim.x) {
        const int s = vslot[v];
        km[v] = s >= 0 ? make_double2(kbar[s], mval[s]) : make_double2(0.0, 0.0);
    }
}

// One workgroup per harmonic p: (Kbar + sigma_p M) x = b by Jacobi-preconditioned COCG
// over the ELL pattern, for meshes whose search direction fits LDS.  p lives in LDS; the
// row values q = A p and z = D^{-1} r stay in registers between the passes that use
// them (rows tid + k B, k < R); x, r and D^{-1} live in memory.  The SpMV streams one
// 16-byte (Kbar, M) pair and one 16-bit column per position (raw buffer loads: rows >= n
// load nothing, slots past the arrays read zero) and gathers p from LDS.  A single tail
// row of at most B entries is spread over all threads and reduced with p^T q; longer or
// several tail rows take one wave each (q in LDS after p).
template <int R>
__device__ __forceinline__ void cocg_ell_body(const CocgArgs& a, const int hp, double2* p_l, double* lds) {
    constexpr int B = kCocgBlock;
    const int tid = threadIdx.x, n = a.n;
    const int lane = tid & 63, wave = tid >> 6, nw = B >> 6;
    const long NP = a.ell_pad;
    const int W = a.W;
    double2* tq_l = p_l + a.n_pad;
    const double2 sg = a.sig[hp];
    const double2* b = a.B + (long)hp * n;
    double2* x = a.X + (long)hp * n;
    double2* r = a.work + ((long)hp * 4 + 0) * a.n_pad;
    double2* dv = a.work + ((long)hp * 4 + 3) * a.n_pad;
    // x, r, D^{-1} through buffer resources: one lane offset per row, no per-row addresses
    const __amdgpu_buffer_rsrc_t bx = buffer_rsrc(x, (unsigned)(n * sizeof(double2)));
    const __amdgpu_buffer_rsrc_t br = buffer_rsrc(r, (unsigned)(n * sizeof(double2)));
    const __amdgpu_buffer_rsrc_t bd = buffer_rsrc(dv, (unsigned)(n * sizeof(double2)));
    const __amdgpu_buffer_rsrc_t rk = buffer_rsrc(a.km, (unsigned)(W * NP * sizeof(double2)));
    const __amdgpu_buffer_rsrc_t rc = buffer_rsrc(a.ecol16, (unsigned)(W * NP * 2));
    const bool tail1 = a.ntail == 1 && a.tail_ptr[1] - a.tail_ptr[0] <= B;
    const int t_beg = tail1 ? a.tail_ptr[0] : 0;
    const int t_len = tail1 ? a.tail_ptr[1] - t_beg : 0;
    const int t_row = tail1 ? a.tail_row[0] : 0;
    const __amdgpu_buffer_rsrc_t rtk = buffer_rsrc(a.km + W * NP + t_beg, (unsigned)(t_len * sizeof(double2)));
    const __amdgpu_buffer_rsrc_t rtc = buffer_rsrc(a.tail_col + t_beg, (unsigned)(t_len * 4));
    int ph = 0;
    unsigned tailmask = 0;
    double2 z[R], q[R];
    double v[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int i = tid + k * B;
        z[k] = make_double2(0.0, 0.0);
        if (i < n) {
            const double2 kd = a.km[a.dpos[i]];
            const double2 di = cdiv(make_double2(1.0, 0.0), make_double2(kd.x + sg.x * kd.y, sg.y * kd.y));
            buffer_store16(bd, (unsigned)i * 16u, di);
            const double2 ri = b[i];
            const double2 zi = cmul(di, ri);
            buffer_store16(br, (unsigned)i * 16u, ri);
            p_l[i] = zi;
            buffer_store16(bx, (unsigned)i * 16u, make_double2(0.0, 0.0));
            const double2 rz = cmul(ri, zi);
            v[0] += rz.x;
            v[1] += rz.y;
            v[2] += ri.x * ri.x + ri.y * ri.y;
            if (a.ecol[i] < 0) tailmask |= 1u << k;
        }
    }
    block_sum<double, 3, B / 64>(v, lds, ph);
    double2 rho = make_double2(v[0], v[1]);
    const double bn2 = v[2];
    double rr = bn2;
    const double target2 = a.tol * a.tol * bn2;
    int it = 0, status = 0;
    while (rr > target2 && it < a.max_it) {
        // this thread's tail entry: loads first, used after the ELL rounds
        const double2 tkv = buffer_load<double2>(rtk, tid < t_len ? tid * 16u : kBufferNone);
        const unsigned tcol = (unsigned)__builtin_amdgcn_raw_buffer_load_b32(rtc, tid < t_len ? tid * 4u : kBufferNone, 0, 0);
        // q = (Kbar + sigma M) p in rounds of 4 complex loads: U slots x KC row groups
        // (KC divides R: 4, 3, 2 or 1 row groups per round, U = 4 / KC slots)
        constexpr int KC = R % 4 == 0 ? 4 : (R % 3 == 0 ? 3 : (R % 2 == 0 ? 2 : 1));
        constexpr int U = 4 / KC;
#pragma unroll
        for (int k = 0; k < R; ++k) q[k] = make_double2(0.0, 0.0);
        for (int w0 = 0; w0 < W; w0 += U) {
#pragma unroll
            for (int kc = 0; kc < R; kc += KC) {
                double2 kv[U][KC], pg[U][KC];
                unsigned col[U][KC];
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int kk = 0; kk < KC; ++kk) {
                        const int i = tid + (kc + kk) * B;
                        const unsigned e = (unsigned)((w0 + u) * NP + i);
                        kv[u][kk] = buffer_load<double2>(rk, i < n ? e * 16u : kBufferNone);
                        col[u][kk] = __builtin_amdgcn_raw_buffer_load_b16(rc, i < n ? e * 2u : kBufferNone, 0, 0);
                    }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int kk = 0; kk < KC; ++kk) pg[u][kk] = p_l[col[u][kk]];
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int kk = 0; kk < KC; ++kk) {
                        // coefficient Kbar + sigma M of the position, times p
                        const double cr = kv[u][kk].x + sg.x * kv[u][kk].y, ci = sg.y * kv[u][kk].y;
                        q[kc + kk].x += cr * pg[u][kk].x - ci * pg[u][kk].y;
                        q[kc + kk].y += cr * pg[u][kk].y + ci * pg[u][kk].x;
                    }
            }
        }
        double m4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int i = tid + k * B;
            if (i < n && !((tailmask >> k) & 1u)) {
                const double2 pq = cmul(p_l[i], q[k]);
                m4[0] += pq.x;
                m4[1] += pq.y;
            }
        }
        if (tail1) {
            const double2 coef = make_double2(tkv.x + sg.x * tkv.y, sg.y * tkv.y);
            const double2 cv = cmul(coef, p_l[tcol]);
            m4[2] = cv.x;
            m4[3] = cv.y;
            const double2 pq = cmul(p_l[t_row], cv);
            m4[0] += pq.x;
            m4[1] += pq.y;
        } else {
            const long base = (long)W * NP;
            for (int t = wave; t < a.ntail; t += nw) {
                double ax = 0.0, ay = 0.0;
                const int j1 = a.tail_ptr[t + 1];
                for (int j = a.tail_ptr[t] + lane; j < j1; j += 64) {
                    const double2 kk = a.km[base + j];
                    const double2 pc = p_l[a.tail_col[j]];
                    const double cr = kk.x + sg.x * kk.y, ci = sg.y * kk.y;
                    ax += cr * pc.x - ci * pc.y;
                    ay += cr * pc.y + ci * pc.x;
                }
                ax = wave_sum(ax);
                ay = wave_sum(ay);
                if (lane == 0) {
                    const double2 qt = make_double2(ax, ay);
                    tq_l[t] = qt;
                    const double2 pq = cmul(p_l[a.tail_row[t]], qt);
                    m4[0] += pq.x;
                    m4[1] += pq.y;
                }
            }
        }
        block_sum<double, 4, B / 64>(m4, lds, ph);
        const double2 mu = make_double2(m4[0], m4[1]);
        if (mu.x == 0.0 && mu.y == 0.0) { status = PPC_ERR_BREAKDOWN; break; }
        const double2 alpha = cdiv(rho, mu);
        double v2[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int i = tid + k * B;
            if (i < n) {
                double2 qi = q[k];
                if ((tailmask >> k) & 1u) {
                    if (tail1) {
                        qi = make_double2(m4[2], m4[3]);
                    } else {
                        for (int t = 0; t < a.ntail; ++t)
                            if (a.tail_row[t] == i) qi = tq_l[t];
                    }
                }
                const unsigned off = (unsigned)i * 16u;
                const double2 pi = p_l[i];
                const double2 ap = cmul(alpha, pi), aq = cmul(alpha, qi);
                double2 xi = buffer_load<double2>(bx, off);
                double2 ri = buffer_load<double2>(br, off);
                const double2 di = buffer_load<double2>(bd, off);
                xi.x += ap.x;
                xi.y += ap.y;
                buffer_store16(bx, off, xi);
                ri.x -= aq.x;
                ri.y -= aq.y;
                buffer_store16(br, off, ri);
                z[k] = cmul(di, ri);
                const double2 rz = cmul(ri, z[k]);
                v2[0] += rz.x;
                v2[1] += rz.y;
                v2[2] += ri.x * ri.x + ri.y * ri.y;
            }
        }
        block_sum<double, 3, B / 64>(v2, lds, ph);
        const double2 rho_new = make_double2(v2[0], v2[1]);
        rr = v2[2];
        ++it;
        if (rr <= target2) break;
        if (rho_new.x == 0.0 && rho_new.y == 0.0) { status = PPC_ERR_BREAKDOWN; break; }
        if (!isfinite(rr)) { status = PPC_ERR_NONFINITE; break; }
        const double2 beta = cdiv(rho_new, rho);
        rho = rho_new;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int i = tid + k * B;
            if (i < n) {
                const double2 bp = cmul(beta, p_l[i]);
                p_l[i] = make_double2(z[k].x + bp.x, z[k].y + bp.y);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        a.count[4 * hp + 0] = status;
        a.count[4 * hp + 1] = it;
        a.count[4 * hp + 2] = (rr <= target2) ? 1 : 0;
        a.count[4 * hp + 3] = 0;
    }
}

template <int R>
__global__ __launch_bounds__(kCocgBlock) void k_cocg_ell(CocgArgs a) {
    extern __shared__ double2 p_l[];
    __shared__ double lds[2 * 16 * 4];
    cocg_ell_body<R>(a, blockIdx.x, p_l, lds);
}

// Batched designs of one ELL shape: block b solves harmonic work[b].y of design work[b].x.
template <int R>
__global__ __launch_bounds__(kCocgBlock) void k_cocg_ell_batch(const CocgArgs* __restrict__ args,
                                                               const int2* __restrict__ work) {
    extern __shared__ double2 p_l[];
    __shared__ double lds[2 * 16 * 4];
    const int2 wk = work[blockIdx.x];
    cocg_ell_body<R>(args[wk.x], wk.y, p_l, lds);
}

__device__ inline float2 cmulf(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Complex-FP32 COCG refined to FP64: x = 0; repeat r = b - A x (FP64); stop when
// ||r|| <= tol ||b||; solve A d = r in complex FP32 (FP32 K, M copies, FP32 vectors and
// accumulation) to kInnerTol relative; x += d.
__device__ __forceinline__ void cocg_mixed_body(const CocgArgs& a, const int p, double* lds) {
    constexpr double kInnerTol = 1e-5;
    constexpr int kMaxRefine = 30;
    const int n = a.n;
    const double2 sg = a.sig[p];
    const float2 sgf = make_float2((float)sg.x, (float)sg.y);
    const double2* __restrict__ b = a.B + (long)p * n;
    double2* __restrict__ x = a.X + (long)p * n;
    double2* wk = a.work + (long)p * 4 * a.n_pad;               // 4 * n_pad double2 of room
    double2* rd = wk;                                          // FP64 residual
    float2* rf = reinterpret_cast<float2*>(wk + a.n_pad);      // FP32 r, p, q, dinv, d
    float2* pf = rf + a.n_pad;
    float2* qf = pf + a.n_pad;
    float2* df = qf + a.n_pad;
    float2* xf = df + a.n_pad;
    int ph = 0;
    constexpr int G = kRowGroup;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int sub = lane % G, grp = lane / G;
    constexpr int RPW = 64 / G;
    double v0[1] = {0.0};
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double2 bi = b[i];
        x[i] = make_double2(0.0, 0.0);
        rd[i] = bi;
        v0[0] += bi.x * bi.x + bi.y * bi.y;
        const int dd = a.diag[i];
        const double2 D = make_double2(a.kbar[dd] + sg.x * a.mval[dd], sg.y * a.mval[dd]);
        const double2 di = cdiv(make_double2(1.0, 0.0), D);
        df[i] = make_float2((float)di.x, (float)di.y);
    }
    block_sum_d<1>(v0, lds, ph);
    const double bn2 = v0[0];
    double rr = bn2;
    int total = 0, status = 0, refine = 0;
    while (rr > a.tol * a.tol * bn2 && refine < kMaxRefine && total < a.max_it && status == 0) {
        ++refine;
        // inner complex-FP32 COCG on A d = r / ||r|| (unit right-hand side: FP32 keeps its
        // range whatever the harmonic's magnitude), then x += ||r|| d
        const double rs = 1.0 / sqrt(rr);
        double v[3] = {0.0, 0.0, 0.0};
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const double2 r64 = rd[i];
            const float2 ri = make_float2((float)(r64.x * rs), (float)(r64.y * rs));
            const float2 zi = cmulf(df[i], ri);
            rf[i] = ri;
            pf[i] = zi;
            xf[i] = make_float2(0.f, 0.f);
            const float2 rz = cmulf(ri, zi);
            v[0] += rz.x;
            v[1] += rz.y;
            v[2] += (double)(ri.x * ri.x + ri.y * ri.y);
        }
        block_sum_d<3>(v, lds, ph);
        float2 rho = make_float2((float)v[0], (float)v[1]);
        const double in2 = v[2];
        double irr = in2, best = in2;
        // the iterations left are shared among the refinements left, so that an inner solve
        // that FP32 cannot finish (ill-conditioned harmonics) leaves room for the next one
        const int inner_end = total + max(1, (a.max_it - total) / (kMaxRefine - refine + 1));
        while (irr > kInnerTol * kInnerTol * in2 && total < inner_end) {
            double m2[2] = {0.0, 0.0};
            for (int base = wave * RPW; base < n; base += nw * RPW) {
                const int i = base + grp;
                float ax = 0.f, ay = 0.f, bx = 0.f, by = 0.f;
                if (i < n) {
                    const int k1 = a.rowptr[i + 1];
                    for (int kk = a.rowptr[i] + sub; kk < k1; kk += G) {
                        const float2 pc = pf[a.colidx[kk]];
                        const float kv = a.kbar32[kk], mv = a.mval32[kk];
                        ax += kv * pc.x;
                        ay += kv * pc.y;
                        bx += mv * pc.x;
                        by += mv * pc.y;
                    }
                }
#pragma unroll
                for (int off = G / 2; off > 0; off >>= 1) {
                    ax += __shfl_xor(ax, off);
                    ay += __shfl_xor(ay, off);
                    bx += __shfl_xor(bx, off);
                    by += __shfl_xor(by, off);
                }
                if (i < n && sub == 0) {
                    const float2 qi = make_float2(ax + sgf.x * bx - sgf.y * by, ay + sgf.x * by + sgf.y * bx);
                    qf[i] = qi;
                    const float2 pq = cmulf(pf[i], qi);
                    m2[0] += pq.x;
                    m2[1] += pq.y;
                }
            }
            block_sum_d<2>(m2, lds, ph);
            const double2 mu = make_double2(m2[0], m2[1]);
            if (mu.x == 0.0 && mu.y == 0.0) { status = PPC_ERR_BREAKDOWN; break; }
            const double2 al = cdiv(make_double2(rho.x, rho.y), mu);
            const float2 alpha = make_float2((float)al.x, (float)al.y);
            double v2[3] = {0.0, 0.0, 0.0};
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                const float2 ap = cmulf(alpha, pf[i]), aq = cmulf(alpha, qf[i]);
                float2 xi = xf[i];
                xi.x += ap.x;
                xi.y += ap.y;
                xf[i] = xi;
                float2 ri = rf[i];
                ri.x -= aq.x;
                ri.y -= aq.y;
                rf[i] = ri;
                const float2 rz = cmulf(ri, cmulf(df[i], ri));
                v2[0] += rz.x;
                v2[1] += rz.y;
                v2[2] += (double)(ri.x * ri.x + ri.y * ri.y);
            }
            block_sum_d<3>(v2, lds, ph);
            ++total;
            irr = v2[2];
            if (irr <= kInnerTol * kInnerTol * in2) break;
            if (v2[0] == 0.0 && v2[1] == 0.0) { status = PPC_ERR_BREAKDOWN; break; }
            if (!isfinite(irr)) { status = PPC_ERR_NONFINITE; break; }
            best = fmin(best, irr);
            if (irr > 1e8 * best) break;          // FP32 recurrence diverging: refine from here
            const double2 be = cdiv(make_double2(v2[0], v2[1]), make_double2(rho.x, rho.y));
            const float2 beta = make_float2((float)be.x, (float)be.y);
            rho = make_float2((float)v2[0], (float)v2[1]);
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                const float2 zi = cmulf(df[i], rf[i]);
                const float2 bp = cmulf(beta, pf[i]);
                pf[i] = make_float2(zi.x + bp.x, zi.y + bp.y);
            }
            __syncthreads();
        }
        // x += ||r|| d ; r = b - A x in FP64.  A refinement that does not lower the FP64
        // residual is taken back (x -= ||r|| d, residual recomputed) and ends the solve: the
        // FP32 inner solves cannot resolve this system any further.
        const double rsc = sqrt(rr);
        bool stop = false;
        double rr_new = rr;
        for (int pass = 0; pass < 2; ++pass) {     // pass 1: take the refinement back
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            double2 xi = x[i];
            xi.x += (pass ? -rsc : rsc) * (double)xf[i].x;
            xi.y += (pass ? -rsc : rsc) * (double)xf[i].y;
            x[i] = xi;
        }
        __syncthreads();
        double v3[1] = {0.0};
        for (int base = wave * RPW; base < n; base += nw * RPW) {
            const int i = base + grp;
            double ax = 0.0, ay = 0.0, bx = 0.0, by = 0.0;
            if (i < n) {
                const int k1 = a.rowptr[i + 1];
                for (int kk = a.rowptr[i] + sub; kk < k1; kk += G) {
                    const double2 xc = x[a.colidx[kk]];
                    const double kv = a.kbar[kk], mv = a.mval[kk];
                    ax += kv * xc.x;
                    ay += kv * xc.y;
                    bx += mv * xc.x;
                    by += mv * xc.y;
                }
            }
#pragma unroll
            for (int off = G / 2; off > 0; off >>= 1) {
                ax += __shfl_xor(ax, off);
                ay += __shfl_xor(ay, off);
                bx += __shfl_xor(bx, off);
                by += __shfl_xor(by, off);
            }
            if (i < n && sub == 0) {
                const double2 bi = b[i];
                const double2 ri = make_double2(bi.x - (ax + sg.x * bx - sg.y * by),
                                                bi.y - (ay + sg.x * by + sg.y * bx));
                rd[i] = ri;
                v3[0] += ri.x * ri.x + ri.y * ri.y;
            }
        }
        block_sum_d<1>(v3, lds, ph);
        rr_new = v3[0];
        if (pass == 0 && rr_new < rr) break;       // progress: the refinement stays
        if (pass == 1) stop = true;
        }
        rr = rr_new;
        if (stop) break;
    }
    if (threadIdx.x == 0) {
        a.count[4 * p + 0] = status;
        a.count[4 * p + 1] = total;
        a.count[4 * p + 2] = (rr <= a.tol * a.tol * bn2) ? 1 : 0;
        a.count[4 * p + 3] = refine;
    }
}

__device__ __forceinline__ void cocg_dispatch(const CocgArgs& a, const int p, double* lds) {
    if (a.mixed) cocg_mixed_body(a, p, lds);
    else cocg_body(a, p, lds);
}

__global__ __launch_bounds__(1024) void k_cocg(CocgArgs a) {
    __shared__ double lds[2 * 16 * 3];
    cocg_dispatch(a, blockIdx.x, lds);
}

// Batched designs: block b solves harmonic work[b].y of design work[b].x.
__global__ __launch_bounds__(1024) void k_cocg_batch(const CocgArgs* __restrict__ args,
                                                     const int2* __restrict__ work) {
    __shared__ double lds[2 * 16 * 3];
    const int2 wk = work[blockIdx.x];
    cocg_dispatch(args[wk.x], wk.y, lds);
}

// sigma_p, p = 0..N/2: exact implicit-Euler symbol (1 - e^{-i w_p dT})/dT or i w_p
__global__ void k_shifts(int N, double T, int mode, double2* __restrict__ sig) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q > N / 2) return;
    const double dT = T / N;
    if (mode == 0) {
        double sn, cs;
        sincospi(2.0 * q / N, &sn, &cs);
        sig[q] = make_double2((1.0 - cs) / dT, sn / dT);
    } else {
        sig[q] = make_double2(0.0, 2.0 * M_PI * q / T);
    }
}

// dU[s][i] = (1/N) [ Re X_0 + (-1)^s Re X_{N/2} + 2 sum_{p=1}^{N/2-1} Re(X_p e^{+2 pi i p s/N}) ]
// written to out (accumulate: out += dU)
__global__ void k_idft(int n, int N, const double2* __restrict__ X, const double2* __restrict__ tw,
                       double* __restrict__ out, int accumulate) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (i >= n) return;
    const int H = N / 2;
    double acc = X[i].x;
    acc += ((s & 1) ? -1.0 : 1.0) * X[(long)H * n + i].x;
    double sum = 0.0;
    for (int p = 1; p < H; ++p) {
        const double2 xp = X[(long)p * n + i];
        const double2 w = tw[(int)(((long)p * s) % N)];   // exp(-i theta); use its conjugate
        sum += xp.x * w.x + xp.y * w.y;                     // Re(x e^{+i theta})
    }
    acc += 2.0 * sum;
    const double du = acc / N;
    const long k = (long)s * n + i;
    if (accumulate) out[k] += du;
    else out[k] = du;
}

__global__ void k_to_nodal(int n, int nn, int N, const int* __restrict__ free_node,
                           const double* __restrict__ Uf, double* __restrict__ Un) {
    const long total = (long)N * nn;
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < total; k += (long)gridDim.x * blockDim.x)
        Un[k] = 0.0;
}

__global__ void k_scatter_free(int n, int nn, int N, const int* __restrict__ free_node,
                               const double* __restrict__ Uf, double* __restrict__ Un) {
    const long total = (long)N * n;
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < total; k += (long)gridDim.x * blockDim.x) {
        const long s = k / n;
        const int i = (int)(k - s * n);
        Un[s * nn + free_node[i]] = Uf[k];
    }
}

__global__ void k_gather_free(int n, int nn, int N, const int* __restrict__ free_node,
                              const double* __restrict__ Un, double* __restrict__ Uf) {
    const long total = (long)N * n;
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < total; k += (long)gridDim.x * blockDim.x) {
        const long s = k / n;
        const int i = (int)(k - s * n);
        Uf[k] = Un[s * nn + free_node[i]];
    }
}

// max |B| over Brauer elements and samples (per-block partial maxima)
__global__ void k_max_b(int ne, int n, int N, const double* __restrict__ U, const int* __restrict__ efree,
                        const double* __restrict__ gx, const double* __restrict__ gy,
                        const int* __restrict__ mat, const double* __restrict__ lawtab,
                        double* __restrict__ part) {
    __shared__ double red[1024];
    double mx = 0.0;
    const long total = (long)N * ne;
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < total; k += (long)gridDim.x * blockDim.x) {
        const long s = k / ne;
        const int e = (int)(k - s * ne);
        if (lawtab[5 * mat[e]] == 0.0) continue;
        double bx = 0.0, by = 0.0;
        for (int q = 0; q < 3; ++q) {
            const int g = efree[q * ne + e];
            const double uv = g >= 0 ? U[s * n + g] : 0.0;
            bx += gx[q * ne + e] * uv;
            by += gy[q * ne + e] * uv;
        }
        mx = fmax(mx, sqrt(bx * bx + by * by));
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Per block: max |B| over the Brauer elements and samples of U and of U + dU (pairs).
__global__ void k_max_b_pair(int ne, int n, int N, const double* __restrict__ U, const double* __restrict__ dU,
                             const int* __restrict__ efree, const double* __restrict__ gx,
                             const double* __restrict__ gy, const int* __restrict__ mat,
                             const double* __restrict__ lawtab, double* __restrict__ part) {
    __shared__ double red[2][256];
    double m0 = 0.0, m1 = 0.0;
    const long total = (long)N * ne;
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < total; k += (long)gridDim.x * blockDim.x) {
        const long s = k / ne;
        const int e = (int)(k - s * ne);
        if (lawtab[5 * mat[e]] == 0.0) continue;
        double ax = 0.0, ay = 0.0, bx = 0.0, by = 0.0;
        for (int q = 0; q < 3; ++q) {
            const int g = efree[q * ne + e];
            const double u0 = g >= 0 ? U[s * n + g] : 0.0;
            const double u1 = g >= 0 ? u0 + dU[s * n + g] : 0.0;
            ax += gx[q * ne + e] * u0;
            ay += gy[q * ne + e] * u0;
            bx += gx[q * ne + e] * u1;
            by += gy[q * ne + e] * u1;
        }
        m0 = fmax(m0, sqrt(ax * ax + ay * ay));
        m1 = fmax(m1, sqrt(bx * bx + by * by));
    }
    red[0][threadIdx.x] = m0;
    red[1][threadIdx.x] = m1;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] = fmax(red[0][threadIdx.x], red[0][threadIdx.x + w]);
            red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = red[0][0];
        part[2 * blockIdx.x + 1] = red[1][0];
    }
}

// Step of the safeguarded correction: with b_U = max |B(U)| and b_new = max |B(U + dU)|
// over the Brauer elements, theta = 1 if b_new <= cap, else (cap - b_U) / (b_new - b_U)
// (so that max |B(U + theta dU)| <= cap, B being linear in u), else 1/2 when U itself is
// beyond the cap.  out = {theta, b_new, b_U}.
__global__ void k_damp_theta(int nb, const double* __restrict__ part, double cap, double* __restrict__ out) {
    if (threadIdx.x == 0) {
        double bu = 0.0, bn = 0.0;
        for (int b = 0; b < nb; ++b) {
            bu = fmax(bu, part[2 * b]);
            bn = fmax(bn, part[2 * b + 1]);
        }
        double theta = 1.0;
        if (!(bn <= cap)) theta = bu < cap ? (cap - bu) / (bn - bu) : 0.5;
        out[0] = theta;
        out[1] = bn;
        out[2] = bu;
    }
}

// U += theta dU with theta read from the device
__global__ void k_axpy_theta(long total, const double* __restrict__ theta, const double* __restrict__ dU,
                             double* __restrict__ U) {
    const double t = theta[0];
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < total; k += (long)gridDim.x * blockDim.x)
        U[k] += t * dU[k];
}

__global__ void k_max_partials(int nb, const double* __restrict__ part, double* __restrict__ out) {
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int b = 0; b < nb; ++b) m = fmax(m, part[b]);
        out[0] = m;
    }
}

// ------------------------------------------------------------------------------------
// host launchers
// ------------------------------------------------------------------------------------
void launch_jumps(ppc_problem* pr, int N, const double* U, const double* F, double* J,
                  double* out3, hipStream_t s) {
    const int n = pr->mesh.n_free;
    const long total = (long)N * n;
    hipLaunchKernelGGL(k_jumps, dim3(kRedBlocks), dim3(256), 0, s, total, n, U, F, J, pr->ws.partial);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, s, kRedBlocks, 3, pr->ws.partial, out3);
    PPC_HIP(hipGetLastError());
}

// Linearisation, coarse right-hand side, DFT along time and the shifts: everything of the
// correction before the harmonic solves.
namespace {

// Frozen coarse stiffness Kbar over the samples U (null: at u = 0), in CSR order (FP64 and
// FP32) and as (Kbar, M) pairs in ELL order.
void launch_linearisation(ppc_problem* pr, const ppc_params* p, const double* U, hipStream_t s) {
    const DeviceMesh& d = pr->mesh;
    Workspace& w = pr->ws;
    const int n = d.n_free, ne = d.n_tri;
    const int eb = 256;
    const int eg = std::max(1, std::min((ne + eb - 1) / eb, 4096));
    hipLaunchKernelGGL(k_linearise, dim3(eg), dim3(eb), 0, s, ne, n, p->N, U, d.efree, d.gx, d.gy, d.area,
                       d.k0, d.mat, pr->lawtab, p->lin_mode, w.nubar);
    const int sg = std::max(1, std::min((d.nnz + eb - 1) / eb, 4096));
    hipLaunchKernelGGL(k_kbar, dim3(sg), dim3(eb), 0, s, d.nnz, ne, d.slot_ptr, d.slot_src, d.area, d.gx,
                       d.gy, w.nubar, w.kbar, w.kbar32);
    const int vg = std::max(1, std::min((d.n_vals + eb - 1) / eb, 4096));
    hipLaunchKernelGGL(k_km, dim3(vg), dim3(eb), 0, s, d.n_vals, d.vslot, w.kbar, d.mval, w.ckm);
}

}  // namespace

void launch_coarse_pre(ppc_problem* pr, const ppc_params* p, const double* U, const double* J,
                       bool excitation_rhs, hipStream_t s) {
    const DeviceMesh& d = pr->mesh;
    Workspace& w = pr->ws;
    const int n = d.n_free, N = p->N, H = N / 2 + 1;
    const double dT = p->T / N;
    launch_linearisation(pr, p, excitation_rhs ? nullptr : U, s);
    const dim3 rg((n + 255) / 256, N);
    if (excitation_rhs)
        hipLaunchKernelGGL(k_excitation_rows, rg, dim3(256), 0, s, n, N, p->T, d.fload, pr->wavtab,
                           pr->wave.n_h, pr->wave.f0, w.R);
    else
        hipLaunchKernelGGL(k_coarse_rhs, rg, dim3(256), 0, s, n, N, d.rowptr, d.colidx, d.mval, w.kbar,
                           1.0 / dT, J, w.R);
    hipLaunchKernelGGL(k_twiddle, dim3((N + 255) / 256), dim3(256), 0, s, N, w.twiddle);
    const int Hs = solved_harmonics(p, excitation_rhs);
    hipLaunchKernelGGL(k_dft, dim3((n + 255) / 256, Hs), dim3(256), 0, s, n, N, 0, w.R, w.twiddle, w.rhat);
    // truncated harmonic set: the unsolved harmonics of the correction are those of the jumps,
    // written straight into the solution block
    if (Hs < H)
        hipLaunchKernelGGL(k_dft, dim3((n + 255) / 256, H - Hs), dim3(256), 0, s, n, N, Hs, J, w.twiddle,
                           w.rhat + (long)H * n);
    hipLaunchKernelGGL(k_shifts, dim3((H + 63) / 64), dim3(64), 0, s, N, p->T, p->shift_mode, w.sig);
    PPC_HIP(hipGetLastError());
}

CocgArgs make_cocg_args(ppc_problem* pr, const ppc_params* p) {
    const DeviceMesh& d = pr->mesh;
    Workspace& w = pr->ws;
    const int H = p->N / 2 + 1;
    CocgArgs a{};
    a.n = d.n_free;
    a.H = solved_harmonics(p, false);    // the solution block still holds all H harmonics
    a.rowptr = d.rowptr;
    a.colidx = d.colidx;
    a.kbar = w.kbar;
    a.mval = d.mval;
    a.diag = d.diag;
    a.sig = w.sig;
    a.B = w.rhat;
    a.X = w.rhat + (long)H * d.n_free;   // solution block follows the right-hand sides
    a.work = w.cwork;
    a.n_pad = (long)w.n_pad;
    a.tol = p->tol_cocg;
    a.max_it = p->max_cocg;
    a.count = w.ccount;
    a.mixed = (p->coarse_precision < 0 ? p->precision : p->coarse_precision) == 1 ? 1 : 0;
    a.kbar32 = w.kbar32;
    a.mval32 = d.mval32;
    a.km = w.ckm;
    a.ecol16 = d.ecol16;
    a.ecol = d.ecol;
    a.dpos = d.dpos;
    a.ell_pad = (long)d.ell_pad;
    a.W = d.ell_w;
    a.ntail = d.n_tail;
    a.tail_row = d.tail_row;
    a.tail_ptr = d.tail_ptr;
    a.tail_col = d.tail_col;
    return a;
}

namespace {

// Rows per thread of the ELL COCG for this problem (0: use the CSR form): FP64 solves of
// meshes with 16-bit columns whose search direction (and tail sums) fit LDS.
int cocg_ell_rows(const ppc_problem* pr, const CocgArgs& a, size_t& lds) {
    const DeviceMesh& d = pr->mesh;
    if (a.mixed || !d.ecol16) return 0;
    lds = (pr->ws.n_pad + (size_t)std::max(d.n_tail, 1)) * sizeof(double2);
    if (lds > kLdsBudget) return 0;
    for (int R : {1, 2, 3, 4, 5, 6, 7, 8, 12})
        if ((long)R * kCocgBlock >= d.n_free) return R;
    return 0;
}

template <int R>
void launch_cocg_ell(const CocgArgs& a, size_t lds, hipStream_t s) {
    static bool attr_set = false;
    if (!attr_set) {
        PPC_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_cocg_ell<R>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBudget));
        attr_set = true;
    }
    hipLaunchKernelGGL(k_cocg_ell<R>, dim3(a.H), dim3(kCocgBlock), lds, s, a);
}

template <int R>
void launch_cocg_ell_batch(const CocgArgs* d_args, const int2* d_work, int nblocks, size_t lds,
                           hipStream_t s) {
    static bool attr_set = false;
    if (!attr_set) {
        PPC_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_cocg_ell_batch<R>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBudget));
        attr_set = true;
    }
    hipLaunchKernelGGL(k_cocg_ell_batch<R>, dim3(nblocks), dim3(kCocgBlock), lds, s, d_args, d_work);
}

}  // namespace

// Inverse DFT of the harmonic solutions into dU (accumulate: U += dU).
void launch_coarse_post(ppc_problem* pr, const ppc_params* p, double* dU, bool accumulate,
                        hipStream_t s) {
    const DeviceMesh& d = pr->mesh;
    Workspace& w = pr->ws;
    const int n = d.n_free, N = p->N, H = N / 2 + 1;
    const double2* X = w.rhat + (long)H * n;
    hipLaunchKernelGGL(k_idft, dim3((n + 255) / 256, N), dim3(256), 0, s, n, N, X, w.twiddle, dU,
                       accumulate ? 1 : 0);
    PPC_HIP(hipGetLastError());
}

namespace {

// One COCG launch over the a.H systems of a (one workgroup each), in the form the mesh takes.
void launch_cocg_solves(const ppc_problem* pr, const CocgArgs& a, hipStream_t s) {
    size_t lds = 0;
    switch (cocg_ell_rows(pr, a, lds)) {
        case 1: launch_cocg_ell<1>(a, lds, s); break;
        case 2: launch_cocg_ell<2>(a, lds, s); break;
        case 3: launch_cocg_ell<3>(a, lds, s); break;
        case 4: launch_cocg_ell<4>(a, lds, s); break;
        case 5: launch_cocg_ell<5>(a, lds, s); break;
        case 6: launch_cocg_ell<6>(a, lds, s); break;
        case 7: launch_cocg_ell<7>(a, lds, s); break;
        case 8: launch_cocg_ell<8>(a, lds, s); break;
        case 12: launch_cocg_ell<12>(a, lds, s); break;
        default: hipLaunchKernelGGL(k_cocg, dim3(a.H), dim3(kCocgBlock), 0, s, a);
    }
    PPC_HIP(hipGetLastError());
}

}  // namespace

void launch_coarse(ppc_problem* pr, const ppc_params* p, const double* U, const double* J,
                   double* dU, bool accumulate, bool excitation_rhs, hipStream_t s) {
    launch_coarse_pre(pr, p, U, J, excitation_rhs, s);
    CocgArgs a = make_cocg_args(pr, p);
    a.H = solved_harmonics(p, excitation_rhs);
    launch_cocg_solves(pr, a, s);
    launch_coarse_post(pr, p, dU, accumulate, s);
}

void launch_coarse_setup(ppc_problem* pr, const ppc_params* p, const double* Ulin, hipStream_t s) {
    const int N = p->N, H = N / 2 + 1;
    launch_linearisation(pr, p, Ulin, s);
    hipLaunchKernelGGL(k_twiddle, dim3((N + 255) / 256), dim3(256), 0, s, N, pr->ws.twiddle);
    hipLaunchKernelGGL(k_shifts, dim3((H + 63) / 64), dim3(64), 0, s, N, p->T, p->shift_mode, pr->ws.sig);
    PPC_HIP(hipGetLastError());
}

void launch_coarse_apply(ppc_problem* pr, const ppc_params* p, const double* r, double* z, hipStream_t s) {
    const int n = pr->mesh.n_free, N = p->N, H = N / 2 + 1;
    hipLaunchKernelGGL(k_dft, dim3((n + 255) / 256, H), dim3(256), 0, s, n, N, 0, r, pr->ws.twiddle, pr->ws.rhat);
    CocgArgs a = make_cocg_args(pr, p);
    a.H = H;
    launch_cocg_solves(pr, a, s);
    launch_coarse_post(pr, p, z, false, s);
}

void launch_ic_propagation(ppc_problem* pr, const ppc_params* p, hipStream_t s) {
    const DeviceMesh& d = pr->mesh;
    Workspace& w = pr->ws;
    const int n = d.n_free, N = p->N;
    const double inv_dT = N / p->T;
    launch_linearisation(pr, p, w.U, s);
    const dim3 g((n + 255) / 256), b(256);
    hipLaunchKernelGGL(k_ic_start, g, b, 0, s, n, inv_dT, w.ic_un, w.U, w.ic_e, w.sig);
    // one real shifted system (Kbar + M/dT) x = C e per step: the harmonic solver with a
    // single system and the real shift 1/dT, right-hand side in rhat[0], solution in rhat[1]
    CocgArgs a = make_cocg_args(pr, p);
    a.H = 1;
    a.X = w.rhat + n;
    for (int step = 1; step <= N; ++step) {
        hipLaunchKernelGGL(k_ic_rhs, g, b, 0, s, n, d.rowptr, d.colidx, d.mval, inv_dT, w.ic_e, w.rhat);
        a.count = w.ccount + 4 * (step - 1);
        launch_cocg_solves(pr, a, s);
        const int row = step % N;
        hipLaunchKernelGGL(k_ic_update, g, b, 0, s, n, w.rhat + n, w.F + (long)row * n,
                           step < N ? w.U + (long)step * n : nullptr, w.ic_e, w.ic_un);
    }
    PPC_HIP(hipGetLastError());
}

// Harmonic solves of the designs in list (descriptors d_args, one per design): the
// (design, harmonic) work items are grouped by the designs' COCG form (as the single-
// design launch picks it, so a design's arithmetic does not depend on its batch) and
// each group is one launch.  The plan uploads the work list and synchronises.
void cocg_batch_plan(const std::vector<ppc_problem*>& parts, const std::vector<int>& list, const ppc_params* p,
                     int H, int2* d_work, CocgBatchPlan& plan, hipStream_t s) {
    plan.spans.clear();
    plan.cw.clear();
    for (int R : {0, 1, 2, 3, 4, 5, 6, 7, 8, 12}) {
        CocgBatchPlan::Span sp{R, 0, (int)plan.cw.size(), 0};
        for (int d : list) {
            const CocgArgs a = make_cocg_args(parts[d], p);
            size_t lds = 0;
            if (cocg_ell_rows(parts[d], a, lds) != R) continue;
            sp.lds = std::max(sp.lds, lds);
            for (int q = 0; q < H; ++q) plan.cw.push_back(make_int2(d, q));
        }
        sp.count = (int)plan.cw.size() - sp.begin;
        if (sp.count > 0) plan.spans.push_back(sp);
    }
    if (plan.cw.empty()) return;
    PPC_HIP(hipMemcpyAsync(d_work, plan.cw.data(), sizeof(int2) * plan.cw.size(), hipMemcpyHostToDevice, s));
    PPC_HIP(hipStreamSynchronize(s));
}

Lanes::Lanes(ppc_handle* h_, hipStream_t s_) : h(h_), s(s_) {
    if (h) PPC_HIP(hipEventRecord(h->fork, s));
}

hipStream_t Lanes::lane(int i) {
    const int l = h ? i % (1 + ppc_handle::kSide) : 0;
    if (l == 0) return s;
    if (!used[l - 1]) {
        PPC_HIP(hipStreamWaitEvent(h->side[l - 1], h->fork, 0));
        used[l - 1] = true;
    }
    return h->side[l - 1];
}

void Lanes::join() {
    for (int i = 0; i < ppc_handle::kSide; ++i)
        if (used[i]) {
            PPC_HIP(hipEventRecord(h->join[i], h->side[i]));
            PPC_HIP(hipStreamWaitEvent(s, h->join[i], 0));
            used[i] = false;
        }
}

// One launch per COCG form; with a handle the forms run side by side on its lanes.
void cocg_batch_run(const CocgBatchPlan& plan, const CocgArgs* d_args, const int2* d_work, hipStream_t s,
                    ppc_handle* h) {
    Lanes lanes(plan.spans.size() > 1 ? h : nullptr, s);
    for (size_t g = 0; g < plan.spans.size(); ++g) {
        const auto& sp = plan.spans[g];
        const int2* w = d_work + sp.begin;
        hipStream_t sg = lanes.lane((int)g);
        switch (sp.R) {
            case 1: launch_cocg_ell_batch<1>(d_args, w, sp.count, sp.lds, sg); break;
            case 2: launch_cocg_ell_batch<2>(d_args, w, sp.count, sp.lds, sg); break;
            case 3: launch_cocg_ell_batch<3>(d_args, w, sp.count, sp.lds, sg); break;
            case 4: launch_cocg_ell_batch<4>(d_args, w, sp.count, sp.lds, sg); break;
            case 5: launch_cocg_ell_batch<5>(d_args, w, sp.count, sp.lds, sg); break;
            case 6: launch_cocg_ell_batch<6>(d_args, w, sp.count, sp.lds, sg); break;
            case 7: launch_cocg_ell_batch<7>(d_args, w, sp.count, sp.lds, sg); break;
            case 8: launch_cocg_ell_batch<8>(d_args, w, sp.count, sp.lds, sg); break;
            case 12: launch_cocg_ell_batch<12>(d_args, w, sp.count, sp.lds, sg); break;
            default: hipLaunchKernelGGL(k_cocg_batch, dim3(sp.count), dim3(kCocgBlock), 0, sg, d_args, w);
        }
    }
    lanes.join();
    PPC_HIP(hipGetLastError());
}

void launch_cocg_batch(const std::vector<ppc_problem*>& parts, const std::vector<int>& list,
                       const ppc_params* p, int H, const CocgArgs* d_args, int2* d_work, std::vector<int2>& cw,
                       hipStream_t s) {
    CocgBatchPlan plan;
    cocg_batch_plan(parts, list, p, H, d_work, plan, s);
    cocg_batch_run(plan, d_args, d_work, s);
    cw = plan.cw;
}

void launch_to_nodal(const ppc_problem* pr, int N, const double* Ufree, double* Unodal,
                     hipStream_t s) {
    const DeviceMesh& d = pr->mesh;
    hipLaunchKernelGGL(k_to_nodal, dim3(1024), dim3(256), 0, s, d.n_free, d.n_nodes, N, d.free_node,
                       Ufree, Unodal);
    hipLaunchKernelGGL(k_scatter_free, dim3(1024), dim3(256), 0, s, d.n_free, d.n_nodes, N, d.free_node,
                       Ufree, Unodal);
    PPC_HIP(hipGetLastError());
}

void launch_to_free(const ppc_problem* pr, int N, const double* Unodal, double* Ufree,
                    hipStream_t s) {
    const DeviceMesh& d = pr->mesh;
    hipLaunchKernelGGL(k_gather_free, dim3(1024), dim3(256), 0, s, d.n_free, d.n_nodes, N, d.free_node,
                       Unodal, Ufree);
    PPC_HIP(hipGetLastError());
}

// U += theta dU with the safeguard step of k_damp_theta; out3 = {theta, b_new, b_U}.
void launch_safeguarded_update(ppc_problem* pr, int N, double cap, const double* dU, double* U,
                               double* out3, hipStream_t s) {
    const DeviceMesh& d = pr->mesh;
    hipLaunchKernelGGL(k_max_b_pair, dim3(kRedBlocks), dim3(256), 0, s, d.n_tri, d.n_free, N, U, dU, d.efree,
                       d.gx, d.gy, d.mat, pr->lawtab, pr->ws.partial);
    hipLaunchKernelGGL(k_damp_theta, dim3(1), dim3(64), 0, s, kRedBlocks, pr->ws.partial, cap, out3);
    const long total = (long)N * d.n_free;
    hipLaunchKernelGGL(k_axpy_theta, dim3(1024), dim3(256), 0, s, total, out3, dU, U);
    PPC_HIP(hipGetLastError());
}

void launch_max_b(ppc_problem* pr, int N, const double* U, double* out, hipStream_t s) {
    const DeviceMesh& d = pr->mesh;
    hipLaunchKernelGGL(k_max_b, dim3(kRedBlocks), dim3(256), 0, s, d.n_tri, d.n_free, N, U, d.efree, d.gx,
                       d.gy, d.mat, pr->lawtab, pr->ws.partial);
    hipLaunchKernelGGL(k_max_partials, dim3(1), dim3(64), 0, s, kRedBlocks, pr->ws.partial, out);
    PPC_HIP(hipGetLastError());
}

}  // namespace ppc

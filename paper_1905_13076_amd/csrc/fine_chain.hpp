// Fine sweep: all N fine propagators F_n (Section 2, eqs. (2)-(3)) in one launch.
//
// One workgroup owns one chain n = 1..N: it starts from U_{n-1} at T_{n-1} and takes
// m implicit-Euler steps of size dt = T/(N m).  Each step solves
//     R(u) = M (u - u_prev)/dt + K(u) u - i(t_j) F = 0,   t_j = T_{n-1} + j dt,
// by damped Newton with the exact Jacobian
//     J = M/dt + sum_e [ nu_e K0_e + (2 nu'_e / A_e) (K0_e u_e)(K0_e u_e)^T ],
// (nu' = d nu / d|B|^2) solved by Jacobi-PCG.  Linear elements make J and R affine in u,
// so both are split into a base matrix Jb = M/dt + sum over linear e of nu_e K0_e, built
// once per sweep, and a Brauer part: a Newton iteration re-evaluates only the Brauer
// elements, the value positions they reach (a deterministic gather over a position ->
// contribution list, no atomics) and R = Jb u - M u_prev/dt + Brauer forces - i F.
//
// Mapping to CDNA: the chain's vectors and Jacobian values live in HBM (L2 / MALL
// resident for small meshes), the PCG keeps p (and for meshes that fit, r and the FP32
// Jacobi diagonal) in LDS and its rows in registers; the ELL SpMV streams values and
// 16-bit columns with raw buffer loads (a static count in flight, out-of-range lanes
// read zero) and gathers p from LDS.  Dot products are DPP wave sums followed by a
// fixed-order sum over the waves, so results are bitwise reproducible.  The PCG scalar
// type S is double (FP64 form) or float (mixed form: FP32 Jacobian and PCG, FP64 Newton
// residual refining it).
//
// This header holds the device code; fine.hip (1024-thread workgroups and every host
// launcher) and fine_blocks.hip (256- and 512-thread register-row forms) instantiate it.
#pragma once

#include <cfloat>
#include <cmath>

#include "internal.hpp"
#include "wave.hpp"

namespace ppc {



// Imposed current i(t) = sum_h amp_h sin(2 pi order_h f0 t + phase_h).
__device__ inline double current(double t, double f0, int n_h, const double* __restrict__ w) {
    double s = 0.0;
    for (int h = 0; h < n_h; ++h) s = s + w[3 * h + 1] * sin(2.0 * M_PI * w[3 * h] * f0 * t + w[3 * h + 2]);
    return s;
}

// Brauer / linear reluctivity and its derivative with respect to b2 = |B|^2.
__device__ inline void reluct(const double* __restrict__ lawtab, int mid, double b2, double& nu,
                              double& dnu) {
    const double* L = lawtab + 5 * mid;
    if (L[0] == 0.0) {
        nu = L[1];
        dnu = 0.0;
    } else {
        const double e = exp(L[3] * b2);
        nu = L[2] * e + L[4];
        dnu = L[2] * L[3] * e;
    }
}

enum { E_F0 = 0, E_W0 = 3, E_NU = 6, E_SF = 7 };

// Newton accepts a residual that stops halving (or a stalled line search) once it is
// below kFloorCap * scale: it then sits at the rounding floor of its evaluation.
constexpr double kFloorCap = 1e-9;
enum { V_U = 0, V_UP = 1, V_R = 2, V_RT = 3, V_UPP = 4, V_UT = 5, V_CP = 6, V_UP3 = 7, V_UP4 = 8 };
enum { P_R = 0, P_P = 1, P_Q = 2, P_X = 3, P_D = 4, P_H0 = 5, P_W0 = 5 + kHist };
enum { C_STATUS = 0, C_NEWTON = 1, C_LIN = 2, C_NEWTON_MAX = 3, C_LIN_MAX = 4, C_CAPPED = 5,
       C_FAILSTEP = 6, C_RESID = 7 };

// The Jacobian and residual split into a state-independent base and a Brauer part:
//     J(u) = Jb + sum over Brauer e [ nu_e K0_e + (2 nu'_e / A_e) w_e w_e^T ],
//     R(u) = Jb u - M u_prev / dt + sum over Brauer e nu_e K0_e u_e - i(t) F,
// with Jb = M/dt + sum over linear e nu_e K0_e built once per sweep (k_jbase), so a
// Newton iteration touches only the Brauer elements and the value positions they reach.

// Brauer element pass at the state ut: w = K0 ut_e, b2 = ut_e.w / A, nu, nu' and the
// element force nu w (scratch el, planes of nl_pad).
__device__ inline void nl_element_pass(const FineArgs& a, const double* __restrict__ ut,
                                       double* __restrict__ el) {
    const int nl = a.n_nl;
    const long P = a.nl_pad;
    for (int j = threadIdx.x; j < nl; j += blockDim.x) {
        double x[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int g = a.nl_efree[q * nl + j];
            x[q] = g >= 0 ? ut[g] : 0.0;
        }
        const double k00 = a.nl_k0[j], k01 = a.nl_k0[nl + j], k02 = a.nl_k0[2 * nl + j];
        const double k11 = a.nl_k0[3 * nl + j], k12 = a.nl_k0[4 * nl + j], k22 = a.nl_k0[5 * nl + j];
        const double w0 = k00 * x[0] + k01 * x[1] + k02 * x[2];
        const double w1 = k01 * x[0] + k11 * x[1] + k12 * x[2];
        const double w2 = k02 * x[0] + k12 * x[1] + k22 * x[2];
        const double A = a.nl_area[j];
        const double b2 = (x[0] * w0 + x[1] * w1 + x[2] * w2) / A;
        double nu, dnu;
        reluct(a.lawtab, a.nl_mat[j], b2, nu, dnu);
        el[(E_F0 + 0) * P + j] = nu * w0;
        el[(E_F0 + 1) * P + j] = nu * w1;
        el[(E_F0 + 2) * P + j] = nu * w2;
        el[(E_W0 + 0) * P + j] = w0;
        el[(E_W0 + 1) * P + j] = w1;
        el[(E_W0 + 2) * P + j] = w2;
        el[E_NU * P + j] = nu;
        el[E_SF * P + j] = 2.0 * dnu / A;
    }
}

// Brauer element forces of row i (node order)
__device__ inline double nl_force(const FineArgs& a, const double* __restrict__ el, int i) {
    const long P = a.nl_pad;
    double acc = 0.0;
    for (int k = a.nlf_ptr[i]; k < a.nlf_ptr[i + 1]; ++k) {
        const int code = a.nlf_src[k];
        const int j = code / 3, q = code - 3 * j;
        acc += el[(E_F0 + q) * P + j];
    }
    return acc;
}

// R = Jb ut - cp + (Brauer forces) - cur F over all rows, cp = M u_prev / dt; returns the
// partial ||R||^2 of this thread.  ELL rows load all their slots before the gathers; the
// tail rows are summed by one wave each.
__device__ inline double resid_rows(const FineArgs& a, const double* __restrict__ ut,
                                    const double* __restrict__ cp, const double* __restrict__ el,
                                    double cur, double* __restrict__ R) {
    const long NP = a.ell_pad;
    const int n = a.n, W = a.W;
    double part = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        int col[kEllMaxWidth];
        double val[kEllMaxWidth];
#pragma unroll
        for (int w = 0; w < kEllMaxWidth; ++w) {
            col[w] = w < W ? a.ecol[w * NP + i] : 0;
            val[w] = w < W ? a.jbase[w * NP + i] : 0.0;
        }
        if (col[0] < 0) continue;                 // tail row
        double acc = 0.0;
#pragma unroll
        for (int w = 0; w < kEllMaxWidth; ++w)
            if (w < W) acc += val[w] * ut[col[w]];
        acc = acc - cp[i] + nl_force(a, el, i) - cur * a.fload[i];
        R[i] = acc;
        part += acc * acc;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const long base = (long)W * NP;
    for (int t = wave; t < a.ntail; t += nw) {
        double acc = 0.0;
        const int j1 = a.tail_ptr[t + 1];
        for (int j = a.tail_ptr[t] + lane; j < j1; j += 64) acc += a.jbase[base + j] * ut[a.tail_col[j]];
        acc = wave_sum(acc);
        if (lane == 0) {
            const int i = a.tail_row[t];
            acc = acc - cp[i] + nl_force(a, el, i) - cur * a.fload[i];
            R[i] = acc;
            part += acc * acc;
        }
    }
    return part;
}

// Jacobian values of the Brauer-touched positions: Jb plus, per contribution of slot
// order, nu K0_ab + (2nu'/A) w_a w_b; every other position keeps its base value.
template <typename S>
__device__ inline void assemble_nl(const FineArgs& a, const double* __restrict__ el, S* __restrict__ jv) {
    const long P = a.nl_pad;
    const int nl = a.n_nl;
    for (int t = threadIdx.x; t < a.n_nlv; t += blockDim.x) {
        const int v = a.nlv_val[t];
        double acc = a.jbase[v];
        for (int k = a.nlv_ptr[t]; k < a.nlv_ptr[t + 1]; ++k) {
            const int code = a.nlv_src[k];
            const int j = code / 9, ab = code - 9 * j;
            const int qa = ab / 3, qb = ab - 3 * qa;
            const int lo = qa < qb ? qa : qb, hi = qa < qb ? qb : qa;
            const int kidx = lo == 0 ? hi : (lo == 1 ? 2 + hi : 5);
            acc += el[E_NU * P + j] * a.nl_k0[kidx * nl + j] +
                   el[E_SF * P + j] * el[(E_W0 + qa) * P + j] * el[(E_W0 + qb) * P + j];
        }
        jv[v] = (S)acc;
    }
}

// every value position takes its base value (start of a chain)
template <typename S>
__device__ inline void init_jac(const FineArgs& a, S* __restrict__ jv) {
    for (int v = threadIdx.x; v < a.nvals; v += blockDim.x) jv[v] = (S)a.jbase[v];
}

// cp = M u_prev / dt (once per time step) by ELL rows in the form of resid_rows: every row
// loads its W values of M (mell) and columns before its gathers, tail rows by one wave each;
// returns the partial ||cp||^2.
__device__ inline double mass_prev(const FineArgs& a, const double* __restrict__ up, double inv_dt,
                                   double* __restrict__ cp) {
    const long NP = a.ell_pad;
    const int n = a.n, W = a.W;
    double part = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        int col[kEllMaxWidth];
        double val[kEllMaxWidth];
#pragma unroll
        for (int w = 0; w < kEllMaxWidth; ++w) {
            col[w] = w < W ? a.ecol[w * NP + i] : 0;
            val[w] = w < W ? a.mell[w * NP + i] : 0.0;
        }
        if (col[0] < 0) continue;                 // tail row
        double acc = 0.0;
#pragma unroll
        for (int w = 0; w < kEllMaxWidth; ++w)
            if (w < W) acc += val[w] * up[col[w]];
        const double v = acc * inv_dt;
        cp[i] = v;
        part += v * v;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const long base = (long)W * NP;
    for (int t = wave; t < a.ntail; t += nw) {
        double acc = 0.0;
        const int j1 = a.tail_ptr[t + 1];
        for (int j = a.tail_ptr[t] + lane; j < j1; j += 64) acc += a.mell[base + j] * up[a.tail_col[j]];
        acc = wave_sum(acc);
        if (lane == 0) {
            const int i = a.tail_row[t];
            const double v = acc * inv_dt;
            cp[i] = v;
            part += v * v;
        }
    }
    return part;
}

// Row-sum of one tail (long) row by a whole wave; returns the sum on every lane.
template <typename S, typename PV>
__device__ inline S tail_row_sum(const FineArgs& a, const S* __restrict__ jv, PV p, int t, int lane) {
    const long base = (long)a.W * a.ell_pad;
    S acc = 0;
    const int j1 = a.tail_ptr[t + 1];
    for (int j = a.tail_ptr[t] + lane; j < j1; j += 64) acc += jv[base + j] * p[a.tail_col[j]];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    return acc;
}

// Jacobi-PCG on J x = -R for meshes that fit the CU: the rows of each thread keep x and q in
// registers; p, r and the inverse diagonal (FP32: it only shapes the preconditioner) live
// in LDS, so the SpMV gathers and every vector pass stay on the CU and only the ELL values
// and columns stream from memory.
//
// Rows go to threads in groups of G = 16 / sizeof(S) consecutive rows (2 in FP64, 4 in
// FP32): group q of thread t is rows G (t + q B) .. G (t + q B) + G - 1, so one 16-byte load
// brings a slot's values for the whole group and one 4- or 8-byte load its 16-bit columns,
// and the vector passes move a group through LDS in one 16-byte access.  Load instructions,
// not bytes, set the cost of this SpMV on the CU, so this halves it against a load per row.
// The R - G (R / G) rows left over go one per thread after the groups (row G Q B + t + j B).
//
// With kh > 0 the iteration starts from x0 = sum_j cg_j V_j (hist: the chain's last Newton
// corrections, wv: their products J V_j, both from galerkin_start): x starts there and r
// at b - sum_j cg_j J V_j.  xout may be one of the V_j (read here before it is written).
template <typename S, int R, int B>
__device__ int pcg_regs(const FineArgs& a, const S* __restrict__ jv, S* __restrict__ p_l,
                        S* __restrict__ r_l, const float* __restrict__ d_l, S* __restrict__ tq_l,
                        const double* __restrict__ Rres, double rs, S* xout, double tgt,
                        S* lds_s, int& ph, const S* hist = nullptr, const S* wv = nullptr, int kh = 0,
                        const double* cg = nullptr) {
    constexpr int G = 16 / (int)sizeof(S);
    constexpr int Q = R / G;                  // row groups per thread
    constexpr int L = R - Q * G;              // single rows per thread
    constexpr int QA = Q > 0 ? Q : 1, LA = L > 0 ? L : 1;
    using SG = S __attribute__((ext_vector_type(G)));
    using FG = float __attribute__((ext_vector_type(G)));
    using U4 = unsigned __attribute__((ext_vector_type(4)));
    using U2 = unsigned __attribute__((ext_vector_type(2)));
    const int tid = threadIdx.x, n = a.n;
    const int lane = tid & 63, wave = tid >> 6, nw = B >> 6;
    const long NP = a.ell_pad;
    const int W = a.W;
    // register slot k holds row row_of(k): the groups' rows first, then the single rows
    auto row_of = [&](int k) -> int {
        return k < Q * G ? G * (tid + (k / G) * B) + k % G : G * Q * B + tid + (k - Q * G) * B;
    };
    S x[R], q[R];
    unsigned tailmask = 0, padmask = 0;       // bit k: row_of(k) is a tail row / lies at or past n
    const __amdgpu_buffer_rsrc_t rv_j = buffer_rsrc(jv, (unsigned)(W * NP * sizeof(S)));
    const __amdgpu_buffer_rsrc_t rv_c = buffer_rsrc(a.ecol16, (unsigned)(W * NP * 2));
    // One tail row of at most B entries (the usual case): every thread takes one of its
    // entries and the first block reduction of an iteration carries the row's product
    // with p.q, so no wave runs a serial row sum.  Otherwise one wave per tail row.
    const bool tail1 = a.ntail == 1 && a.tail_ptr[1] - a.tail_ptr[0] <= B;
    const int t_beg = tail1 ? a.tail_ptr[0] : 0;
    const int t_len = tail1 ? a.tail_ptr[1] - t_beg : 0;
    const int t_row = tail1 ? a.tail_row[0] : 0;
    const __amdgpu_buffer_rsrc_t rv_tv = buffer_rsrc(jv + W * NP + t_beg, (unsigned)(t_len * sizeof(S)));
    const __amdgpu_buffer_rsrc_t rv_tc = buffer_rsrc(a.tail_col + t_beg, (unsigned)(t_len * 4));
    // rows at or past n: p, r and the diagonal's copies there are never read as data, but
    // the group passes touch them, so r and p are written as zero and the diagonal masked
    S loc[2] = {0, 0};
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int i = row_of(k);
        x[k] = 0;
        q[k] = 0;
        S rv = 0;
        if (i < n) {
            rv = (S)(-Rres[i] * rs);
            for (int j = 0; j < kh; ++j) {
                x[k] += (S)cg[j] * hist[j * NP + i];
                rv -= (S)cg[j] * wv[j * NP + i];
            }
            if (a.ecol[i] < 0) tailmask |= 1u << k;
        } else {
            padmask |= 1u << k;
        }
        const S z = i < n ? (S)d_l[i] * rv : (S)0;
        if (k < Q * G ? i - k % G < n : i < n) {
            r_l[i] = rv;
            p_l[i] = z;
        }
        loc[0] += rv * z;
        loc[1] += rv * rv;
    }
    block_sum<S, 2, B / 64>(loc, lds_s, ph);
    S rz = loc[0];
    double rr = (double)loc[1];
    int it = 0;
    // the diagonal of a row, zero past n
    auto dg = [&](int k, float d) -> S { return ((padmask >> k) & 1u) ? (S)0 : (S)d; };
    while (rr > tgt * tgt && it < a.max_lin) {
        // this thread's tail entry: loads issued first, used after the ELL rounds
        const S tv = buffer_load<S>(rv_tv, tid < t_len ? tid * (unsigned)sizeof(S) : kBufferNone);
        const unsigned tc = (unsigned)__builtin_amdgcn_raw_buffer_load_b32(rv_tc, tid < t_len ? tid * 4u : kBufferNone, 0, 0);
#pragma unroll
        for (int k = 0; k < R; ++k) q[k] = 0;
        // ELL slots in rounds of U, all loads of a round issued before its LDS gathers and
        // those before its FMAs.  A group past n loads nothing; slots >= W fall past the ELL
        // arrays; both read value 0 and column 0, as do the padded rows of a group that
        // straddles n.  Tail rows hold zero values and column 0.  Every row adds its slots
        // in order 0..W-1, then exact zeros.
        constexpr int NL = Q + L;             // value loads per slot
        constexpr int U = NL >= 4 ? 1 : 4 / NL;
        for (int w0 = 0; w0 < W; w0 += U) {
            SG vg[U][QA];
            unsigned cg2[U][QA][G / 2];       // G 16-bit columns, two per word
            S vs[U][LA], pg[U][R];
            unsigned cs[U][LA];
#pragma unroll
            for (int u = 0; u < U; ++u) {
#pragma unroll
                for (int g = 0; g < Q; ++g) {
                    const int i0 = G * (tid + g * B);
                    const unsigned e = (unsigned)((w0 + u) * NP + i0);
                    vg[u][g] = __builtin_bit_cast(SG, __builtin_amdgcn_raw_buffer_load_b128(
                                                          rv_j, i0 < n ? e * (unsigned)sizeof(S) : kBufferNone, 0, 0));
                    if constexpr (G == 2) {
                        cg2[u][g][0] = (unsigned)__builtin_amdgcn_raw_buffer_load_b32(rv_c, i0 < n ? e * 2u : kBufferNone, 0, 0);
                    } else {
                        const U2 c2 = __builtin_bit_cast(U2, __builtin_amdgcn_raw_buffer_load_b64(rv_c, i0 < n ? e * 2u : kBufferNone, 0, 0));
                        cg2[u][g][0] = c2.x;
                        cg2[u][g][1] = c2.y;
                    }
                }
#pragma unroll
                for (int j = 0; j < L; ++j) {
                    const int i = G * Q * B + tid + j * B;
                    const unsigned e = (unsigned)((w0 + u) * NP + i);
                    vs[u][j] = buffer_load<S>(rv_j, i < n ? e * (unsigned)sizeof(S) : kBufferNone);
                    cs[u][j] = __builtin_amdgcn_raw_buffer_load_b16(rv_c, i < n ? e * 2u : kBufferNone, 0, 0);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < U; ++u) {
#pragma unroll
                for (int g = 0; g < Q; ++g)
#pragma unroll
                    for (int h = 0; h < G; ++h)
                        pg[u][g * G + h] = p_l[(cg2[u][g][h >> 1] >> (16 * (h & 1))) & 0xffffu];
#pragma unroll
                for (int j = 0; j < L; ++j) pg[u][Q * G + j] = p_l[cs[u][j]];
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < U; ++u) {
#pragma unroll
                for (int g = 0; g < Q; ++g)
#pragma unroll
                    for (int h = 0; h < G; ++h) q[g * G + h] += vg[u][g][h] * pg[u][g * G + h];
#pragma unroll
                for (int j = 0; j < L; ++j) q[Q * G + j] += vs[u][j] * pg[u][Q * G + j];
            }
        }
        // p of this thread's rows: groups in one 16-byte LDS read each (a group past n
        // reads nothing: it may lie beyond the arrays).  FP32 keeps them in registers
        // through the iteration; FP64 rereads them from LDS after each reduction, since
        // the extra live registers cost more in spills than the reads save.
        constexpr bool kCache = sizeof(S) == 4;
        S pc[R];
#pragma unroll
        for (int g = 0; g < Q; ++g) {
            const int i0 = G * (tid + g * B);
            SG v = (SG)(S)0;
            if (i0 < n) v = *reinterpret_cast<const SG*>(p_l + i0);
#pragma unroll
            for (int h = 0; h < G; ++h) pc[g * G + h] = v[h];
        }
#pragma unroll
        for (int j = 0; j < L; ++j) {
            const int i = G * Q * B + tid + j * B;
            pc[Q * G + j] = i < n ? p_l[i] : (S)0;
        }
        S dot[2] = {0, 0};
#pragma unroll
        for (int k = 0; k < R; ++k)
            if (!((tailmask >> k) & 1u)) dot[0] += pc[k] * q[k];
        if (tail1) {
            const S qt = tv * p_l[tc];
            dot[1] = qt;
            dot[0] += p_l[t_row] * qt;
        } else {
            for (int t = wave; t < a.ntail; t += nw) {
                const S acc = tail_row_sum<S>(a, jv, p_l, t, lane);
                if (lane == 0) {
                    tq_l[t] = acc;
                    dot[0] += p_l[a.tail_row[t]] * acc;
                }
            }
        }
        block_sum<S, 2, B / 64>(dot, lds_s, ph);
        const S pq = dot[0];
        if (!(pq > (S)0)) break;                 // loss of positivity: Newton decides
        const S alpha = rz / pq;
        S l2[2] = {0, 0};
#pragma unroll
        for (int k = 0; k < R; ++k)
            if ((tailmask >> k) & 1u) q[k] = tail1 ? dot[1] : tq_l[a.ecol[NP + row_of(k)]];
        // x += alpha p, r -= alpha q, z = D r (z is kept in q: q is dead after r's update)
#pragma unroll
        for (int g = 0; g < Q; ++g) {
            const int i0 = G * (tid + g * B);
            if (i0 < n) {
                SG rv = *reinterpret_cast<const SG*>(r_l + i0);
                const FG dv = *reinterpret_cast<const FG*>(d_l + i0);
                SG pv;
                if constexpr (!kCache) pv = *reinterpret_cast<const SG*>(p_l + i0);
#pragma unroll
                for (int h = 0; h < G; ++h) {
                    const int k = g * G + h;
                    x[k] += alpha * (kCache ? pc[k] : pv[h]);
                    rv[h] = rv[h] - alpha * q[k];
                    q[k] = dg(k, dv[h]) * rv[h];
                    l2[0] += rv[h] * q[k];
                    l2[1] += rv[h] * rv[h];
                }
                *reinterpret_cast<SG*>(r_l + i0) = rv;
            }
        }
#pragma unroll
        for (int j = 0; j < L; ++j) {
            const int k = Q * G + j, i = G * Q * B + tid + j * B;
            if (i < n) {
                x[k] += alpha * (kCache ? pc[k] : p_l[i]);
                const S rv = r_l[i] - alpha * q[k];
                r_l[i] = rv;
                q[k] = (S)d_l[i] * rv;
                l2[0] += rv * q[k];
                l2[1] += rv * rv;
            }
        }
        block_sum<S, 2, B / 64>(l2, lds_s, ph);
        ++it;
        rr = (double)l2[1];
        if (rr <= tgt * tgt) break;
        const S beta = l2[0] / rz;
        rz = l2[0];
        // p = z + beta p
#pragma unroll
        for (int g = 0; g < Q; ++g) {
            const int i0 = G * (tid + g * B);
            if (i0 < n) {
                SG pv;
                if constexpr (!kCache) pv = *reinterpret_cast<const SG*>(p_l + i0);
#pragma unroll
                for (int h = 0; h < G; ++h) pv[h] = q[g * G + h] + beta * (kCache ? pc[g * G + h] : pv[h]);
                *reinterpret_cast<SG*>(p_l + i0) = pv;
            }
        }
#pragma unroll
        for (int j = 0; j < L; ++j) {
            const int i = G * Q * B + tid + j * B;
            if (i < n) p_l[i] = q[Q * G + j] + beta * (kCache ? pc[Q * G + j] : p_l[i]);
        }
        __syncthreads();
    }
    // padded rows [n, n_pad) are written as zero: xout is a stored correction whose rows
    // the Galerkin start reads in groups
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int i = row_of(k);
        if (i < NP) xout[i] = i < n ? x[k] : (S)0;
    }
    return it;
}

// Galerkin start of pcg_stream: coefficients cg (kh of them) of x0 = V c with
// (V^T J V) c = V^T b over the last kh Newton corrections V_j = hist + j n_pad; J V_j is kept
// in wv + j n_pad.  Two passes (the products, then the Galerkin sums from the stored
// vectors) keep the live registers of each near those of one SpMV pass.
template <typename S, int NW = 0>
__device__ inline void galerkin_start(const FineArgs& a, const S* __restrict__ jv, const S* hist, int kh,
                                      S* __restrict__ wv, S* __restrict__ tq_l,
                                      const double* __restrict__ Rres, double rs, double* lds_d, int& ph_d,
                                      double (&cg)[kHist]) {
    constexpr int V = 16 / (int)sizeof(S);
    typedef S vS __attribute__((ext_vector_type(V)));
    typedef int vI __attribute__((ext_vector_type(V)));
    const int B = blockDim.x, tid = threadIdx.x, n = a.n;
    const int lane = tid & 63, wave = tid >> 6, nw = B >> 6;
    const long NP = a.n_pad;
    const int W = a.W;
    const int G = (int)(NP / V);
    auto ld = [](const S* q, long i) { return *reinterpret_cast<const vS*>(q + i); };
    auto st = [](S* q, long i, vS v) { *reinterpret_cast<vS*>(q + i) = v; };
    for (int t = wave; t < a.ntail; t += nw)
        for (int j = 0; j < kh; ++j) {
            const S acc = tail_row_sum<S>(a, jv, hist + j * NP, t, lane);
            if (lane == 0) tq_l[j * a.ntail + t] = acc;
        }
    __syncthreads();
    // pass 1: W_j = J V_j
    for (int g = tid; g < G; g += B) {
        const int i0 = g * V;
        vS w[kHist];
#pragma unroll
        for (int j = 0; j < kHist; ++j) w[j] = (vS)(S)0;
        vI tl = (vI)0;
#pragma unroll
        for (int w0 = 0; w0 < kEllMaxWidth; w0 += 4) {
            if (w0 >= W) break;
            vS v[4];
            vI c[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int ww = w0 + u;
                if (ww < W) {
                    v[u] = ld(jv, ww * NP + i0);
                    c[u] = *reinterpret_cast<const vI*>(a.ecol + ww * NP + i0);
                } else {
                    v[u] = (vS)(S)0;
                    c[u] = (vI)0;
                }
            }
            if (w0 == 0)
#pragma unroll
                for (int k = 0; k < V; ++k) tl[k] = c[0][k] < 0 ? 1 + c[1][k] : 0;
#pragma unroll
            for (int j = 0; j < kHist; ++j) {
                if (j >= kh) break;
                const S* hj = hist + j * NP;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    vS gp;
#pragma unroll
                    for (int k = 0; k < V; ++k) gp[k] = hj[c[u][k] < 0 ? 0 : c[u][k]];
                    w[j] += v[u] * gp;
                }
            }
        }
#pragma unroll
        for (int j = 0; j < kHist; ++j) {
            if (j >= kh) break;
#pragma unroll
            for (int k = 0; k < V; ++k)
                if (tl[k] > 0) w[j][k] = tq_l[j * a.ntail + tl[k] - 1];
            st(wv + j * NP, i0, w[j]);
        }
    }
    __syncthreads();
    // pass 2: V_i^T W_j (i <= j) and V_i^T b, in FP64
    constexpr int NG = kHist * kHist + kHist;
    double gs[NG];
#pragma unroll
    for (int q = 0; q < NG; ++q) gs[q] = 0.0;
    for (int g = tid; g < G; g += B) {
        const int i0 = g * V;
        vS b;
#pragma unroll
        for (int k = 0; k < V; ++k) b[k] = i0 + k < n ? (S)(-Rres[i0 + k] * rs) : (S)0;
        vS hv[kHist], wj[kHist];
#pragma unroll
        for (int j = 0; j < kHist; ++j) {
            hv[j] = j < kh ? ld(hist + j * NP, i0) : (vS)(S)0;
            wj[j] = j < kh ? ld(wv + j * NP, i0) : (vS)(S)0;
#pragma unroll
            for (int k = 0; k < V; ++k)
                if (i0 + k >= n) hv[j][k] = (S)0;    // padded rows take no part
        }
#pragma unroll
        for (int i = 0; i < kHist; ++i) {
#pragma unroll
            for (int j = i; j < kHist; ++j)
#pragma unroll
                for (int k = 0; k < V; ++k) gs[i * kHist + j] += (double)hv[i][k] * (double)wj[j][k];
#pragma unroll
            for (int k = 0; k < V; ++k) gs[kHist * kHist + i] += (double)hv[i][k] * (double)b[k];
        }
    }
    // workgroup sums, four values at a time (the reduction buffer holds four)
#pragma unroll
    for (int q0 = 0; q0 < NG; q0 += 4) {
        double t4[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) t4[u] = q0 + u < NG ? gs[q0 + u] : 0.0;
        block_sum<double, 4, NW>(t4, lds_d, ph_d);
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (q0 + u < NG) gs[q0 + u] = t4[u];
    }
    // Cholesky of the kh x kh Galerkin matrix (unrolled over kHist, entries beyond kh
    // inactive); a pivot at rounding level relative to its diagonal marks a dependent
    // direction, whose coefficient stays 0
    double L[kHist][kHist];
    bool on[kHist];
#pragma unroll
    for (int j = 0; j < kHist; ++j) {
#pragma unroll
        for (int i = 0; i < kHist; ++i) L[i][j] = 0.0;
        double d = gs[j * kHist + j];
#pragma unroll
        for (int m = 0; m < j; ++m) d -= L[j][m] * L[j][m];
        on[j] = j < kh && d > (sizeof(S) == 4 ? 1e-5 : 1e-10) * gs[j * kHist + j] && isfinite(d);
        if (on[j]) {
            L[j][j] = sqrt(d);
#pragma unroll
            for (int i = j + 1; i < kHist; ++i) {
                double e = gs[j * kHist + i];
#pragma unroll
                for (int m = 0; m < j; ++m) e -= L[i][m] * L[j][m];
                L[i][j] = i < kh ? e / L[j][j] : 0.0;
            }
        }
    }
    double y[kHist];
#pragma unroll
    for (int j = 0; j < kHist; ++j) {
        double e = gs[kHist * kHist + j];
#pragma unroll
        for (int m = 0; m < j; ++m) e -= L[j][m] * y[m];
        y[j] = on[j] ? e / L[j][j] : 0.0;
    }
#pragma unroll
    for (int j = kHist - 1; j >= 0; --j) {
        double e = y[j];
#pragma unroll
        for (int m = j + 1; m < kHist; ++m) e -= L[m][j] * cg[m];
        cg[j] = on[j] ? e / L[j][j] : 0.0;
    }
}

// Same algorithm for meshes beyond the register rows, streaming the chain's vectors from
// memory.  Each thread owns groups of V = 16 / sizeof(S) consecutive rows, so every value,
// column and vector access is one 16-byte load or store per lane (four FP32 or two FP64
// rows), and a group issues the loads of a round of ELL slots before the gathers that use
// them.  Three passes per iteration, two workgroup reductions:
//   q = J p (gathers of p; tail rows summed first by one wave each into LDS), p.q;
//   x += alpha p, r -= alpha q, with r.Dr and r.r (D the Jacobi inverse diagonal);
//   p = D r + beta p.
// p lives in LDS when PL == 1 (the gathers then stay on the CU), else in memory.  The
// inverse diagonal is formed here from the Jacobian's diagonal positions.  Rows of the
// padded tail [n, n_pad) hold zero in every vector.
//
// Start: with kh > 0 the iteration starts from the Galerkin projection of the solution on
// the span of the chain's last kh Newton corrections V_j (hist, kh <= kHist): x0 = V c with
// (V^T J V) c = V^T b, the point of that span closest to the solution in the J-norm.  The
// corrections of successive steps vary smoothly in time, so the projection removes most of
// the right-hand side before the first iteration.  One pass forms J V_j (kept in wv) with
// the Galerkin sums; a Cholesky factorisation that drops dependent directions gives c on
// every thread alike; x0 and r0 = b - (J V) c follow in the initial pass.  The solution is
// accumulated in xout, which may be the oldest history vector (read before it is written).
template <typename S, int PL, int NW = 0>
__device__ int pcg_stream(const FineArgs& a, const S* __restrict__ jv, S* __restrict__ pv,
                          S* __restrict__ p_l, S* __restrict__ tq_l, const double* __restrict__ Rres,
                          double rs, double tgt, S* lds_s, int& ph, S* xout, const S* hist, int kh,
                          S* __restrict__ wv, double* lds_d, int& ph_d) {
    constexpr int V = 16 / (int)sizeof(S);
    typedef S vS __attribute__((ext_vector_type(V)));
    typedef int vI __attribute__((ext_vector_type(V)));
    const int B = blockDim.x, tid = threadIdx.x, n = a.n;
    const int lane = tid & 63, wave = tid >> 6, nw = B >> 6;
    const long NP = a.n_pad;
    const int W = a.W;
    const int G = (int)(NP / V);
    S* pr = pv + P_R * NP;
    S* pq = pv + P_Q * NP;
    S* px = xout;
    S* pd = pv + P_D * NP;
    S* pp = PL ? p_l : pv + P_P * NP;
    auto ld = [](const S* q, long i) { return *reinterpret_cast<const vS*>(q + i); };
    auto st = [](S* q, long i, vS v) { *reinterpret_cast<vS*>(q + i) = v; };
    auto rhs = [&](int i0) {
        vS b;
#pragma unroll
        for (int k = 0; k < V; ++k) b[k] = i0 + k < n ? (S)(-Rres[i0 + k] * rs) : (S)0;
        return b;
    };
    double cg[kHist] = {0.0};
    if (kh > 0) galerkin_start<S, NW>(a, jv, hist, kh, wv, tq_l, Rres, rs, lds_d, ph_d, cg);
    // ---- initial residual, diagonal, direction ------------------------------------------------
    S loc[2] = {0, 0};
    for (int g = tid; g < G; g += B) {
        const int i0 = g * V;
        vS r = rhs(i0), x = (vS)(S)0, d;
#pragma unroll
        for (int j = 0; j < kHist; ++j) {
            if (j >= kh) break;
            x += (S)cg[j] * ld(hist + j * NP, i0);
            r -= (S)cg[j] * ld(wv + j * NP, i0);
        }
#pragma unroll
        for (int k = 0; k < V; ++k)
            if (i0 + k >= n) {          // padded rows stay zero in every vector
                x[k] = (S)0;
                r[k] = (S)0;
            }
#pragma unroll
        for (int k = 0; k < V; ++k) d[k] = i0 + k < n ? (S)1 / jv[a.dpos[i0 + k]] : (S)0;
        const vS z = d * r;
        st(pr, i0, r);
        st(pd, i0, d);
        st(pp, i0, z);
        st(px, i0, x);
#pragma unroll
        for (int k = 0; k < V; ++k) {
            loc[0] += r[k] * z[k];
            loc[1] += r[k] * r[k];
        }
    }
    block_sum<S, 2, NW>(loc, lds_s, ph);
    S rz = loc[0];
    double rr = (double)loc[1];
    int it = 0;
    while (rr > tgt * tgt && it < a.max_lin) {
        // tail rows (longer than the ELL width): one wave per row, kept in LDS for the
        // rows' owners below
        for (int t = wave; t < a.ntail; t += nw) {
            const S acc = tail_row_sum<S>(a, jv, pp, t, lane);
            if (lane == 0) tq_l[t] = acc;
        }
        __syncthreads();
        S dot[1] = {0};
        for (int g = tid; g < G; g += B) {
            const int i0 = g * V;
            vS acc = (vS)(S)0;
            vI tl = (vI)0;        // tail rows: slot 0 holds -1 and slot 1 the tail index
            // slots in rounds of four: the value and column loads of a round in flight
            // together, then its gathers, then its products
#pragma unroll
            for (int w0 = 0; w0 < kEllMaxWidth; w0 += 4) {
                if (w0 >= W) break;
                vS v[4];
                vI c[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int w = w0 + u;
                    if (w < W) {
                        v[u] = ld(jv, w * NP + i0);
                        c[u] = *reinterpret_cast<const vI*>(a.ecol + w * NP + i0);
                    } else {
                        v[u] = (vS)(S)0;
                        c[u] = (vI)0;
                    }
                }
                if (w0 == 0)
#pragma unroll
                    for (int k = 0; k < V; ++k) tl[k] = c[0][k] < 0 ? 1 + c[1][k] : 0;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    vS gp;
#pragma unroll
                    for (int k = 0; k < V; ++k) gp[k] = pp[c[u][k] < 0 ? 0 : c[u][k]];
                    acc += v[u] * gp;
                }
            }
#pragma unroll
            for (int k = 0; k < V; ++k)
                if (tl[k] > 0) acc[k] = tq_l[tl[k] - 1];
            st(pq, i0, acc);
            const vS pown = ld(pp, i0);
#pragma unroll
            for (int k = 0; k < V; ++k) dot[0] += pown[k] * acc[k];
        }
        block_sum<S, 1, NW>(dot, lds_s, ph);
        const S pqv = dot[0];
        if (!(pqv > (S)0)) break;                 // loss of positivity: Newton decides
        const S alpha = rz / pqv;
        S l2[2] = {0, 0};
        for (int g = tid; g < G; g += B) {
            const int i0 = g * V;
            const vS x = ld(px, i0) + alpha * ld(pp, i0);
            const vS r = ld(pr, i0) - alpha * ld(pq, i0);
            const vS z = ld(pd, i0) * r;
            st(px, i0, x);
            st(pr, i0, r);
#pragma unroll
            for (int k = 0; k < V; ++k) {
                l2[0] += r[k] * z[k];
                l2[1] += r[k] * r[k];
            }
        }
        block_sum<S, 2, NW>(l2, lds_s, ph);
        ++it;
        rr = (double)l2[1];
        if (rr <= tgt * tgt) break;
        const S beta = l2[0] / rz;
        rz = l2[0];
        for (int g = tid; g < G; g += B) {
            const int i0 = g * V;
            st(pp, i0, ld(pd, i0) * ld(pr, i0) + beta * ld(pp, i0));
        }
        __syncthreads();
    }
    return it;
}

// R > 0: PCG rows in registers, p / diagonal / tail sums in dynamic LDS;
// R == 0: PCG vectors streamed from memory, with p in LDS when LP == 1; the tail-row sums
// in LDS after it.
template <typename S, int R, int BLOCK, int LP>
__device__ __forceinline__ void fine_chain(const FineArgs& a, const int c, unsigned char* dyn_lds,
                                           double* lds_d, S* lds_s) {
    int ph_d = 0, ph_s = 0;                   // chain n = c + 1
    const int n = a.n;
    const long NP = a.n_pad;
    double* vec = a.vec + (long)c * kFineVec * NP;
    double* u = vec + V_U * NP;
    double* up = vec + V_UP * NP;
    double* R_ = vec + V_R * NP;
    double* Rt = vec + V_RT * NP;
    double* upp = vec + V_UPP * NP;
    double* up3 = vec + V_UP3 * NP;           // u_{j-3}
    double* up4 = vec + V_UP4 * NP;           // u_{j-4}
    double* ut = vec + V_UT * NP;             // trial state of the line search
    double* cp = vec + V_CP * NP;             // M u_prev / dt
    S* pv = reinterpret_cast<S*>(a.pcg) + (long)c * kPcgVec * NP;
    S* px = pv + P_X * NP;
    S* jv = reinterpret_cast<S*>(a.jac) + (long)c * a.vals_pad;
    double* el = a.elem + (long)c * 8 * a.nl_pad;
    S* p_l = reinterpret_cast<S*>(dyn_lds);
    S* r_l = p_l + NP;                        // register path: r
    float* df_l = reinterpret_cast<float*>(r_l + NP);   // register path: FP32 diagonal
    S* tq_l = R > 0 ? reinterpret_cast<S*>(df_l + NP) : (LP == 1 ? p_l + NP : p_l);

    const double* U0 = a.U + (long)c * n;
    double* Tc = a.traj ? a.traj + (long)c * (a.m + 1) * n : nullptr;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        u[i] = U0[i];
        if (Tc) Tc[i] = U0[i];
    }
    init_jac<S>(a, jv);
    __syncthreads();

    const double t0 = (double)c * (a.T / a.N);
    const double inv_dt = 1.0 / a.dt;
    int status = 0, fail_step = -1;
    int newton_total = 0, lin_total = 0, newton_max = 0, lin_max = 0, capped = 0, resid_evals = 0;
    int n_solves = 0;                         // Newton solves of this chain (history slots filled)
    int prev_newton = 1;                      // Newton iterations of the previous step
    // Newton tolerance of this sweep: fixed, or (adapt_scal set) loosened in proportion to
    // the outer iteration's last relative jump, never looser than kAdaptCap; a first sweep
    // (no jumps yet: ||U|| = 0) takes the cap
    double tol_nt = a.tol_newton;
    if (a.adapt_scal) {
        const double jj = a.adapt_scal[0], uu = a.adapt_scal[1];
        double e = (uu > 0.0 && jj >= 0.0) ? a.tol_adapt * sqrt(jj / uu) : kAdaptCap;
        if (!(e <= kAdaptCap)) e = kAdaptCap;
        tol_nt = fmax(tol_nt, e);
    }

    for (int j = 1; j <= a.m && status == 0; ++j) {
        const double t = t0 + j * a.dt;
        // u_{j-1} -> u_prev (u_{j-2}, u_{j-3}, u_{j-4} kept for the predictor)
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            up4[i] = up3[i];
            up3[i] = upp[i];
            upp[i] = up[i];
            up[i] = u[i];
        }
        __syncthreads();
        const double cur = current(t, a.f0, a.n_h, a.wavtab);
        double v1[1] = {mass_prev(a, up, inv_dt, cp)};
        block_sum<double, 1, BLOCK / 64>(v1, lds_d, ph_d);
        const double scale = fabs(cur) * a.fnorm + sqrt(v1[0]);
        const double target = tol_nt * scale;

        nl_element_pass(a, u, el);
        ++resid_evals;
        __syncthreads();
        double v2[1] = {resid_rows(a, u, cp, el, cur, R_)};
        block_sum<double, 1, BLOCK / 64>(v2, lds_d, ph_d);
        double rn = sqrt(v2[0]);
        if (!isfinite(rn)) { status = PPC_ERR_NONFINITE; fail_step = j; break; }
        // Newton starts from the extrapolation of the previous steps (cubic
        // 4 u_{j-1} - 6 u_{j-2} + 4 u_{j-3} - u_{j-4} from the fourth step on, quadratic
        // 3 u_{j-1} - 3 u_{j-2} + u_{j-3} at the third, linear 2 u_{j-1} - u_{j-2} at the
        // second) when that has the smaller residual; it changes only the iteration count,
        // not the step's solution
        if (j >= 2 && a.predictor && rn > target) {
            if (j >= 4)
                for (int i = threadIdx.x; i < n; i += blockDim.x)
                    ut[i] = 4.0 * (up[i] + up3[i]) - 6.0 * upp[i] - up4[i];
            else if (j >= 3)
                for (int i = threadIdx.x; i < n; i += blockDim.x) ut[i] = 3.0 * (up[i] - upp[i]) + up3[i];
            else
                for (int i = threadIdx.x; i < n; i += blockDim.x) ut[i] = 2.0 * up[i] - upp[i];
            __syncthreads();
            nl_element_pass(a, ut, el);
            ++resid_evals;
            __syncthreads();
            double v4[1] = {resid_rows(a, ut, cp, el, cur, Rt)};
            block_sum<double, 1, BLOCK / 64>(v4, lds_d, ph_d);
            const double rp = sqrt(v4[0]);
            if (rp < rn) {
                double* tmp = R_;
                R_ = Rt;
                Rt = tmp;
                tmp = u;
                u = ut;
                ut = tmp;
                rn = rp;
            } else {
                nl_element_pass(a, u, el);
                ++resid_evals;
                __syncthreads();
            }
        }

        int it = 0;
        // forcing of the linear solves (lin_forcing 1): a step whose predecessor needed
        // several Newton iterations sits in the nonlinear regime, where a tight first solve
        // is wasted; later iterations follow the observed contraction (Eisenstat-Walker,
        // choice 2: eta = 0.9 (||R_k|| / ||R_{k-1}||)^2, safeguarded by 0.9 eta_{k-1}^2),
        // always within [tol_lin, 0.1]
        double eta = (a.lin_forcing && prev_newton >= 2) ? fmax(a.tol_lin, 1e-3) : a.tol_lin;
        double rn_last = rn;
        for (;; ++it) {
            if (rn <= target) break;
            if (it == a.max_newton) { status = PPC_ERR_NEWTON; fail_step = j; break; }
            if (a.lin_forcing && it > 0) {
                const double q = rn / rn_last;
                double e = 0.9 * q * q;
                const double sg = 0.9 * eta * eta;
                if (sg > 0.1) e = fmax(e, sg);
                eta = fmin(0.1, fmax(a.tol_lin, e));
            }
            rn_last = rn;
            assemble_nl<S>(a, el, jv);
            __syncthreads();
            if constexpr (R > 0) {
                for (int i = threadIdx.x; i < n; i += blockDim.x) df_l[i] = (float)(1.0 / (double)jv[a.dpos[i]]);
                __syncthreads();
            }
            const double ltarget = fmax(eta * rn, 0.5 * target);
            // FP32 PCG solves for the unit right-hand side -R/||R|| (near convergence the
            // residual and its products would fall below FP32's range); the step px * xs
            // is formed in FP64.  FP64 solves use R itself.
            const double rs = (sizeof(S) == 4 && rn > 0.0) ? 1.0 / rn : 1.0;
            const double xs = (sizeof(S) == 4 && rn > 0.0) ? rn : 1.0;
            int k;
            // the first Newton correction of a step goes to the oldest history slot, and with
            // lin_start 0 the last (at most kHist) first corrections seed its solve.  Later
            // corrections of a step refine that step: their right-hand sides are not the smooth
            // continuation in time that the history spans (a start from its span measured up
            // to twice the PCG iterations of the zero start on chains taking five Newton
            // iterations per step), so they start from zero and are not kept.
            const bool first = it == 0;
            px = pv + (long)(first ? P_H0 + n_solves % kHist : P_X) * NP;
            const int kh = (a.lin_start == 0 && first) ? (n_solves < kHist ? n_solves : kHist) : 0;
            if constexpr (R > 0) {
                double cg[kHist] = {0.0};
                if (kh > 0) galerkin_start<S, BLOCK / 64>(a, jv, pv + P_H0 * NP, kh, pv + P_W0 * NP, tq_l, R_, rs, lds_d, ph_d, cg);
                k = pcg_regs<S, R, BLOCK>(a, jv, p_l, r_l, df_l, tq_l, R_, rs, px, ltarget * rs, lds_s, ph_s,
                                          pv + P_H0 * NP, pv + P_W0 * NP, kh, cg);
            } else {
                k = pcg_stream<S, LP, BLOCK / 64>(a, jv, pv, p_l, tq_l, R_, rs, ltarget * rs, lds_s, ph_s, px, pv + P_H0 * NP,
                                      kh, pv + P_W0 * NP, lds_d, ph_d);
            }
            if (first) ++n_solves;
            __syncthreads();
            lin_total += k;
            lin_max = k > lin_max ? k : lin_max;
            if (k == a.max_lin) ++capped;
            // ---- Newton update with backtracking -------------------------------------------
            double nrm[2] = {0.0, 0.0};
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                const double dv = (double)px[i] * xs;
                nrm[0] += dv * dv;
                nrm[1] += u[i] * u[i];
            }
            block_sum<double, 2, BLOCK / 64>(nrm, lds_d, ph_d);
            if (sqrt(nrm[0]) <= 4.0 * DBL_EPSILON * sqrt(nrm[1])) {
                for (int i = threadIdx.x; i < n; i += blockDim.x) u[i] = u[i] + (double)px[i] * xs;
                __syncthreads();
                ++it;
                break;
            }
            double lam = 1.0;
            double rt = 0.0;
            bool accepted = false, stalled = false;
            while (true) {
                for (int i = threadIdx.x; i < n; i += blockDim.x) ut[i] = u[i] + lam * ((double)px[i] * xs);
                __syncthreads();
                nl_element_pass(a, ut, el);
                ++resid_evals;
                __syncthreads();
                double v3[1] = {resid_rows(a, ut, cp, el, cur, Rt)};
                block_sum<double, 1, BLOCK / 64>(v3, lds_d, ph_d);
                rt = sqrt(v3[0]);
                if (rt <= (1.0 - 1e-4 * lam) * rn) { accepted = true; break; }
                lam *= 0.5;
                if (lam < 0x1p-20) { stalled = true; break; }
            }
            if (stalled) {
                if (rn <= kFloorCap * scale) { ++it; break; }
                status = isfinite(rt) ? PPC_ERR_NEWTON : PPC_ERR_NONFINITE;
                fail_step = j;
                break;
            }
            if (accepted) {
                double* tmp = u;
                u = ut;
                ut = tmp;
                tmp = R_;
                R_ = Rt;
                Rt = tmp;
                // a step that fails to halve a residual below the floor cap: the residual
                // sits at the rounding floor of its own evaluation
                const bool floor = rt > 0.5 * rn && rt <= kFloorCap * scale;
                rn = rt;
                if (floor) { ++it; break; }
            }
        }
        newton_total += it;
        newton_max = it > newton_max ? it : newton_max;
        prev_newton = it;
        if (Tc)
            for (int i = threadIdx.x; i < n; i += blockDim.x) Tc[(long)j * n + i] = u[i];
    }

    double* Fo = a.F + (long)((c + 1) % a.N) * n;
    for (int i = threadIdx.x; i < n; i += blockDim.x) Fo[i] = u[i];
    if (threadIdx.x == 0) {
        int* cnt = a.count + 8 * c;
        cnt[C_STATUS] = status;
        cnt[C_NEWTON] = newton_total;
        cnt[C_LIN] = lin_total;
        cnt[C_NEWTON_MAX] = newton_max;
        cnt[C_LIN_MAX] = lin_max;
        cnt[C_CAPPED] = capped;
        cnt[C_FAILSTEP] = fail_step;
        cnt[C_RESID] = resid_evals;
    }
}

// out_i = -(M y)_i (CSR, kRowGroup lanes per row); returns the partial ||M y||^2
__device__ inline double mass_apply_neg(const FineArgs& a, const double* __restrict__ y,
                                        double* __restrict__ out) {
    constexpr int G = kRowGroup;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int sub = lane % G, grp = lane / G;
    constexpr int RPW = 64 / G;
    double part = 0.0;
    for (int base = wave * RPW; base < a.n; base += nw * RPW) {
        const int i = base + grp;
        double acc = 0.0;
        if (i < a.n) {
            const int k1 = a.rowptr[i + 1];
            for (int k = a.rowptr[i] + sub; k < k1; k += G) acc += a.mval[k] * y[a.colidx[k]];
        }
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
        if (i < a.n && sub == 0) {
            out[i] = -acc;
            part += acc * acc;
        }
    }
    return part;
}

// One chain of the adjoint backward sweep: from Lambda_{c+1} down to lambda_{cm+1},
// solving J_j lambda_j = M (lambda_{j+1}/dt + 2/(T dt) (du_j - du_{j+1})) for
// j = (c+1)m .. cm+1 with J_j assembled at the stored forward state u_j.
template <typename S, int R, int BLOCK, int LP>
__device__ __forceinline__ void adjoint_chain(const FineArgs& a, const AdjArgs& b, const int c,
                                              unsigned char* dyn_lds, double* lds_d, S* lds_s) {
    int ph_d = 0, ph_s = 0;
    const int n = a.n, m = a.m, N = a.N;
    const long NP = a.n_pad;
    double* vec = a.vec + (long)c * kFineVec * NP;
    double* lam = vec + V_U * NP;
    double* y = vec + V_UP * NP;
    double* rhs = vec + V_R * NP;
    S* pv = reinterpret_cast<S*>(a.pcg) + (long)c * kPcgVec * NP;
    S* px = pv + P_X * NP;
    S* jv = reinterpret_cast<S*>(a.jac) + (long)c * a.vals_pad;
    double* el = a.elem + (long)c * 8 * a.nl_pad;
    S* p_l = reinterpret_cast<S*>(dyn_lds);
    S* r_l = p_l + NP;
    float* df_l = reinterpret_cast<float*>(r_l + NP);
    S* tq_l = R > 0 ? reinterpret_cast<S*>(df_l + NP) : (LP == 1 ? p_l + NP : p_l);
    const double* T0 = b.traj + (long)c * (m + 1) * n;
    const double* T1 = b.traj + (long)((c + 1) % N) * (m + 1) * n;
    const double* Lin = b.lam_in + (long)((c + 1) % N) * n;
    for (int i = threadIdx.x; i < n; i += blockDim.x) lam[i] = Lin[i];
    init_jac<S>(a, jv);
    __syncthreads();
    const double inv_dt = 1.0 / a.dt;
    const double gcoef = 2.0 / (b.T * a.dt);
    int lin_total = 0, lin_max = 0, capped = 0;
    for (int jl = m; jl >= 1; --jl) {
        const double* uj = T0 + (long)jl * n;
        const double* ujm = T0 + (long)(jl - 1) * n;
        const double* nx0 = jl < m ? uj : T1;
        const double* nx1 = jl < m ? T0 + (long)(jl + 1) * n : T1 + n;
        for (int i = threadIdx.x; i < n; i += blockDim.x)
            y[i] = lam[i] * inv_dt + gcoef * ((uj[i] - ujm[i]) - (nx1[i] - nx0[i]));
        __syncthreads();
        double v[1] = {mass_apply_neg(a, y, rhs)};
        block_sum<double, 1, BLOCK / 64>(v, lds_d, ph_d);
        const double rn = sqrt(v[0]);
        nl_element_pass(a, uj, el);
        __syncthreads();
        assemble_nl<S>(a, el, jv);
        __syncthreads();
        if constexpr (R > 0) {
            for (int i = threadIdx.x; i < n; i += blockDim.x) df_l[i] = (float)(1.0 / (double)jv[a.dpos[i]]);
            __syncthreads();
        }
        int k = 0;
        if (rn > 0.0) {
            if constexpr (R > 0)
                k = pcg_regs<S, R, BLOCK>(a, jv, p_l, r_l, df_l, tq_l, rhs, 1.0, px, b.tol_lin * rn, lds_s, ph_s);
            else
                k = pcg_stream<S, LP, BLOCK / 64>(a, jv, pv, p_l, tq_l, rhs, 1.0, b.tol_lin * rn, lds_s, ph_s, px, pv, 0,
                                      pv, lds_d, ph_d);
        } else {
            for (int i = threadIdx.x; i < n; i += blockDim.x) px[i] = 0;
        }
        __syncthreads();
        lin_total += k;
        lin_max = k > lin_max ? k : lin_max;
        if (k == a.max_lin) ++capped;
        double* Lall = b.lam_all + ((long)c * m + (jl - 1)) * n;
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const double vv = (double)px[i];
            lam[i] = vv;
            Lall[i] = vv;
        }
        __syncthreads();
    }
    double* out = b.lam_out + (long)c * n;
    for (int i = threadIdx.x; i < n; i += blockDim.x) out[i] = lam[i];
    if (threadIdx.x == 0) {
        int* cnt = a.count + 8 * c;
        cnt[C_STATUS] = 0;
        cnt[C_NEWTON] = 0;
        cnt[C_LIN] = lin_total;
        cnt[C_NEWTON_MAX] = 0;
        cnt[C_LIN_MAX] = lin_max;
        cnt[C_CAPPED] = capped;
        cnt[C_FAILSTEP] = -1;
        cnt[C_RESID] = 0;
    }
}

template <typename S, int R, int BLOCK, int LP>
__global__ __launch_bounds__(BLOCK) void k_adjoint_sweep(FineArgs a, AdjArgs b) {
    extern __shared__ unsigned char dyn_lds[];
    __shared__ double lds_d[2 * 16 * 4];
    __shared__ S lds_s[2 * 16 * 4];
    adjoint_chain<S, R, BLOCK, LP>(a, b, blockIdx.x, dyn_lds, lds_d, lds_s);
}

template <typename S, int R, int BLOCK, int LP>
__global__ __launch_bounds__(BLOCK) void k_fine_sweep(FineArgs a) {
    extern __shared__ unsigned char dyn_lds[];
    __shared__ double lds_d[2 * 16 * 4];
    __shared__ S lds_s[2 * 16 * 4];
    fine_chain<S, R, BLOCK, LP>(a, blockIdx.x, dyn_lds, lds_d, lds_s);
}

// Batched designs: block b runs chain work[b].y of design work[b].x, whose arguments are
// args[work[b].x] (a work list over every design of one kernel shape, longest first).
template <typename S, int R, int BLOCK, int LP>
__global__ __launch_bounds__(BLOCK) void k_fine_sweep_batch(const FineArgs* __restrict__ args,
                                                            const int2* __restrict__ work) {
    extern __shared__ unsigned char dyn_lds[];
    __shared__ double lds_d[2 * 16 * 4];
    __shared__ S lds_s[2 * 16 * 4];
    const int2 wk = work[blockIdx.x];
    fine_chain<S, R, BLOCK, LP>(args[wk.x], wk.y, dyn_lds, lds_d, lds_s);
}

}  // namespace ppc

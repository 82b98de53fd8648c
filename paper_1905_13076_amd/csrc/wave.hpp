// Wave- and workgroup-level building blocks shared by the fine and coarse kernels:
// DPP wave sums and fixed-order workgroup sums (bitwise reproducible), and raw buffer
// loads whose out-of-range lanes read zero.
#pragma once

#include <hip/hip_runtime.h>

namespace ppc {

// DPP lane move within 16-lane rows (CTRL: quad_perm / mirror codes of the gfx9 DPP
// encoding); every lane of the wave must be active.
template <int CTRL, typename T>
__device__ inline T dpp_mov(T v) {
    if constexpr (sizeof(T) == 8) {
        const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
        const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)u, CTRL, 0xF, 0xF, false);
        const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, false);
        return __builtin_bit_cast(T, ((unsigned long long)hi << 32) | lo);
    } else {
        return __builtin_bit_cast(T, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
    }
}

template <typename T>
__device__ inline T read_lane(T v, int l) {
    if constexpr (sizeof(T) == 8) {
        const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
        const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
        const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
        return __builtin_bit_cast(T, ((unsigned long long)hi << 32) | lo);
    } else {
        return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
    }
}

// Wave sum in a fixed order: pairs, quads, half rows and rows by DPP (each step adds two
// partial sums that commute, so all lanes of a row hold the same bits), then the four
// row sums as (r0 + r1) + (r2 + r3).  Returns the same value on every lane.
template <typename T>
__device__ inline T wave_sum(T v) {
    v += dpp_mov<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_mov<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_mov<0x141>(v);   // row_half_mirror
    v += dpp_mov<0x140>(v);   // row_mirror
    return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

// Sum of K values over the workgroup in a fixed order; every thread gets the result.
// NW > 0 states the wave count at compile time (NW <= 16, K <= 4): lane 16 k + j of every
// wave then reads wave j's partial of value k, one LDS read per wave for all K values, and
// each 16-lane row adds its partials by the DPP steps of wave_sum, so every wave forms the
// same bits.  NW == 0 adds the partials in wave order.
template <typename T, int K, int NW = 0>
__device__ inline void block_sum(T (&v)[K], T* lds, int& phase) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    T* buf = lds + phase * 16 * K;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) buf[k * 16 + w] = v[k];
    __syncthreads();
    if constexpr (NW > 0) {
        static_assert(NW <= 16 && K <= 4, "one 64-lane read covers at most 4 values of 16 waves");
        T t = (lane < 16 * K && (lane & 15) < NW) ? buf[lane] : (T)0;
        t += dpp_mov<0xB1>(t);    // quad_perm [1,0,3,2]
        t += dpp_mov<0x4E>(t);    // quad_perm [2,3,0,1]
        t += dpp_mov<0x141>(t);   // row_half_mirror
        t += dpp_mov<0x140>(t);   // row_mirror
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = read_lane(t, 16 * k);
    } else {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int nw = blockDim.x >> 6;
            T s = 0;
            for (int j = 0; j < nw; ++j) s += buf[k * 16 + j];
            v[k] = s;
        }
    }
    phase ^= 1;
}

// Raw buffer resource over [base, base + bytes) (gfx9 word 3: 32-bit untyped data).
// The hardware range check covers the lane offset (voffset) only, so callers put the
// whole byte offset there: a load at an offset >= bytes returns 0 without a memory
// access, and kBufferNone marks a lane that loads nothing.
// base and bytes must be the same in every lane of the wave.  Taking them through
// readfirstlane states that to the compiler: where it cannot prove it (arguments read from
// a device array, counters of a loop whose exit depends on a reduction) it would otherwise
// keep the descriptor in vector registers and wrap every load in a loop over lanes.
__device__ inline __amdgpu_buffer_rsrc_t buffer_rsrc(const void* base, unsigned bytes) {
    const unsigned long long p = reinterpret_cast<unsigned long long>(base);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)p);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(p >> 32));
    void* u = reinterpret_cast<void*>(((unsigned long long)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(u, 0, (int)__builtin_amdgcn_readfirstlane(bytes), 0x00020000);
}

constexpr unsigned kBufferNone = 0x80000000u;

template <typename S>
__device__ inline S buffer_load(__amdgpu_buffer_rsrc_t r, unsigned voff) {
    if constexpr (sizeof(S) == 16)
        return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b128(r, voff, 0, 0));
    else if constexpr (sizeof(S) == 8)
        return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b64(r, voff, 0, 0));
    else
        return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b32(r, voff, 0, 0));
}

// Raw buffer store of a 16-byte value at byte offset voff (dropped past the range).
__device__ inline void buffer_store16(__amdgpu_buffer_rsrc_t r, unsigned voff, double2 v) {
    using u32x4 = __attribute__((__vector_size__(4 * sizeof(unsigned)))) unsigned;
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, voff, 0, 0);
}

}  // namespace ppc

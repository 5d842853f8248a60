// Device-side building blocks shared by the gfx950 kernels of the hot path:
// the Philox4x64-10 counter generator, the FP64 squared distance, and
// deterministic wave/workgroup reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hpclust.h"

namespace hpc {

constexpr int kWave = 64;

enum : uint64_t { kTagSample = 0, kTagSeed = 1, kTagReseed = 2 };

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC 2011): ten rounds, each two
// 64x64->128-bit products of the even counter words with the published
// multipliers, XOR of the high halves with the odd words and the round key;
// the key advances by the published Weyl constants between rounds.
// Key (seed, tag), counter (block, sample_id, call_id, 0).
// ---------------------------------------------------------------------------
struct Words4 {
    uint64_t w[4];
};

__device__ __forceinline__ Words4 philox_block(uint64_t seed, uint64_t tag, uint64_t block,
                                               uint64_t sample_id, uint64_t call_id) {
    uint64_t c0 = block, c1 = sample_id, c2 = call_id, c3 = 0;
    uint64_t k0 = seed, k1 = tag;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B97F4A7C15ull;
            k1 += 0xBB67AE8584CAA73Bull;
        }
        const uint64_t p0_hi = __umul64hi(0xD2E7470EE14C6C93ull, c0);
        const uint64_t p0_lo = 0xD2E7470EE14C6C93ull * c0;
        const uint64_t p1_hi = __umul64hi(0xCA5A826395121157ull, c2);
        const uint64_t p1_lo = 0xCA5A826395121157ull * c2;
        const uint64_t n0 = p1_hi ^ c1 ^ k0;
        const uint64_t n2 = p0_hi ^ c3 ^ k1;
        c0 = n0;
        c1 = p1_lo;
        c2 = n2;
        c3 = p0_lo;
    }
    return Words4{{c0, c1, c2, c3}};
}

// floor(r * n / 2^64): uniform integer in [0, n).
__device__ __forceinline__ int64_t bounded_index(uint64_t r, uint64_t n) {
    return (int64_t)__umul64hi(r, n);
}

// (r >> 11) * 2^-53: uniform double in [0, 1).
__device__ __forceinline__ double unit_double(uint64_t r) {
    return (double)(r >> 11) * 0x1.0p-53;
}

// |x - c|^2 in FP64 from FP32 coordinates x and an FP64 centroid c (LDS,
// 16-byte aligned).  Used wherever a distance decides an index or enters an
// objective: the rounding is then ~1e-16 relative, far below any FP32
// effect.
template <int D>
__device__ __forceinline__ double sqdist64(const float (&x)[D], const double* __restrict__ c) {
    double a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int t = 0; t < D; t += 2) {
        const double2 cv = *reinterpret_cast<const double2*>(c + t);
        const double e0 = (double)x[t] - cv.x, e1 = (double)x[t + 1] - cv.y;
        a0 = __fma_rn(e0, e0, a0);
        a1 = __fma_rn(e1, e1, a1);
    }
    return a0 + a1;
}

// Load a zero-padded row of D floats (stride D, 16-byte aligned).
template <int D>
__device__ __forceinline__ void load_row(const float* __restrict__ p, float (&x)[D]) {
#pragma unroll
    for (int t = 0; t < D; t += 4) {
        const float4 v = *reinterpret_cast<const float4*>(p + t);
        x[t] = v.x;
        x[t + 1] = v.y;
        x[t + 2] = v.z;
        x[t + 3] = v.w;
    }
}

// ---------------------------------------------------------------------------
// Reductions.  XOR butterflies leave the identical value in every lane
// (IEEE addition is commutative), and wave partials are combined in wave
// order, so each result is a fixed function of the inputs and the launch
// shape.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Sum over the workgroup; every thread returns the same value.  red: LDS,
// NT/64 doubles.  Contains two barriers; call from uniform control flow.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (lane == 0) red[w] = v;
    __syncthreads();
    double tot = 0.0;
#pragma unroll
    for (int i = 0; i < NT / kWave; ++i) tot += red[i];
    __syncthreads();
    return tot;
}

// Data exchanged between workgroups, stored and loaded as relaxed
// device-scope atomics: on gfx950 these accesses are coherent across the
// XCDs' L2 caches by themselves, so an exchange needs no cache write-back or
// invalidation (which device-scope fences perform on the whole L2).  A
// writer waits for its stores to complete (wait_stores) before it signals.
__device__ __forceinline__ void store_dev(double* p, double v) {
    __hip_atomic_store(reinterpret_cast<unsigned long long*>(p),
                       (unsigned long long)__double_as_longlong(v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double load_dev(const double* p) {
    return __longlong_as_double((long long)__hip_atomic_load(
        reinterpret_cast<unsigned long long*>(const_cast<double*>(p)), __ATOMIC_RELAXED,
        __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ void store_dev(int32_t* p, int32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Wait until every memory access this wave issued has completed.
__device__ __forceinline__ void wait_stores() { __builtin_amdgcn_s_waitcnt(0); }

__device__ __forceinline__ bool is_nan_f(float v) { return v != v; }

// FP64 data in LDS addressed as such (32-bit addresses; a generic pointer
// into LDS keeps 64-bit address arithmetic), and its atomic add.
typedef __attribute__((address_space(3))) double lds_f64;
__device__ __forceinline__ lds_f64* as_lds(double* p) { return (lds_f64*)p; }
__device__ __forceinline__ void lds_add(lds_f64* p, double v) {
    __builtin_amdgcn_ds_atomic_fadd_f64(p, v);
}

// ---------------------------------------------------------------------------
// Exchange with lane l ^ 16 / l ^ 32 through the gfx950 row-swap
// instructions (VALU, no LDS round trip).  v_permlane16_swap(a, a) leaves,
// in every lane, the value of lane l ^ 16 in its first result for odd rows
// of 16 and in its second result for even rows; v_permlane32_swap(a, a)
// does the same for halves of 32 lanes.
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned xor16_u32(unsigned v) {
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return (threadIdx.x & 16) ? r[0] : r[1];
}
__device__ __forceinline__ unsigned xor32_u32(unsigned v) {
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return (threadIdx.x & 32) ? r[0] : r[1];
}
__device__ __forceinline__ float lane_xor(float v, int o) {
    const unsigned u = __float_as_uint(v);
    return __uint_as_float(o == 16 ? xor16_u32(u) : xor32_u32(u));
}
__device__ __forceinline__ int lane_xor(int v, int o) {
    const unsigned u = (unsigned)v;
    return (int)(o == 16 ? xor16_u32(u) : xor32_u32(u));
}
// Both values of the lane pair {l, l ^ 16} (O = 16) or {l, l ^ 32} (O = 32),
// the lower lane's first, identical in the two lanes of the pair: in the
// swap of v with itself the first result keeps the lower row's value and
// the second the upper row's.  A combination of the two is therefore the
// same in both lanes without a per-lane select.
template <int O>
__device__ __forceinline__ void lane_pair(unsigned v, unsigned& lo, unsigned& hi) {
    static_assert(O == 16 || O == 32, "pair distance");
    if constexpr (O == 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        lo = r[0];
        hi = r[1];
    } else {
        const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        lo = r[0];
        hi = r[1];
    }
}
// Sum over the lane pair (same value, same rounding, in both lanes).
template <int O>
__device__ __forceinline__ float pair_sum(float v) {
    unsigned lo, hi;
    lane_pair<O>(__float_as_uint(v), lo, hi);
    return __uint_as_float(lo) + __uint_as_float(hi);
}
template <int O>
__device__ __forceinline__ double pair_sum(double v) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    unsigned l0, h0, l1, h1;
    lane_pair<O>((unsigned)u, l0, h0);
    lane_pair<O>((unsigned)(u >> 32), l1, h1);
    const double lo = __longlong_as_double((long long)(((unsigned long long)l1 << 32) | l0));
    const double hi = __longlong_as_double((long long)(((unsigned long long)h1 << 32) | h0));
    return lo + hi;
}
__device__ __forceinline__ double lane_xor(double v, int o) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)u, hi = (unsigned)(u >> 32);
    const unsigned nlo = o == 16 ? xor16_u32(lo) : xor32_u32(lo);
    const unsigned nhi = o == 16 ? xor16_u32(hi) : xor32_u32(hi);
    return __longlong_as_double((long long)(((unsigned long long)nhi << 32) | nlo));
}

}  // namespace hpc

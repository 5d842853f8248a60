// Device-side building blocks shared by the gfx950 kernels of the hot path:
// the Philox4x64-10 counter generator, the FP32 squared distance, and
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

// ---------------------------------------------------------------------------
// Squared distance |x - c|^2 in FP32 (Eq. (1)).  x lives in registers, c in
// LDS or global memory (16-byte aligned, D floats, zero-padded beyond d).
// Four interleaved accumulators with explicit FMAs: the rounding sequence is
// fixed by this code, so every kernel that calls it on the same operands
// gets bit-identical results.
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ float sqdist(const float (&x)[D], const float* __restrict__ c) {
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
#pragma unroll
    for (int t = 0; t < D; t += 4) {
        const float4 cv = *reinterpret_cast<const float4*>(c + t);
        const float e0 = x[t] - cv.x, e1 = x[t + 1] - cv.y, e2 = x[t + 2] - cv.z,
                    e3 = x[t + 3] - cv.w;
        a0 = __fmaf_rn(e0, e0, a0);
        a1 = __fmaf_rn(e1, e1, a1);
        a2 = __fmaf_rn(e2, e2, a2);
        a3 = __fmaf_rn(e3, e3, a3);
    }
    return (a0 + a1) + (a2 + a3);
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

// Certificate of an FP32 screening argmin.  The screened distance of x to
// centroid j is sqdist<D>(x, fl32(c_j)); relative to the exact distance to
// the FP64 centroid c_j its error is at most g*dist + 2r*sqrt(dist) + r^2,
// with g = (d + 8) 2^-24 bounding the FP32 arithmetic of sqdist (d
// subtractions, d/4 FMAs per accumulator, three adds) and r = 2^-24 max|c_j|
// bounding the rounding of the centroid to FP32.  The screening winner is
// the exact argmin whenever the gap to the runner-up exceeds both error
// bounds; `tau` = 4g (a factor 2 of slack for the rounding of this test).
__device__ __forceinline__ bool screen_certified(float b1, float b2, float tau, float rmax) {
    if (!(b2 < __builtin_huge_valf())) return true;  // a single candidate
    const float sb2 = sqrtf(b2);
    return (b2 - b1) > tau * b2 + 5.f * rmax * sb2 + 4.f * rmax * rmax;
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

__device__ __forceinline__ bool is_nan_f(float v) { return v != v; }

}  // namespace hpc

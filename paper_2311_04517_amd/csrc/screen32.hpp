// Nearest-centroid screening with 32 x 32 matrix-core tiles, for rows of up
// to 32 coordinates.
//
// The same screening, certificate and FP64 re-decision as mfma_screen.hpp,
// on tiles of 32 points and blocks of 32 centroids:
//   FP32   : v_mfma_f32_32x32x2f32    (one k-slice of 2 per instruction)
//   BF16   : v_mfma_f32_32x32x16_bf16 (16-wide k-slice)
//   BF16x3 : the same instruction three times per k-slice on the two-term
//            split of each operand (hi.hi + lo.hi + hi.lo)
// The error bounds of mfma_screen.hpp hold unchanged: they depend on the
// operand roundings and on the number of products accumulated per score,
// not on the tile shape.
//
// Lane layout (32x32 family on gfx950, wave of 64): lane l supplies A row
// l%32 and B column l%32 with the k-values of lane half h = l/32, and
// receives rows 8(i/4) + 4h + i%4, i < 16, of column l%32.  Hence a point
// lives in two lanes (l and l + 32), each with half of its coordinates
// (DH = D/2; dims [h DH, (h+1) DH), permuted consistently in A and B), and
// each lane gets sixteen scores of its point per block.  Against the 16 x
// 16 tiles this halves the lanes a point's three best keys are merged over
// (one exchange instead of two) and the lanes that repeat the per-point
// certificate, norm and bookkeeping; the key insertions per score are the
// same.
#pragma once

#include "common.hpp"
#include "mfma_screen.hpp"

namespace hpc {

typedef float f32x16 __attribute__((ext_vector_type(16)));

template <int D>
struct Lay32 {
    static_assert(D == 8 || D == 16 || D == 32, "32-point tiles serve d <= 32");
    static constexpr int DH = D / 2;         // coordinates per lane
    static constexpr int KC = (DH + 7) / 8;  // BF16 k-chunks of 8 per lane
    static constexpr int CS = D + 1;         // FP64 row stride, as Lay<D>
};

// Row of accumulator element i in lane half h.
__device__ __forceinline__ constexpr int acc_row(int i, int h) {
    return 8 * (i >> 2) + 4 * h + (i & 3);
}

// Bytes of the A-operand tables for nb blocks of 32 centroids.
template <int D, int PREC>
__host__ __device__ constexpr size_t aop32_bytes(int nb) {
    return PREC == kPrecF32 ? (size_t)nb * Lay32<D>::DH * 64 * 4
                            : (size_t)nb * Lay32<D>::KC * 64 * 16 * (PREC == kPrecBF16x3 ? 2 : 1);
}

// A operands (-2 c rounded to the MFMA type, zero for padding rows and
// coordinates) and the score bias |c|^2 (+inf for padding and NaN rows) for
// nb blocks of 32 centroids, from the FP64 rows (stride CS).
template <int D, int PREC, int NT>
__device__ void build_operands32(const double* __restrict__ C64, int k, int d, int nb,
                                 void* __restrict__ aop, float* __restrict__ nrm) {
    constexpr int DH = Lay32<D>::DH, KC = Lay32<D>::KC, CS = Lay32<D>::CS;
    for (int j = threadIdx.x; j < nb * 32; j += NT) {
        float v = __builtin_huge_valf();
        if (j < k && C64[j * CS] == C64[j * CS]) {
            double n2 = 0.0;
            for (int t = 0; t < d; ++t) n2 = __fma_rn(C64[j * CS + t], C64[j * CS + t], n2);
            v = (float)n2;
        }
        nrm[j] = v;
    }
    if (PREC == kPrecF32) {
        float* a = static_cast<float*>(aop);
        for (int e = threadIdx.x; e < nb * DH * 64; e += NT) {
            const int blk = e / (DH * 64), q = (e / 64) % DH, l = e % 64;
            const int j = blk * 32 + (l & 31), t = (l >> 5) * DH + q;
            float v = 0.f;
            if (j < k && C64[j * CS] == C64[j * CS]) v = -2.f * (float)C64[j * CS + t];
            a[e] = v;
        }
    } else {
        // BF16x3: the low parts follow the high parts as a second table
        __bf16* a = static_cast<__bf16*>(aop);
        const int n = nb * KC * 64 * 8;
        for (int e = threadIdx.x; e < n; e += NT) {
            const int v8 = e & 7, l = (e >> 3) & 63, kc = (e >> 9) % KC, blk = (e >> 9) / KC;
            const int j = blk * 32 + (l & 31), q = kc * 8 + v8, t = (l >> 5) * DH + q;
            float v = 0.f;
            if (q < DH && j < k && C64[j * CS] == C64[j * CS]) v = -2.f * (float)C64[j * CS + t];
            const __bf16 hi = (__bf16)v;
            a[e] = hi;
            if (PREC == kPrecBF16x3) a[n + e] = (__bf16)(v - (float)hi);
        }
    }
}

// This lane's half of point row p (row stride D floats, 16-byte aligned,
// zero padded).
template <int D>
__device__ __forceinline__ void load_half(const float* __restrict__ row, int h,
                                          float (&xh)[Lay32<D>::DH]) {
    constexpr int DH = Lay32<D>::DH;
    const float* p = row + h * DH;
#pragma unroll
    for (int t = 0; t < DH; t += 4) {
        const float4 v = *reinterpret_cast<const float4*>(p + t);
        xh[t] = v.x;
        xh[t + 1] = v.y;
        xh[t + 2] = v.z;
        xh[t + 3] = v.w;
    }
}

// |x|^2 of this lane's point (same value in its two lanes).
template <int D>
__device__ __forceinline__ float point_norm2_32(const float (&xh)[Lay32<D>::DH]) {
    float s = 0.f;
#pragma unroll
    for (int t = 0; t < Lay32<D>::DH; ++t) s = __fmaf_rn(xh[t], xh[t], s);
    return pair_sum<32>(s);
}

// Scores (|c_j|^2 - 2 x.c_j, screened) of this lane's point against block
// blk: element i is row blk*32 + acc_row(i, h).
template <int D, int PREC>
__device__ __forceinline__ f32x16 block_scores32(const float (&xh)[Lay32<D>::DH],
                                                 const void* __restrict__ aop,
                                                 const float* __restrict__ nrm, int nb, int blk) {
    constexpr int DH = Lay32<D>::DH, KC = Lay32<D>::KC;
    const int lane = threadIdx.x & 63, h = lane >> 5;
    f32x16 acc;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const f32x4 b = *reinterpret_cast<const f32x4*>(nrm + blk * 32 + 8 * q + 4 * h);
        acc[4 * q] = b[0];
        acc[4 * q + 1] = b[1];
        acc[4 * q + 2] = b[2];
        acc[4 * q + 3] = b[3];
    }
    if constexpr (PREC == kPrecF32) {
        const float* a = static_cast<const float*>(aop);
#pragma unroll
        for (int q = 0; q < DH; ++q)
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[(blk * DH + q) * 64 + lane], xh[q], acc, 0,
                                                       0, 0);
    } else {
        const bf16x8* a = static_cast<const bf16x8*>(aop);
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
            bf16x8 xb, xl;
#pragma unroll
            for (int v = 0; v < 8; v += 2) {
                const int q = kc * 8 + v;
                const float x0 = q < DH ? xh[q < DH ? q : 0] : 0.f;
                const float x1 = q + 1 < DH ? xh[q + 1 < DH ? q + 1 : 0] : 0.f;
                if constexpr (PREC == kPrecBF16x3) {
                    split2(x0, x1, xb, xl, v);
                } else {
                    xb[v] = (__bf16)x0;
                    xb[v + 1] = (__bf16)x1;
                }
            }
            const int o = (blk * KC + kc) * 64 + lane;
            if constexpr (PREC == kPrecBF16x3) {
                const bf16x8* al = a + nb * KC * 64;
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[o], xb, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[o], xl, acc, 0, 0, 0);
            }
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[o], xb, acc, 0, 0, 0);
        }
    }
    return acc;
}

// The three smallest keys of this lane's point over all nb blocks, merged
// over its two lanes (identical in both).  h: the point's shift from
// screen_shift.
template <int D, int PREC>
__device__ __forceinline__ Top3 screen_tile32(const float (&xh)[Lay32<D>::DH],
                                              const void* __restrict__ aop,
                                              const float* __restrict__ nrm, int nb, float h,
                                              unsigned kmask) {
    const int hh = (threadIdx.x & 63) >> 5;
    Top3 t{~0u, ~0u, ~0u};
    for (int blk = 0; blk < nb; ++blk) {
        const f32x16 acc = block_scores32<D, PREC>(xh, aop, nrm, nb, blk);
        const unsigned base = (unsigned)(blk * 32 + 4 * hh);
#pragma unroll
        for (int i = 0; i < 16; ++i)
            top3_insert(t, screen_key(acc[i] + h, kmask, base + (unsigned)acc_row(i, 0)));
    }
    top3_merge<32>(t);
    return t;
}

// FP64 |x - c|^2 of this lane's point to the FP64 row c, summed over its two
// lanes (same value in both).  `fresh`: the coordinates are converted at
// each call (see quarter_dist64_fresh).
template <int D, bool fresh>
__device__ __forceinline__ double half_dist64(const float (&xh)[Lay32<D>::DH],
                                              const double* __restrict__ c) {
    constexpr int DH = Lay32<D>::DH;
    const int h = (threadIdx.x & 63) >> 5;
    double p = 0.0;
#pragma unroll
    for (int t = 0; t < DH; ++t) {
        float x = xh[t];
        if constexpr (fresh) asm volatile("" : "+v"(x));
        const double e = (double)x - c[h * DH + t];
        p = __fma_rn(e, e, p);
    }
    return pair_sum<32>(p);
}

// This lane's FP64 share of |x - c|^2 (its DH coordinates).
template <int D>
__device__ __forceinline__ double half_part64(const float (&xh)[Lay32<D>::DH],
                                              const double* __restrict__ c) {
    constexpr int DH = Lay32<D>::DH;
    const int h = (threadIdx.x & 63) >> 5;
    double p = 0.0;
#pragma unroll
    for (int t = 0; t < DH; ++t) {
        const double e = (double)xh[t] - c[h * DH + t];
        p = __fma_rn(e, e, p);
    }
    return p;
}

// rescan_rows (mfma_screen.hpp) on the 32 x 32 layout: bit 32 h' + p' of
// keep[i] is row acc_row(i, h') of point p'.
template <int D, int PREC>
__device__ __forceinline__ void rescan_rows32(const float (&xh)[Lay32<D>::DH], bool full, float q1,
                                              float e25, float qscale, const void* __restrict__ aop,
                                              const float* __restrict__ nrm, int nb, float h,
                                              unsigned kmask, const double* __restrict__ C64,
                                              double& best, int& bj) {
    constexpr int CS = Lay32<D>::CS;
    const int p = threadIdx.x & 31;
    for (int blk = 0; blk < nb; ++blk) {
        const f32x16 acc = block_scores32<D, PREC>(xh, aop, nrm, nb, blk);
        unsigned long long keep[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const unsigned key = screen_key(acc[i] + h, kmask, 0u);
            const float q = key_value(key, kmask);
            keep[i] = __ballot(full && key < 0x7F800000u && !((q - q1) > e25 + qscale * q));
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            unsigned long long mk = keep[i];
            while (mk) {
                const int hh = __builtin_ctzll(mk) >> 5;
                const unsigned bits = (unsigned)(mk >> (32 * hh));
                mk &= ~(0xFFFFFFFFull << (32 * hh));
                const int j = blk * 32 + acc_row(i, hh);
                const double v = half_dist64<D, true>(xh, C64 + j * CS);
                if (((bits >> p) & 1u) && (v < best || (v == best && j < bj))) {
                    best = v;
                    bj = j;
                }
            }
        }
    }
}

// redecide64 (mfma_screen.hpp) on the 32 x 32 layout.
template <int D, int PREC>
__device__ __forceinline__ int redecide64_32(const float (&xh)[Lay32<D>::DH], const Top3& t,
                                             bool redo, bool pair_ok, int a1, int a2,
                                             const double* __restrict__ C64,
                                             const void* __restrict__ aop,
                                             const float* __restrict__ nrm, int nb, float h,
                                             unsigned kmask, float qscale, float xnorm, float ea,
                                             float eb) {
    constexpr int CS = Lay32<D>::CS;
    int am = a1;
    if (!__any(redo)) return am;
    const double v1 = half_dist64<D, false>(xh, C64 + a1 * CS);
    const double v2 = half_dist64<D, false>(xh, C64 + a2 * CS);
    const bool take2 = v2 < v1 || (v2 == v1 && a2 < a1);
    if (redo && pair_ok && take2) am = a2;
    const bool full = redo && !pair_ok;
    if (!__any(full)) return am;
    double best = take2 ? v2 : v1;
    int bj = take2 ? a2 : a1;
    rescan_rows32<D, PREC>(xh, full, key_value(t.t1, kmask), 2.5f * (ea * xnorm + eb), qscale, aop,
                           nrm, nb, h, kmask, C64, best, bj);
    return full ? bj : am;
}

}  // namespace hpc

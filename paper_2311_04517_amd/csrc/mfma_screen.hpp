// Nearest-centroid screening on the matrix cores of gfx950.
//
// The distance |x - c_j|^2 = |x|^2 + s_j with score s_j = |c_j|^2 - 2 x.c_j;
// the cross term x.c_j over a tile of 16 points and blocks of 16 centroids
// is the one dense contraction of the method and runs on MFMA:
//   FP32   : v_mfma_f32_16x16x4_f32   (one k-slice of 4 per instruction)
//   BF16   : v_mfma_f32_16x16x32_bf16 (32-wide k-slice, FP32 accumulation)
//   BF16x3 : the same instruction three times per k-slice on a two-term
//            split of each operand, v = v_hi + v_lo (v_hi = bf16(v), v_lo =
//            bf16(v - v_hi); v - v_hi is exact in FP32): hi.hi + lo.hi +
//            hi.lo, leaving out lo.lo, for close to FP32 accuracy at a
//            fraction of the FP32 matrix rate's cost
// A = -2 c (centroids x dims), B = x^T (dims x points), the accumulator
// starts at |c_j|^2, so the MFMA result is s_j directly.
//
// Lane layout (16x16 MFMA family on gfx950, wave of 64): lane l supplies A
// row l%16 and B column l%16, the k-values of lane group g = l/16, and
// receives rows 4g..4g+3 of column l%16.  Hence a lane owns point l%16 of
// the tile and dims [g*DL, (g+1)*DL) of that point (DL = D/4; the dims are
// permuted consistently in A and B, which leaves the contraction
// unchanged), and gets the scores of centroids 4g..4g+3 of each block.  The
// four lanes of a point merge their three best with two XOR exchanges.
//
// Keys.  Each screened score becomes the distance estimate v_j = fl(s~_j +
// h) with h = fl(|x|~^2 + b): |x|~^2 is the FP32 norm of the point and b =
// 1.25 E(x) + 2^-16 |x|~^2 bounds the screening error (below) and the
// norm's rounding (under 2^-18 |x|^2 for d <= 128), so that v_j >= +0
// without a clamp; h is the same for every j of the point.  The NB low
// mantissa bits of v_j are replaced by j (2^NB >= padded k).  For
// non-negative floats the bit patterns order like the values, so the three
// smallest keys -- found with integer min/max only -- are the three
// smallest quantised estimates with their indices.  Padding rows (score
// +inf) give keys at or above 0x7F800000, above every finite key.
//
// Certificate.  Let E(x) bound |s~_j - s_j| for the screened score, s_j the
// exact score of the FP64 centroid; E(x) = alpha |x| cmax + beta cmax^2 with
// (u = 2^-24, u_b = 2^-8 plus the FP32-to-BF16 double rounding)
//   FP32   : alpha = (4d + 10) u          beta = (2d + 6) u
//   BF16   : alpha = 4 u_b + 2 u_b^2 + (4d + 10) u (1 + u_b)^2   beta as FP32
//   BF16x3 : alpha = 8 u_b^2 + (12d + 10) u (1 + u_b)^5          beta = (6d + 6) u
// i.e. the rounding of the operands to the MFMA input type, plus twice the
// classical accumulation bound of d + 1 FP32 additions (the factor two
// leaves room for the matrix unit's internal summation order), plus the
// rounding of |c|^2 to FP32.  For BF16x3: per coordinate the split leaves
// |x - x_hi - x_lo| <= u_b^2 |x| and, for a = -2c rounded to FP32 first,
// |a - a_hi - a_lo| <= (u + u_b^2 (1 + u)) |a|; with the omitted lo.lo
// product (<= u_b^2 (1 + u_b)^2 (1 + u) |a||x|) the represented cross term
// is off by about (3 u_b^2 + u) |a||x| (higher-order terms included, below
// 3.03 u_b^2 |a||x|), bounded by 4 u_b^2 |a||x| (Cauchy-Schwarz over
// coordinates, |a| = 2|c|); the accumulation is over 3d exact products
// whose magnitudes sum to at most (1 + u)(1 + u_b)^4 |a||x|.  The quantised key value q_j satisfies
// q_j <= v_j < q_j (1 + 2^(NB-23)), and fl() adds a relative 2^-24; h,
// common to all j, cancels between them (its share of q_j only enlarges
// the right-hand side of the test below).  Hence with q_1 <=
// q_2 the two best keys, every j other than the winner has s_j > s_winner
// whenever  q_2 - q_1 > 2E + 2^(NB-22) q_1 + 2^-23 (q_1 + q_2),  and the
// test below uses the stronger  q_2 - q_1 > 2.5 E + 2^(NB-20) q_2  (the
// left side grows faster in q_j than the right, so the runner-up is the
// binding case).  The same test on the third key shows the exact argmin is
// one of the two best, and on any row j that j is not the argmin.
#pragma once

#include <type_traits>

#include "common.hpp"

namespace hpc {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));

// BF16 head and tail of two FP32 values: the head is x rounded to BF16
// (nearest, ties to even), the tail x minus the head (exact in FP32) rounded
// to BF16.  The heads are
// converted as one pair and widened back to FP32 by shifting and masking
// the packed pair, which spares a second conversion per value.
// Lanes v and v + 1 of h and t receive those of x0 and x1.
__device__ __forceinline__ void split2(float x0, float x1, bf16x8& h, bf16x8& t, int v) {
    const bf16x2v hp = __builtin_convertvector((f32x2v){x0, x1}, bf16x2v);
    const unsigned u = __builtin_bit_cast(unsigned, hp);
    const float w0 = __uint_as_float(u << 16), w1 = __uint_as_float(u & 0xffff0000u);
    const bf16x2v tp = __builtin_convertvector((f32x2v){x0 - w0, x1 - w1}, bf16x2v);
    h[v] = hp[0];
    h[v + 1] = hp[1];
    t[v] = tp[0];
    t[v + 1] = tp[1];
}

enum : int { kPrecF32 = 0, kPrecBF16 = 1, kPrecBF16x3 = 2 };

template <int D>
struct Lay {
    static constexpr int DL = D / 4;              // dims per lane
    static constexpr int KC = (DL + 7) / 8;       // BF16 k-chunks of 8 per lane
    // Row stride (in doubles) of FP64 centroid rows and per-cluster sums in
    // LDS: odd, so that the rows of different centroids start in different
    // LDS banks (a stride of D doubles puts every row on the same banks and
    // serialises the per-lane row reads and the update atomics).
    static constexpr int CS = D + 1;
};

// Bytes of the A-operand buffer for nblk blocks of 16 centroids.
template <int D, int PREC>
__host__ __device__ constexpr size_t aop_bytes(int nblk) {
    return PREC == kPrecF32 ? (size_t)nblk * Lay<D>::DL * 64 * 4
                            : (size_t)nblk * Lay<D>::KC * 64 * 16 * (PREC == kPrecBF16x3 ? 2 : 1);
}

template <int PREC>
__host__ __device__ inline void screen_coeffs(int d, double* alpha, double* beta) {
    const double u = 0x1.0p-24, ub = 0x1.0p-8 + 0x1.0p-24;
    const double acc = (4.0 * d + 10.0) * u;
    *beta = (2.0 * d + 6.0) * u;
    *alpha = PREC == kPrecF32 ? acc : 4.0 * ub + 2.0 * ub * ub + acc * (1.0 + ub) * (1.0 + ub);
    if (PREC == kPrecBF16x3) {
        const double g = 1.0 + ub;
        *beta = (6.0 * d + 6.0) * u;
        *alpha = 8.0 * ub * ub + (12.0 * d + 10.0) * u * g * g * g * g * g;
    }
}

// Fill the A operands (-2 c, rounded to the MFMA type; zero for padding
// rows) and the score bias |c|^2 (FP32; +inf for padding rows) from the
// FP64 centroids (row stride Lay<D>::CS).  Rows whose first coordinate is
// NaN are treated as padding (never chosen).  All threads participate.
template <int D, int PREC, int NT>
__device__ void build_operands(const double* __restrict__ C64, int k, int d, int nblk,
                               void* __restrict__ aop, float* __restrict__ nrm) {
    constexpr int DL = Lay<D>::DL, KC = Lay<D>::KC, CS = Lay<D>::CS;
    for (int j = threadIdx.x; j < nblk * 16; j += NT) {
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
        for (int e = threadIdx.x; e < nblk * DL * 64; e += NT) {
            const int blk = e / (DL * 64), q = (e / 64) % DL, l = e % 64;
            const int j = blk * 16 + (l & 15), t = (l >> 4) * DL + q;
            float v = 0.f;
            if (j < k && C64[j * CS] == C64[j * CS]) v = -2.f * (float)C64[j * CS + t];
            a[e] = v;
        }
    } else {
        // BF16x3: the low parts follow the high parts as a second table
        __bf16* a = static_cast<__bf16*>(aop);
        const int n = nblk * KC * 64 * 8;
        for (int e = threadIdx.x; e < n; e += NT) {
            const int v8 = e & 7, l = (e >> 3) & 63, kc = (e >> 9) % KC, blk = (e >> 9) / KC;
            const int j = blk * 16 + (l & 15), q = kc * 8 + v8, t = (l >> 4) * DL + q;
            float v = 0.f;
            if (q < DL && j < k && C64[j * CS] == C64[j * CS]) v = -2.f * (float)C64[j * CS + t];
            const __bf16 hi = (__bf16)v;
            a[e] = hi;
            if (PREC == kPrecBF16x3) a[n + e] = (__bf16)(v - (float)hi);
        }
    }
}

// Load this lane's DL dims of point row p (row stride D floats, 16-byte
// aligned rows, zero padded).
template <int D>
__device__ __forceinline__ void load_quarter(const float* __restrict__ row, int g,
                                             float (&xq)[Lay<D>::DL]) {
    constexpr int DL = Lay<D>::DL;
    const float* p = row + g * DL;
    if constexpr (DL % 4 == 0) {
#pragma unroll
        for (int t = 0; t < DL; t += 4) {
            const float4 v = *reinterpret_cast<const float4*>(p + t);
            xq[t] = v.x;
            xq[t + 1] = v.y;
            xq[t + 2] = v.z;
            xq[t + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int t = 0; t < DL; t += 2) {
            const float2 v = *reinterpret_cast<const float2*>(p + t);
            xq[t] = v.x;
            xq[t + 1] = v.y;
        }
    }
}

// The three smallest screening keys of a point, ascending.
struct Top3 {
    unsigned t1, t2, t3;
};

// Key of centroid j: v (non-negative, see screen_shift) with the low bits
// under `kmask` set to j.
__device__ __forceinline__ unsigned screen_key(float v, unsigned kmask, unsigned j) {
    return (__float_as_uint(v) & ~kmask) | j;
}

// h = |x|~^2 + 1.25 E(x) + 2^-16 |x|~^2 (see Keys above): every distance
// estimate fl(s~_j + h) is >= +0.  ea, eb as in certified().
__device__ __forceinline__ float screen_shift(float xn2, float xnorm, float ea, float eb) {
    return xn2 + (1.25f * __fmaf_rn(ea, xnorm, eb) + 0x1.0p-16f * xn2);
}

// Median of three (one v_med3_u32).
__device__ __forceinline__ unsigned umed3(unsigned a, unsigned b, unsigned c) {
    return max(min(a, b), min(max(a, b), c));
}

// Insert a key into the ascending triple: the new i-th smallest of
// {t1, t2, t3, key} is min(t1, key), med3(t1, t2, key), med3(t2, t3, key).
__device__ __forceinline__ void top3_insert(Top3& t, unsigned key) {
    const unsigned n3 = umed3(t.t2, t.t3, key);
    const unsigned n2 = umed3(t.t1, t.t2, key);
    t.t1 = min(t.t1, key);
    t.t2 = n2;
    t.t3 = n3;
}

// The three smallest of two ascending triples a and b: the r-th smallest of
// their union is the minimum over i + j = r of max(a_i, b_j) (a_0 = b_0 =
// -inf), i.e. min(a1, b1); min(a2, b2, max(a1, b1)); min(a3, b3, max(a2,
// b1), max(a1, b2)).
__device__ __forceinline__ Top3 top3_union(const Top3& a, const Top3& b) {
    Top3 t;
    t.t1 = min(a.t1, b.t1);
    t.t2 = min(min(a.t2, b.t2), max(a.t1, b.t1));
    t.t3 = min(min(min(a.t3, b.t3), max(a.t2, b.t1)), max(a.t1, b.t2));
    return t;
}

// Merge with the lane at XOR distance O: both lanes combine the same two
// triples (the lower lane's and the upper lane's), so they end with the
// same result.
template <int O>
__device__ __forceinline__ void top3_merge(Top3& t) {
    Top3 lo, hi;
    lane_pair<O>(t.t1, lo.t1, hi.t1);
    lane_pair<O>(t.t2, lo.t2, hi.t2);
    lane_pair<O>(t.t3, lo.t3, hi.t3);
    t = top3_union(lo, hi);
}

__device__ __forceinline__ unsigned key_index(unsigned key, unsigned kmask) { return key & kmask; }
__device__ __forceinline__ float key_value(unsigned key, unsigned kmask) {
    return __uint_as_float(key & ~kmask);
}

// Index bits for nblk blocks of 16 centroids, and the certificate's
// quantisation factor 2^(NB - 20).
__device__ __forceinline__ void key_params(int nblk, unsigned* kmask, float* qscale) {
    int nb = 4;
    while ((1 << nb) < nblk * 16) ++nb;
    *kmask = (1u << nb) - 1u;
    *qscale = __builtin_ldexpf(1.0f, nb - 20);
}

// BF16x3 B operands: this lane's coordinates as x_hi = bf16(x) and x_lo =
// bf16(x - x_hi) (the difference is exact in FP32), in the k-chunk layout
// of the BF16 operands (zero past DL).
template <int D>
__device__ __forceinline__ void split_point(const float (&xq)[Lay<D>::DL],
                                            bf16x8 (&xh)[Lay<D>::KC], bf16x8 (&xl)[Lay<D>::KC]) {
    constexpr int DL = Lay<D>::DL, KC = Lay<D>::KC;
#pragma unroll
    for (int kc = 0; kc < KC; ++kc)
#pragma unroll
        for (int v = 0; v < 8; v += 2) {
            const int q = kc * 8 + v;
            const float x0 = q < DL ? xq[q < DL ? q : 0] : 0.f;
            const float x1 = q + 1 < DL ? xq[q + 1 < DL ? q + 1 : 0] : 0.f;
            split2(x0, x1, xh[kc], xl[kc], v);
        }
}

// Keys of this lane's point against all nblk*16 centroids; returns the
// merged three best (identical in the point's four lanes).  h: the point's
// shifted norm from screen_shift.  PAIRED takes the blocks in pairs with
// their MFMA chains interleaved, so that one block's dependent products do
// not wait on each other alone (for kernels at two waves per SIMD, where
// little else hides that latency, and with the registers for a second
// accumulator); the keys are inserted in block order either way, so the
// result is the same.
template <int D, int PREC, bool PAIRED = false>
__device__ __forceinline__ Top3 screen_tile(const float (&xq)[Lay<D>::DL],
                                            const void* __restrict__ aop,
                                            const float* __restrict__ nrm, int nblk, float h,
                                            unsigned kmask) {
    if constexpr (!PAIRED) {
        constexpr int DL = Lay<D>::DL, KC = Lay<D>::KC;
        const int lane = threadIdx.x & 63, g = lane >> 4;
        Top3 t{~0u, ~0u, ~0u};
        if constexpr (PREC == kPrecF32) {
            const float* a = static_cast<const float*>(aop);
            for (int blk = 0; blk < nblk; ++blk) {
                f32x4 acc = *reinterpret_cast<const f32x4*>(nrm + blk * 16 + 4 * g);
#pragma unroll
                for (int q = 0; q < DL; ++q)
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[(blk * DL + q) * 64 + lane], xq[q],
                                                               acc, 0, 0, 0);
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    top3_insert(t, screen_key(acc[r] + h, kmask, (unsigned)(blk * 16 + 4 * g + r)));
            }
        } else if constexpr (PREC == kPrecBF16x3) {
            bf16x8 xh[KC], xl[KC];
            split_point<D>(xq, xh, xl);
            const bf16x8* a = static_cast<const bf16x8*>(aop);
            const bf16x8* al = a + nblk * KC * 64;
            for (int blk = 0; blk < nblk; ++blk) {
                f32x4 acc = *reinterpret_cast<const f32x4*>(nrm + blk * 16 + 4 * g);
#pragma unroll
                for (int kc = 0; kc < KC; ++kc) {
                    const int o = (blk * KC + kc) * 64 + lane;
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[o], xh[kc], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[o], xl[kc], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[o], xh[kc], acc, 0, 0, 0);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    top3_insert(t, screen_key(acc[r] + h, kmask, (unsigned)(blk * 16 + 4 * g + r)));
            }
        } else {
            bf16x8 xb[KC];
#pragma unroll
            for (int kc = 0; kc < KC; ++kc)
#pragma unroll
                for (int v = 0; v < 8; ++v) {
                    const int q = kc * 8 + v;
                    xb[kc][v] = (__bf16)(q < DL ? xq[q < DL ? q : 0] : 0.f);
                }
            const bf16x8* a = static_cast<const bf16x8*>(aop);
            for (int blk = 0; blk < nblk; ++blk) {
                f32x4 acc = *reinterpret_cast<const f32x4*>(nrm + blk * 16 + 4 * g);
#pragma unroll
                for (int kc = 0; kc < KC; ++kc)
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[(blk * KC + kc) * 64 + lane], xb[kc],
                                                                  acc, 0, 0, 0);
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    top3_insert(t, screen_key(acc[r] + h, kmask, (unsigned)(blk * 16 + 4 * g + r)));
            }
        }
        top3_merge<16>(t);
        top3_merge<32>(t);
        return t;
    } else {
        constexpr int DL = Lay<D>::DL, KC = Lay<D>::KC;
        constexpr int PAIR = PAIRED ? 2 : 1;
        const int lane = threadIdx.x & 63, g = lane >> 4;
        Top3 t{~0u, ~0u, ~0u};
        bf16x8 xh[KC], xl[KC];
        if constexpr (PREC == kPrecBF16x3) {
            split_point<D>(xq, xh, xl);
        } else if constexpr (PREC == kPrecBF16) {
#pragma unroll
            for (int kc = 0; kc < KC; ++kc)
#pragma unroll
                for (int v = 0; v < 8; ++v) {
                    const int q = kc * 8 + v;
                    xh[kc][v] = (__bf16)(q < DL ? xq[q < DL ? q : 0] : 0.f);
                }
        }
        // the screened scores of NB consecutive blocks from blk on, their MFMA
        // chains interleaved
        auto scores = [&](int blk, auto nbc, f32x4 (&acc)[decltype(nbc)::value]) {
            constexpr int NB = decltype(nbc)::value;
#pragma unroll
            for (int u = 0; u < NB; ++u)
                acc[u] = *reinterpret_cast<const f32x4*>(nrm + (blk + u) * 16 + 4 * g);
            if constexpr (PREC == kPrecF32) {
                const float* a = static_cast<const float*>(aop);
#pragma unroll
                for (int q = 0; q < DL; ++q)
#pragma unroll
                    for (int u = 0; u < NB; ++u)
                        acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                            a[((blk + u) * DL + q) * 64 + lane], xq[q], acc[u], 0, 0, 0);
            } else if constexpr (PREC == kPrecBF16x3) {
                const bf16x8* a = static_cast<const bf16x8*>(aop);
                const bf16x8* al = a + nblk * KC * 64;
#pragma unroll
                for (int kc = 0; kc < KC; ++kc) {
#pragma unroll
                    for (int u = 0; u < NB; ++u) {
                        const int o = ((blk + u) * KC + kc) * 64 + lane;
                        acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[o], xh[kc], acc[u], 0, 0, 0);
                    }
#pragma unroll
                    for (int u = 0; u < NB; ++u) {
                        const int o = ((blk + u) * KC + kc) * 64 + lane;
                        acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[o], xl[kc], acc[u], 0, 0, 0);
                    }
#pragma unroll
                    for (int u = 0; u < NB; ++u) {
                        const int o = ((blk + u) * KC + kc) * 64 + lane;
                        acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[o], xh[kc], acc[u], 0, 0, 0);
                    }
                }
            } else {
                const bf16x8* a = static_cast<const bf16x8*>(aop);
#pragma unroll
                for (int kc = 0; kc < KC; ++kc)
#pragma unroll
                    for (int u = 0; u < NB; ++u)
                        acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            a[((blk + u) * KC + kc) * 64 + lane], xh[kc], acc[u], 0, 0, 0);
            }
        };
        int blk = 0;
        if constexpr (PAIR == 2) {
            for (; blk + 1 < nblk; blk += 2) {
                f32x4 acc[2];
                scores(blk, std::integral_constant<int, 2>{}, acc);
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        top3_insert(t, screen_key(acc[u][r] + h, kmask,
                                                  (unsigned)((blk + u) * 16 + 4 * g + r)));
            }
        }
        for (; blk < nblk; ++blk) {
            f32x4 acc[1];
            scores(blk, std::integral_constant<int, 1>{}, acc);
#pragma unroll
            for (int r = 0; r < 4; ++r)
                top3_insert(t, screen_key(acc[0][r] + h, kmask, (unsigned)(blk * 16 + 4 * g + r)));
        }
        top3_merge<16>(t);
        top3_merge<32>(t);
        return t;
    }
}

// |x|^2 of this lane's point (same value in its four lanes).  Used by the
// key shift and the certificate, whose factors cover its rounding.
template <int D>
__device__ __forceinline__ float point_norm2(const float (&xq)[Lay<D>::DL]) {
    float s = 0.f;
#pragma unroll
    for (int t = 0; t < Lay<D>::DL; ++t) s = __fmaf_rn(xq[t], xq[t], s);
    return pair_sum<32>(pair_sum<16>(s));
}

// FP64 |x - c|^2 of this lane's point to the FP64 centroid row c,
// summed over the four lanes of the point (same value in all four).
template <int D>
__device__ __forceinline__ double quarter_dist64(const float (&xq)[Lay<D>::DL],
                                                 const double* __restrict__ c) {
    constexpr int DL = Lay<D>::DL;
    const int g = (threadIdx.x & 63) >> 4;
    double p = 0.0;
#pragma unroll
    for (int t = 0; t < DL; ++t) {
        const double e = (double)xq[t] - c[g * DL + t];
        p = __fma_rn(e, e, p);
    }
    return pair_sum<32>(pair_sum<16>(p));
}

// quarter_dist64 for use inside loops: the point's coordinates are
// converted to FP64 at each call (the empty asm hides that they are
// loop-invariant, so the compiler does not hoist the conversions and hold
// 2 DL registers for the whole loop).
template <int D>
__device__ __forceinline__ double quarter_dist64_fresh(const float (&xq)[Lay<D>::DL],
                                                       const double* __restrict__ c) {
    constexpr int DL = Lay<D>::DL;
    const int g = (threadIdx.x & 63) >> 4;
    double p = 0.0;
#pragma unroll
    for (int t = 0; t < DL; ++t) {
        float x = xq[t];
        asm volatile("" : "+v"(x));
        const double e = (double)x - c[g * DL + t];
        p = __fma_rn(e, e, p);
    }
    return pair_sum<32>(pair_sum<16>(p));
}

// |x| for the certificate: hardware square root (within 1 ulp), the 2.5
// factor of the test covers its error.
__device__ __forceinline__ float cert_norm(float n2) { return __builtin_amdgcn_sqrtf(n2); }

// Screening winner certified (see the certificate above)?  E = ea |x| +
// eb (alpha and beta already multiplied by cmax and cmax^2).
__device__ __forceinline__ bool certified(const Top3& t, unsigned kmask, float qscale, float xnorm,
                                          float ea, float eb) {
    if (t.t2 >= 0x7F800000u) return true;  // fewer than two valid centroids
    const float q1 = key_value(t.t1, kmask), q2 = key_value(t.t2, kmask);
    return (q2 - q1) > 2.5f * (ea * xnorm + eb) + qscale * q2;
}

// The exact argmin is one of the two best screened centroids when the third
// is separated from the best by the same margin.
__device__ __forceinline__ bool top2_suffices(const Top3& t, unsigned kmask, float qscale,
                                              float xnorm, float ea, float eb) {
    if (t.t3 >= 0x7F800000u) return true;
    const float q1 = key_value(t.t1, kmask), q3 = key_value(t.t3, kmask);
    return (q3 - q1) > 2.5f * (ea * xnorm + eb) + qscale * q3;
}

// Rows that may still hold the exact minimum of this lane's point when its
// three best keys leave more than two in contention (`full`): the screening
// tile is computed again, and every row whose key fails the certificate's
// exclusion test against the best key q1 (q_j - q1 > 2.5 E + 2^(NB-20) q_j;
// the argument above shows an excluded row scores strictly above the
// screening winner, so exact ties are never excluded) is ranked in FP64.
// Each such row is evaluated once for all points of the wave that keep it
// (wave-uniform loops over ballots).  best / bj carry the exact value and
// index of the best row so far and are updated in place, lowest index on
// exact ties.  Padding and invalid rows (keys at or above 0x7F800000) are
// never kept.
template <int D, int PREC>
__device__ __forceinline__ void rescan_rows(const float (&xq)[Lay<D>::DL], bool full, float q1,
                                            float e25, float qscale, const void* __restrict__ aop,
                                            const float* __restrict__ nrm, int nblk, float h,
                                            unsigned kmask, const double* __restrict__ C64,
                                            double& best, int& bj) {
    constexpr int DL = Lay<D>::DL, KC = Lay<D>::KC, CS = Lay<D>::CS;
    const int lane = threadIdx.x & 63, g = lane >> 4, p = lane & 15;
    for (int blk = 0; blk < nblk; ++blk) {
        f32x4 acc = *reinterpret_cast<const f32x4*>(nrm + blk * 16 + 4 * g);
        if constexpr (PREC == kPrecF32) {
            const float* a = static_cast<const float*>(aop);
#pragma unroll
            for (int q = 0; q < DL; ++q)
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[(blk * DL + q) * 64 + lane], xq[q],
                                                           acc, 0, 0, 0);
        } else if constexpr (PREC == kPrecBF16x3) {
            bf16x8 xh[KC], xl[KC];
            split_point<D>(xq, xh, xl);
            const bf16x8* a = static_cast<const bf16x8*>(aop);
            const bf16x8* al = a + nblk * KC * 64;
#pragma unroll
            for (int kc = 0; kc < KC; ++kc) {
                const int o = (blk * KC + kc) * 64 + lane;
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[o], xh[kc], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[o], xl[kc], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[o], xh[kc], acc, 0, 0, 0);
            }
        } else {
            const bf16x8* a = static_cast<const bf16x8*>(aop);
#pragma unroll
            for (int kc = 0; kc < KC; ++kc) {
                bf16x8 xb;
#pragma unroll
                for (int v = 0; v < 8; ++v) {
                    const int q = kc * 8 + v;
                    xb[v] = (__bf16)(q < DL ? xq[q < DL ? q : 0] : 0.f);
                }
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[(blk * KC + kc) * 64 + lane], xb,
                                                              acc, 0, 0, 0);
            }
        }
        // kept rows of this block: bit 16 g' + p' of keep[r] is row 4 g' + r
        // for point p'
        unsigned long long keep[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const unsigned key = screen_key(acc[r] + h, kmask, 0u);
            const float q = key_value(key, kmask);
            keep[r] = __ballot(full && key < 0x7F800000u && !((q - q1) > e25 + qscale * q));
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            unsigned long long mk = keep[r];
            while (mk) {
                const int gg = __builtin_ctzll(mk) >> 4;
                const unsigned bits = (unsigned)(mk >> (16 * gg)) & 0xFFFFu;
                mk &= ~(0xFFFFull << (16 * gg));
                const int j = blk * 16 + 4 * gg + r;
                const double v = quarter_dist64_fresh<D>(xq, C64 + j * CS);
                if (((bits >> p) & 1u) && (v < best || (v == best && j < bj))) {
                    best = v;
                    bj = j;
                }
            }
        }
    }
}

// Exact FP64 decision for the points of this wave whose screening was not
// certified (`redo` true in their four lanes): between the two best
// screened rows when the third is clear (`pair_ok`), otherwise over the
// rows rescan_rows keeps.  Lowest index on exact ties.  Wave-uniform
// branches; returns the decided index (a1 where redo is false).  h, xnorm,
// ea and eb are the values the point's keys t were screened with.
template <int D, int PREC>
__device__ __forceinline__ int redecide64(const float (&xq)[Lay<D>::DL], const Top3& t, bool redo,
                                          bool pair_ok, int a1, int a2,
                                          const double* __restrict__ C64,
                                          const void* __restrict__ aop,
                                          const float* __restrict__ nrm, int nblk, float h,
                                          unsigned kmask, float qscale, float xnorm, float ea,
                                          float eb) {
    constexpr int CS = Lay<D>::CS;
    int am = a1;
    if (!__any(redo)) return am;
    const double v1 = quarter_dist64<D>(xq, C64 + a1 * CS);
    const double v2 = quarter_dist64<D>(xq, C64 + a2 * CS);
    const bool take2 = v2 < v1 || (v2 == v1 && a2 < a1);
    if (redo && pair_ok && take2) am = a2;
    const bool full = redo && !pair_ok;
    if (!__any(full)) return am;
    double best = take2 ? v2 : v1;
    int bj = take2 ? a2 : a1;
    rescan_rows<D, PREC>(xq, full, key_value(t.t1, kmask), 2.5f * (ea * xnorm + eb), qscale, aop,
                         nrm, nblk, h, kmask, C64, best, bj);
    return full ? bj : am;
}

// This lane's FP64 share of |x - c|^2 (its DL coordinates; the four lanes
// of a point together give the distance).
template <int D>
__device__ __forceinline__ double quarter_part64(const float (&xq)[Lay<D>::DL],
                                                 const double* __restrict__ c) {
    constexpr int DL = Lay<D>::DL;
    const int g = (threadIdx.x & 63) >> 4;
    double p = 0.0;
#pragma unroll
    for (int t = 0; t < DL; ++t) {
        const double e = (double)xq[t] - c[g * DL + t];
        p = __fma_rn(e, e, p);
    }
    return p;
}

}  // namespace hpc

// Streaming full-data assignment with its FP64 objective, the counter-based
// sample draw, and the keep-the-best / best-worker selection kernels.
#pragma once

#include "common.hpp"

namespace hpc {

// ---------------------------------------------------------------------------
// Sample draw (Section 3): index j of a sample is word j%4 of block j/4 of
// stream (seed, tag 0) / (block, sample_id, 0, 0), mapped to [0, m) by a
// 64x64 multiply-high.  One thread per block of four indices.
// ---------------------------------------------------------------------------
__global__ void k_draw_one(int64_t m, int32_t s, uint64_t seed, uint64_t sample_id,
                           int64_t* __restrict__ idx) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t j0 = q * 4;
    if (j0 >= s) return;
    const Words4 w = philox_block(seed, kTagSample, (uint64_t)q, sample_id, 0);
#pragma unroll
    for (int t = 0; t < 4; ++t)
        if (j0 + t < s) idx[j0 + t] = bounded_index(w.w[t], (uint64_t)m);
}

// grid.y = sample, grid.x strides over that sample's blocks of four.
__global__ void k_draw_batch(int64_t m, const hpc_sample_desc* __restrict__ desc,
                             int64_t* __restrict__ idx) {
    const hpc_sample_desc ds = desc[blockIdx.y];
    const int64_t nq = ((int64_t)ds.s + 3) / 4;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nq;
         q += (int64_t)gridDim.x * blockDim.x) {
        const Words4 w = philox_block(ds.seed, kTagSample, (uint64_t)q, ds.sample_id, 0);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int64_t j = q * 4 + t;
            if (j < ds.s) idx[ds.idx_offset + j] = bounded_index(w.w[t], (uint64_t)m);
        }
    }
}

// ---------------------------------------------------------------------------
// Full assignment + objective (Section 3 final step; Eq. (1)).  HBM-bound
// stream over the rows of X: each thread takes whole rows (grid-stride),
// centroids are staged in LDS (FP32 for the screening, FP64 for the exact
// distance; zero padded to D, degenerate rows flagged).  The FP32 screening
// winner is certified (the centroids are exact in FP32 here, so only the
// arithmetic bound applies) or re-decided in FP64; the objective adds the
// FP64 distance to the chosen centroid.  Counts go to an LDS histogram; the
// objective is an FP64 per-thread partial reduced per workgroup in fixed
// order, then across workgroups by k_reduce_partials in fixed order.
// ---------------------------------------------------------------------------
template <int D>
__host__ __device__ inline size_t assign_lds_bytes(int k, int nt) {
    return (size_t)k * D * 8 + (((size_t)k * D * 4 + (size_t)k * 8 + 15) / 16) * 16 +
           (size_t)(nt / kWave) * 8;
}

template <int D, int NT>
__global__ __launch_bounds__(NT) void k_assign_sse(const float* __restrict__ X, int64_t m, int d,
                                                   const float* __restrict__ C, int k,
                                                   int32_t* __restrict__ labels,
                                                   unsigned long long* __restrict__ counts,
                                                   double* __restrict__ partials, bool vec) {
    extern __shared__ __align__(16) char smem[];
    double* C64 = reinterpret_cast<double*>(smem);
    float* C32 = reinterpret_cast<float*>(smem + (size_t)k * D * 8);
    int* valid = reinterpret_cast<int*>(C32 + (size_t)k * D);
    int* hist = valid + k;
    double* red = reinterpret_cast<double*>(
        smem + (size_t)k * D * 8 + (((size_t)k * D * 4 + (size_t)k * 8 + 15) / 16) * 16);
    const int tid = threadIdx.x;
    for (int e = tid; e < k * D; e += NT) {
        const int j = e / D, t = e % D;
        const float v = t < d ? C[(int64_t)j * d + t] : 0.f;
        C32[e] = v;
        C64[e] = (double)v;
    }
    for (int j = tid; j < k; j += NT) {
        valid[j] = !is_nan_f(C[(int64_t)j * d]);
        hist[j] = 0;
    }
    __syncthreads();
    const float tau = 4.f * (float)(d + 8) * 0x1.0p-24f;
    double fl = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * NT + tid; i < m; i += (int64_t)gridDim.x * NT) {
        float x[D];
        if (vec) {
            load_row<D>(X + i * D, x);
        } else {
#pragma unroll
            for (int t = 0; t < D; ++t) x[t] = t < d ? X[i * d + t] : 0.f;
        }
        float b1 = __builtin_huge_valf(), b2 = __builtin_huge_valf();
        int am = -1;
        for (int j = 0; j < k; ++j) {
            if (!valid[j]) continue;
            const float v = sqdist<D>(x, C32 + j * D);
            if (v < b1) {
                b2 = b1;
                b1 = v;
                am = j;
            } else if (v < b2) {
                b2 = v;
            }
        }
        double dm = __builtin_huge_val();
        if (am >= 0) {
            if (screen_certified(b1, b2, tau, 0.f)) {
                dm = sqdist64<D>(x, C64 + am * D);
            } else {
                for (int j = 0; j < k; ++j) {
                    if (!valid[j]) continue;
                    const double v = sqdist64<D>(x, C64 + j * D);
                    if (v < dm) {
                        dm = v;
                        am = j;
                    }
                }
            }
        }
        fl += dm;
        if (labels) labels[i] = am;
        if (counts && am >= 0) atomicAdd(&hist[am], 1);
    }
    const double tot = block_sum<NT>(fl, red);
    if (tid == 0) partials[blockIdx.x] = tot;
    if (counts)
        for (int j = tid; j < k; j += NT)
            if (hist[j]) atomicAdd(&counts[j], (unsigned long long)hist[j]);
}

// Sum of n partials in a fixed order by one workgroup of NT threads.
template <int NT>
__global__ __launch_bounds__(NT) void k_reduce_partials(const double* __restrict__ partials, int n,
                                                        double* __restrict__ out) {
    __shared__ double red[NT / kWave];
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += NT) v += partials[i];
    const double tot = block_sum<NT>(v, red);
    if (threadIdx.x == 0) *out = tot;
}

__global__ void k_fill_u64(unsigned long long* __restrict__ p, int64_t n, unsigned long long v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------------------
// Keep the best (Algorithm 3): one workgroup per worker.
// ---------------------------------------------------------------------------
__global__ void k_keep_best(const float* __restrict__ C_new, const double* __restrict__ f_new,
                            float* __restrict__ C_inc, double* __restrict__ f_inc, int64_t kd,
                            int32_t* __restrict__ updated) {
    const int w = blockIdx.x;
    const double fn = f_new[w], fi = f_inc[w];
    const bool take = fn < fi;
    if (take)
        for (int64_t e = threadIdx.x; e < kd; e += blockDim.x)
            C_inc[(int64_t)w * kd + e] = C_new[(int64_t)w * kd + e];
    __syncthreads();
    if (threadIdx.x == 0) {
        if (take) f_inc[w] = fn;
        if (updated) updated[w] = take ? 1 : 0;
    }
}

// Best worker: argmin of f_inc (lowest index on ties), then copy its block.
template <int NT>
__global__ __launch_bounds__(NT) void k_select_best(const float* __restrict__ C_inc,
                                                    const double* __restrict__ f_inc, int n,
                                                    int64_t kd, float* __restrict__ C_best,
                                                    double* __restrict__ f_best,
                                                    int32_t* __restrict__ w_best) {
    __shared__ double bv[NT];
    __shared__ int bi[NT];
    double v = __builtin_huge_val();
    int ix = -1;
    for (int w = threadIdx.x; w < n; w += NT) {
        const double f = f_inc[w];
        if (ix < 0 || f < v) {
            v = f;
            ix = w;
        }
    }
    bv[threadIdx.x] = v;
    bi[threadIdx.x] = ix;
    __syncthreads();
    for (int o = NT / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            const double v2 = bv[threadIdx.x + o];
            const int i2 = bi[threadIdx.x + o];
            const int i1 = bi[threadIdx.x];
            const double v1 = bv[threadIdx.x];
            const bool take2 = i2 >= 0 && (i1 < 0 || v2 < v1 || (v2 == v1 && i2 < i1));
            if (take2) {
                bv[threadIdx.x] = v2;
                bi[threadIdx.x] = i2;
            }
        }
        __syncthreads();
    }
    const int wb = bi[0] < 0 ? 0 : bi[0];  // every f NaN: report worker 0
    for (int64_t e = threadIdx.x; e < kd; e += NT) C_best[e] = C_inc[(int64_t)wb * kd + e];
    if (threadIdx.x == 0) {
        *f_best = bv[0];
        if (w_best) *w_best = wb;
    }
}

}  // namespace hpc

// Streaming full-data assignment with its FP64 objective, the counter-based
// sample draw, and the keep-the-best / best-worker selection kernels.
#pragma once

#include "common.hpp"
#include "mfma_screen.hpp"
#include "screen32.hpp"

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
// stream over the rows of X in tiles of 16 rows per wave (grid-stride): the
// nearest valid centroid is screened on MFMA (mfma_screen.hpp) and either
// certified or re-decided in FP64; the objective adds the FP64 distance to
// the chosen centroid.  Centroids live in LDS (FP64 rows, MFMA operands,
// |c|^2 biases; degenerate rows never chosen).  Counts go to an LDS
// histogram; the objective is an FP64 per-lane partial reduced per
// workgroup in fixed order, then across workgroups by k_reduce_partials in
// fixed order.
// ---------------------------------------------------------------------------
template <int D, int PREC>
__host__ __device__ inline size_t assign_lds_bytes(int k, int nt) {
    const int nb = (k + 15) / 16;
    size_t b = (((size_t)k * Lay<D>::CS * 8 + 15) / 16) * 16;
    b += ((aop_bytes<D, PREC>(nb) + 15) / 16) * 16 + (size_t)nb * 64;
    b += (((size_t)k * 8 + 15) / 16) * 16;  // valid + hist
    b += (size_t)(nt / kWave) * 8 + 16;
    return b;
}

// Up to d = 32 five waves per SIMD, each with three tiles of rows in
// flight; wider rows keep three register buffers at the occupancy their
// registers allow.  The 768-thread form (three waves per SIMD from one
// workgroup) is for centroid tables too large for several 256-thread
// workgroups per CU in LDS.
template <int D, int NT, int PREC>
__global__ __launch_bounds__(NT, NT > 256 ? NT / 256 : (D <= 32 ? 5 : (D <= 64 ? 3 : 2))) void k_assign_sse(const float* __restrict__ X, int64_t m, int d,
                                                   const float* __restrict__ C, int k,
                                                   int32_t* __restrict__ labels,
                                                   unsigned long long* __restrict__ counts,
                                                   double* __restrict__ partials, bool vec) {
    extern __shared__ __align__(16) char smem[];
    constexpr int DL = Lay<D>::DL, CS = Lay<D>::CS;
    constexpr int NW = NT / kWave;
    const int nblk = (k + 15) / 16;
    char* p = smem;
    double* C64 = reinterpret_cast<double*>(p);
    p += (((size_t)k * CS * 8 + 15) / 16) * 16;
    void* aop = p;
    p += ((aop_bytes<D, PREC>(nblk) + 15) / 16) * 16;
    float* nrm = reinterpret_cast<float*>(p);
    p += (size_t)nblk * 64;
    int* hist = reinterpret_cast<int*>(p);
    int* flag = hist + k;
    p += (((size_t)k * 8 + 15) / 16) * 16;
    double* red = reinterpret_cast<double*>(p);
    // the wave index is made wave-uniform so that tile indices live in
    // scalar registers
    const int tid = threadIdx.x, lane = tid & 63, g = lane >> 4;
    const int wid = __builtin_amdgcn_readfirstlane(tid / kWave);
    for (int e = tid; e < k * CS; e += NT) {
        const int j = e / CS, t = e % CS;
        C64[e] = t < d ? (double)C[(int64_t)j * d + t] : 0.0;
    }
    for (int j = tid; j < k; j += NT) hist[j] = 0;
    unsigned long long* const mx2 = reinterpret_cast<unsigned long long*>(red + NW);
    if (tid == 0) {
        flag[0] = 0;
        *mx2 = 0ull;
    }
    __syncthreads();
    // valid rows and the largest squared norm, one row per thread (the
    // norms are >= 0, so their bit patterns order as unsigned integers)
    for (int j = tid; j < k; j += NT) {
        if (C64[j * CS] != C64[j * CS]) continue;
        double n2 = 0.0;
        for (int t = 0; t < d; ++t) n2 = __fma_rn(C64[j * CS + t], C64[j * CS + t], n2);
        atomicAdd(&flag[0], 1);
        atomicMax(mx2, (unsigned long long)__double_as_longlong(n2));
    }
    build_operands<D, PREC, NT>(C64, k, d, nblk, aop, nrm);
    __syncthreads();
    const int n_valid = flag[0];
    double alpha, beta;
    screen_coeffs<PREC>(d, &alpha, &beta);
    const double cmax = sqrt(__longlong_as_double((long long)*mx2));
    const float ea = (float)(alpha * cmax), eb = (float)(beta * cmax * cmax);
    unsigned kmask;
    float qscale;
    key_params(nblk, &kmask, &qscale);
    double fl = 0.0;
    const int64_t n_tiles = (m + 15) / 16;
    auto process = [&](int64_t tile, const float (&xq)[DL]) {
        const int64_t i = tile * 16 + (lane & 15);
        const bool valid = i < m;
        const float xn2 = point_norm2<D>(xq);
        const float xn = cert_norm(xn2);
        const float h = screen_shift(xn2, xn, ea, eb);
        const Top3 t3 = screen_tile<D, PREC>(xq, aop, nrm, nblk, h, kmask);
        const bool ok = certified(t3, kmask, qscale, xn, ea, eb) || !valid;
        const int a1 = (int)key_index(t3.t1, kmask), a2 = (int)key_index(t3.t2, kmask);
        int am = redecide64<D, PREC>(xq, t3, !ok, top2_suffices(t3, kmask, qscale, xn, ea, eb),
                                     a1 < k ? a1 : 0, a2 < k ? a2 : 0, C64, aop, nrm, nblk, h,
                                     kmask, qscale, xn, ea, eb);
        if (valid) {
            // this lane's share of the objective: FP64 distance to the choice
            fl += n_valid > 0 ? quarter_part64<D>(xq, C64 + am * CS) : __builtin_huge_val();
            if (n_valid == 0) am = -1;
            if (g == 0) {
                if (labels) labels[i] = am;
                if (counts && am >= 0) atomicAdd(&hist[am], 1);
            }
        }
    };
    const int64_t first = (int64_t)blockIdx.x * NW + wid, stride = (int64_t)gridDim.x * NW;
    if (vec) {
        // rows of D floats, 16-byte aligned: software pipelined over register
        // buffers (rows of the next tiles in flight while one is processed;
        // unrolled so that no buffer with a load in flight is copied); rows
        // past the end re-read the last row, branch-free, and tiles past the
        // end are skipped by wave-uniform guards rather than exits from the
        // unrolled body
        auto fetch = [&](int64_t tile, float (&dst)[DL]) {
            const int64_t r0 = tile * 16;  // wave-uniform
            const float* src;
            if (r0 + 16 <= m) {
                // a full tile: the row base is scalar, the lane's offset a
                // 32-bit constant
                src = X + r0 * D + (lane & 15) * D;
            } else {
                int64_t i = r0 + (lane & 15);
                i = i < m ? i : m - 1;
                src = X + i * D;
            }
            load_quarter<D>(src, g, dst);
        };
        if constexpr (D <= 32) {
            float xa[DL], xb[DL], xc[DL], xd[DL];
            fetch(first, xa);
            fetch(first + stride, xb);
            fetch(first + 2 * stride, xc);
            for (int64_t tile = first; tile < n_tiles; tile += 4 * stride) {
                fetch(tile + 3 * stride, xd);
                process(tile, xa);
                fetch(tile + 4 * stride, xa);
                if (tile + stride < n_tiles) process(tile + stride, xb);
                fetch(tile + 5 * stride, xb);
                if (tile + 2 * stride < n_tiles) process(tile + 2 * stride, xc);
                fetch(tile + 6 * stride, xc);
                if (tile + 3 * stride < n_tiles) process(tile + 3 * stride, xd);
            }
        } else {
            float xa[DL], xb[DL], xc[DL];
            fetch(first, xa);
            fetch(first + stride, xb);
            for (int64_t tile = first; tile < n_tiles; tile += 3 * stride) {
                fetch(tile + 2 * stride, xc);
                process(tile, xa);
                fetch(tile + 3 * stride, xa);
                if (tile + stride < n_tiles) process(tile + stride, xb);
                fetch(tile + 4 * stride, xb);
                if (tile + 2 * stride < n_tiles) process(tile + 2 * stride, xc);
            }
        }
    } else {
        for (int64_t tile = first; tile < n_tiles; tile += stride) {
            const int64_t i = tile * 16 + (lane & 15);
            float xq[DL];
#pragma unroll
            for (int t = 0; t < DL; ++t) {
                const int dim = g * DL + t;
                xq[t] = (i < m && dim < d) ? X[i * d + dim] : 0.f;
            }
            process(tile, xq);
        }
    }
    const double tot = block_sum<NT>(fl, red);
    if (tid == 0) partials[blockIdx.x] = tot;
    if (counts)
        for (int j = tid; j < k; j += NT)
            if (hist[j]) atomicAdd(&counts[j], (unsigned long long)hist[j]);
}

// Bytes of k_assign_sse32's LDS: FP64 centroids, operand tables and biases
// for blocks of 32, valid flags and histogram, wave partials.
template <int D, int PREC>
__host__ __device__ inline size_t assign32_lds_bytes(int k, int nt) {
    const int nb = (k + 31) / 32;
    size_t b = (((size_t)k * Lay32<D>::CS * 8 + 15) / 16) * 16;
    b += ((aop32_bytes<D, PREC>(nb) + 15) / 16) * 16 + (size_t)nb * 128;
    b += (((size_t)k * 8 + 15) / 16) * 16;  // valid + hist
    b += (size_t)nt * 8;                    // per-thread objective shares
    b += (size_t)(nt / kWave) * 8 + 16;
    return b;
}

// ---------------------------------------------------------------------------
// Full assignment for rows of up to 32 coordinates on 32 x 32 tiles
// (screen32.hpp): the same results as k_assign_sse (labels, counts, FP64
// objective share per workgroup), each wave taking tiles of 32 rows, every
// row in two lanes.
// ---------------------------------------------------------------------------
template <int D, int NT, int PREC>
__global__ __launch_bounds__(NT, 4) void k_assign_sse32(const float* __restrict__ X, int64_t m,
                                                        int d, const float* __restrict__ C, int k,
                                                        int32_t* __restrict__ labels,
                                                        unsigned long long* __restrict__ counts,
                                                        double* __restrict__ partials, bool vec) {
    extern __shared__ __align__(16) char smem[];
    constexpr int DH = Lay32<D>::DH, CS = Lay32<D>::CS;
    constexpr int NW = NT / kWave;
    const int nb = (k + 31) / 32;
    char* p = smem;
    double* C64 = reinterpret_cast<double*>(p);
    p += (((size_t)k * CS * 8 + 15) / 16) * 16;
    void* aop = p;
    p += ((aop32_bytes<D, PREC>(nb) + 15) / 16) * 16;
    float* nrm = reinterpret_cast<float*>(p);
    p += (size_t)nb * 128;
    int* hist = reinterpret_cast<int*>(p);
    int* flag = hist + k;
    p += (((size_t)k * 8 + 15) / 16) * 16;
    // each thread's running share of the objective lives in LDS: held in a
    // register across the tile loop it is the value the allocator spills,
    // and a scratch reload waits for every row load in flight
    double* share = reinterpret_cast<double*>(p);
    p += (size_t)NT * 8;
    double* red = reinterpret_cast<double*>(p);
    const int tid = threadIdx.x, lane = tid & 63, hh = lane >> 5;
    const int wid = __builtin_amdgcn_readfirstlane(tid / kWave);
    for (int e = tid; e < k * CS; e += NT) {
        const int j = e / CS, t = e % CS;
        C64[e] = t < d ? (double)C[(int64_t)j * d + t] : 0.0;
    }
    for (int j = tid; j < k; j += NT) hist[j] = 0;
    share[tid] = 0.0;
    unsigned long long* const mx2 = reinterpret_cast<unsigned long long*>(red + NW);
    if (tid == 0) {
        flag[0] = 0;
        *mx2 = 0ull;
    }
    __syncthreads();
    for (int j = tid; j < k; j += NT) {
        if (C64[j * CS] != C64[j * CS]) continue;
        double n2 = 0.0;
        for (int t = 0; t < d; ++t) n2 = __fma_rn(C64[j * CS + t], C64[j * CS + t], n2);
        atomicAdd(&flag[0], 1);
        atomicMax(mx2, (unsigned long long)__double_as_longlong(n2));
    }
    build_operands32<D, PREC, NT>(C64, k, d, nb, aop, nrm);
    __syncthreads();
    const int n_valid = flag[0];
    double alpha, beta;
    screen_coeffs<PREC>(d, &alpha, &beta);
    const double cmax = sqrt(__longlong_as_double((long long)*mx2));
    const float ea = (float)(alpha * cmax), eb = (float)(beta * cmax * cmax);
    unsigned kmask;
    float qscale;
    key_params(2 * nb, &kmask, &qscale);
    const int64_t n_tiles = (m + 31) / 32;
    auto process = [&](int64_t tile, const float (&xh)[DH]) {
        const int64_t i = tile * 32 + (lane & 31);
        const bool valid = i < m;
        const float xn2 = point_norm2_32<D>(xh);
        const float xn = cert_norm(xn2);
        const float h = screen_shift(xn2, xn, ea, eb);
        const Top3 t3 = screen_tile32<D, PREC>(xh, aop, nrm, nb, h, kmask);
        const bool ok = certified(t3, kmask, qscale, xn, ea, eb) || !valid;
        const int a1 = (int)key_index(t3.t1, kmask), a2 = (int)key_index(t3.t2, kmask);
        int am = redecide64_32<D, PREC>(xh, t3, !ok, top2_suffices(t3, kmask, qscale, xn, ea, eb),
                                        a1 < k ? a1 : 0, a2 < k ? a2 : 0, C64, aop, nrm, nb, h,
                                        kmask, qscale, xn, ea, eb);
        if (valid) {
            share[tid] += n_valid > 0 ? half_part64<D>(xh, C64 + am * CS) : __builtin_huge_val();
            if (n_valid == 0) am = -1;
            if (hh == 0) {
                if (labels) labels[i] = am;
                if (counts && am >= 0) atomicAdd(&hist[am], 1);
            }
        }
    };
    const int64_t first = (int64_t)blockIdx.x * NW + wid, stride = (int64_t)gridDim.x * NW;
    if (vec) {
        // rows of D floats, 16-byte aligned: three register buffers, rows of
        // the next two tiles in flight while one is processed; rows past the
        // end re-read the last row, tiles past the end are skipped by
        // wave-uniform guards
        // the tile's base row is wave-uniform (scalar registers) and the
        // lane's row a 32-bit offset from it, so no per-lane 64-bit address
        // is kept across the tile
        auto fetch = [&](int64_t tile, float (&dst)[DH]) {
            const int64_t r0 = min(tile * 32, m - 1);  // wave-uniform
            const int row = (int)min((int64_t)(lane & 31), m - 1 - r0);
            load_half<D>(X + r0 * D + row * D, hh, dst);
        };
        float xa[DH], xb[DH], xc[DH];
        fetch(first, xa);
        fetch(first + stride, xb);
        for (int64_t tile = first; tile < n_tiles; tile += 3 * stride) {
            fetch(tile + 2 * stride, xc);
            process(tile, xa);
            fetch(tile + 3 * stride, xa);
            if (tile + stride < n_tiles) process(tile + stride, xb);
            fetch(tile + 4 * stride, xb);
            if (tile + 2 * stride < n_tiles) process(tile + 2 * stride, xc);
        }
    } else {
        for (int64_t tile = first; tile < n_tiles; tile += stride) {
            const int64_t i = tile * 32 + (lane & 31);
            float xh[DH];
#pragma unroll
            for (int t = 0; t < DH; ++t) {
                const int dim = hh * DH + t;
                xh[t] = (i < m && dim < d) ? X[i * d + dim] : 0.f;
            }
            process(tile, xh);
        }
    }
    const double tot = block_sum<NT>(share[tid], red);
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

// chosen[j] <- tmp[j] where the resident seeding pass picked a point for row
// j (tmp[j] >= 0); the other rows keep what the team kernel wrote (or -1).
__global__ void k_merge_chosen(int32_t* __restrict__ chosen, const int32_t* __restrict__ tmp,
                               int32_t k) {
    for (int j = threadIdx.x; j < k; j += blockDim.x)
        if (tmp[j] >= 0) chosen[j] = tmp[j];
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

// ---------------------------------------------------------------------------
// Per-descriptor forms of the worker-loop bookkeeping (Algorithm 3), for a
// batch whose samples have their own k: sample b's centroid block is the k_b
// x d floats at desc[b].c_offset in both C and the incumbent array.
// ---------------------------------------------------------------------------

// C <- C_inc for every sample (the round starts from the incumbents).
// grid.y = sample.
__global__ void k_copy_blocks(const hpc_sample_desc* __restrict__ desc, int32_t d,
                              const float* __restrict__ src, float* __restrict__ dst) {
    const hpc_sample_desc ds = desc[blockIdx.y];
    const int64_t n = (int64_t)ds.k * d;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        dst[ds.c_offset + e] = src[ds.c_offset + e];
}

// Keep the best: one workgroup per sample; strict < as in k_keep_best.
__global__ void k_keep_best_desc(const hpc_sample_desc* __restrict__ desc, int32_t d,
                                 const float* __restrict__ C_new, const double* __restrict__ f_new,
                                 float* __restrict__ C_inc, double* __restrict__ f_inc) {
    const int b = blockIdx.x;
    const hpc_sample_desc ds = desc[b];
    const double fn = f_new[b], fi = f_inc[b];
    const bool take = fn < fi;
    if (take)
        for (int64_t e = threadIdx.x; e < (int64_t)ds.k * d; e += blockDim.x)
            C_inc[ds.c_offset + e] = C_new[ds.c_offset + e];
    __syncthreads();
    if (threadIdx.x == 0 && take) f_inc[b] = fn;
}

// Next round's samples: sample_id += stride for every descriptor.
__global__ void k_advance_ids(hpc_sample_desc* __restrict__ desc, int32_t n, uint64_t stride) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < n) desc[b].sample_id += stride;
}

}  // namespace hpc

// Workgroup-resident sample processing for gfx950.
//
// One workgroup owns one sample at a time and runs the whole per-sample
// method on it without leaving the kernel: gather of the sample rows,
// K-means++ seeding of degenerate centroids (Section 3; three candidates,
// Section 6.5), and the K-means passes (Algorithm 1) with the stop rule of
// Section 6.5.  A persistent grid pulls samples from a queue in
// longest-first order, so hundreds of samples of uneven size share one
// launch with no inter-workgroup synchronisation at all.
//
// Layout per sample: the gathered rows live in a scratch buffer (row stride
// D floats, zero padded) that stays hot in L2/MALL across passes; centroids
// sit in LDS; per-wave FP64 partial sums of the update live in LDS; D^2 of
// the seeding lives in scratch, each element owned by one thread.
#pragma once

#include "common.hpp"

namespace hpc {

struct LloydArgs {
    const float* X;
    int64_t m;
    int32_t d;
    const int64_t* idx;
    const hpc_sample_desc* desc;
    const int32_t* order;  // processing order (longest first); may be null
    int32_t n_samples;
    float* C;
    int32_t max_iter;
    double rel_tol;
    double* f_out;
    int32_t* iters_out;
    int32_t* labels_out;
    float* sbuf;   // gathered samples, indexed by idx_offset, stride D
    float* d2buf;  // D^2, indexed by idx_offset
    int32_t* queue;
    int32_t kmax;
    int32_t n_copies;  // partial-sum copies in LDS (== waves: no atomics)
    // seeding-only mode
    int32_t seed_only;
    int32_t n_cand;
    uint32_t call_id;
    int32_t* chosen;
};

// Carving of the dynamic LDS allocation; the host computes the same size.
template <int D, int NT>
struct Smem {
    static constexpr int NW = NT / kWave;
    float* Cs;     // kmax x D centroids
    float* crow;   // 4 x D candidate rows
    double* psum;  // n_copies x kmax x D update sums   (union with seeding arrays)
    int* pcnt;     // n_copies x kmax counts
    double* incl;  // NT inclusive scan of chunk sums   (seeding)
    double* csum;  // NT chunk sums of D^2              (seeding)
    double* cpot;  // 4 x NT chunk potentials           (seeding)
    double* red;   // 4 x NW wave partials
    double* dbl;   // 8 scalars
    int* deg;      // kmax degenerate-row list
    int* ints;     // 16 scalars

    static __host__ __device__ size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

    static __host__ __device__ size_t union_bytes(int kmax, int copies) {
        size_t lloyd = (size_t)copies * kmax * D * 8 + align_up((size_t)copies * kmax * 4, 8);
        size_t seed = (size_t)NT * 8 * 6;
        return lloyd > seed ? lloyd : seed;
    }
    static __host__ __device__ size_t bytes(int kmax, int copies) {
        size_t b = align_up((size_t)kmax * D * 4, 16) + 4 * D * 4;
        b += union_bytes(kmax, copies);
        b += 4 * NW * 8 + 8 * 8;
        b += align_up((size_t)kmax * 4, 16) + 16 * 4;
        return b;
    }
    __device__ Smem(char* base, int kmax, int copies) {
        char* p = base;
        Cs = reinterpret_cast<float*>(p);
        p += align_up((size_t)kmax * D * 4, 16);
        crow = reinterpret_cast<float*>(p);
        p += 4 * D * 4;
        char* u = p;
        psum = reinterpret_cast<double*>(u);
        pcnt = reinterpret_cast<int*>(u + (size_t)copies * kmax * D * 8);
        incl = reinterpret_cast<double*>(u);
        csum = incl + NT;
        cpot = csum + NT;
        p += union_bytes(kmax, copies);
        red = reinterpret_cast<double*>(p);
        p += 4 * NW * 8;
        dbl = reinterpret_cast<double*>(p);
        p += 8 * 8;
        deg = reinterpret_cast<int*>(p);
        p += align_up((size_t)kmax * 4, 16);
        ints = reinterpret_cast<int*>(p);
    }
};

// Up to four sums over the workgroup at once (fixed order).  Every thread
// gets the same values.  Two barriers.
template <int NT, int NV>
__device__ __forceinline__ void block_sum_n(double (&v)[NV], double* red) {
    constexpr int NW = NT / kWave;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        v[q] = wave_sum(v[q]);
        if (lane == 0) red[q * NW + w] = v[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double t = 0.0;
#pragma unroll
        for (int i = 0; i < NW; ++i) t += red[q * NW + i];
        v[q] = t;
    }
    __syncthreads();
}

// Inclusive scan of one double per thread over the workgroup (fixed order).
// Result written to out[tid]; two barriers.
template <int NT>
__device__ __forceinline__ void block_incl_scan(double v, double* out, double* red) {
    constexpr int NW = NT / kWave;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const double u = __shfl_up(v, o, kWave);
        if (lane >= o) v += u;
    }
    if (lane == kWave - 1) red[w] = v;
    __syncthreads();
    double base = 0.0;
    for (int i = 0; i < w; ++i) base += red[i];
    out[threadIdx.x] = base + v;
    __syncthreads();
}

// ---------------------------------------------------------------------------
// K-means++ on the gathered sample for every degenerate row of L.Cs.
// Sg: s x D rows; d2: s floats of scratch.  Stream (seed, tag) /
// (block, sid, call, 0).  Thread t owns the contiguous chunk
// [t*cs, (t+1)*cs) of the sample; the inverse-CDF search is a workgroup
// scan of the chunk sums followed by a sequential scan inside the one chunk
// that holds the target, so the prefix order is the sample's index order.
// chosen (nullable, global) receives the picked sample-local indices.
// ---------------------------------------------------------------------------
template <int D, int NT>
__device__ void kmeanspp_wg(const float* __restrict__ Sg, int s, int k, int n_cand,
                            float* __restrict__ d2, uint64_t seed, uint64_t tag, uint64_t sid,
                            uint64_t call, int32_t* __restrict__ chosen, Smem<D, NT>& L) {
    const int tid = threadIdx.x;
    if (tid == 0) {
        int nd = 0, nv = 0;
        for (int j = 0; j < k; ++j) {
            if (is_nan_f(L.Cs[j * D]))
                L.deg[nd++] = j;
            else
                ++nv;
        }
        L.ints[0] = nd;
        L.ints[1] = nv;
    }
    __syncthreads();
    const int n_deg = L.ints[0], n_valid = L.ints[1];
    if (n_deg == 0) return;

    const int cs = (s + NT - 1) / NT;
    const int lo = min(s, tid * cs), hi = min(s, lo + cs);
    int first = 0;
    double acc = 0.0;
    if (n_valid == 0) {
        if (tid == 0) {
            const Words4 w = philox_block(seed, tag, 0, sid, call);
            const int i0 = (int)bounded_index(w.w[0], (uint64_t)s);
            L.ints[2] = i0;
            if (chosen) chosen[L.deg[0]] = i0;
        }
        __syncthreads();
        const int i0 = L.ints[2], j0 = L.deg[0];
        for (int t = tid; t < D; t += NT) L.Cs[j0 * D + t] = Sg[(size_t)i0 * D + t];
        __syncthreads();
        for (int i = lo; i < hi; ++i) {
            float x[D];
            load_row<D>(Sg + (size_t)i * D, x);
            const float v = sqdist<D>(x, L.Cs + j0 * D);
            d2[i] = v;
            acc += v;
        }
        first = 1;
    } else {
        for (int i = lo; i < hi; ++i) {
            float x[D];
            load_row<D>(Sg + (size_t)i * D, x);
            float best = __builtin_huge_valf();
            for (int j = 0; j < k; ++j) {
                if (is_nan_f(L.Cs[j * D])) continue;
                const float v = sqdist<D>(x, L.Cs + j * D);
                best = v < best ? v : best;
            }
            d2[i] = best;
            acc += best;
        }
    }

    for (int r = first; r < n_deg; ++r) {
        // chunk prefix sums of the current D^2 (index order)
        block_incl_scan<NT>(acc, L.incl, L.red);
        const double W = L.incl[NT - 1];
        const uint64_t q = (uint64_t)(r + (n_valid > 0 ? 1 : 0));
        const Words4 w = philox_block(seed, tag, q, sid, call);
        int pick;
        if (!(W > 0.0)) {
            pick = (int)bounded_index(w.w[0], (uint64_t)s);
        } else {
            if (tid < 4) L.ints[4 + tid] = -1;
            __syncthreads();
            const double c_lo = tid == 0 ? 0.0 : L.incl[tid - 1];
            const double c_hi = L.incl[tid];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const double target = unit_double(w.w[t]) * W;
                if (t < n_cand && c_lo <= target && target < c_hi) {
                    double run = c_lo;
                    int found = -1;
                    for (int i = lo; i < hi; ++i) {
                        run += (double)d2[i];
                        if (run > target) {
                            found = i;
                            break;
                        }
                    }
                    if (found < 0)
                        for (int i = hi - 1; i >= lo; --i)
                            if (d2[i] > 0.f) {
                                found = i;
                                break;
                            }
                    L.ints[4 + t] = found;
                }
            }
            __syncthreads();
            if (tid == 0) {
                // a target that rounded up to W: last point of positive weight
                for (int t = 0; t < n_cand; ++t) {
                    if (L.ints[4 + t] >= 0) continue;
                    int found = -1;
                    for (int i = s - 1; i >= 0 && found < 0; --i)
                        if (d2[i] > 0.f) found = i;
                    L.ints[4 + t] = found < 0 ? 0 : found;
                }
            }
            __syncthreads();
            for (int e = tid; e < n_cand * D; e += NT)
                L.crow[e] = Sg[(size_t)L.ints[4 + e / D] * D + (e % D)];
            __syncthreads();
            double p[4] = {0.0, 0.0, 0.0, 0.0};
            for (int i = lo; i < hi; ++i) {
                float x[D];
                load_row<D>(Sg + (size_t)i * D, x);
                const float dd = d2[i];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    if (t < n_cand) {
                        const float v = sqdist<D>(x, L.crow + t * D);
                        p[t] += (double)(v < dd ? v : dd);
                    }
                }
            }
            block_sum_n<NT, 4>(p, L.red);
            int tb = 0;
            double pb = p[0];
#pragma unroll
            for (int t = 1; t < 4; ++t)
                if (t < n_cand && p[t] < pb) {
                    pb = p[t];
                    tb = t;
                }
            pick = L.ints[4 + tb];
        }
        const int jr = L.deg[r];
        if (tid == 0 && chosen) chosen[jr] = pick;
        for (int t = tid; t < D; t += NT) L.Cs[jr * D + t] = Sg[(size_t)pick * D + t];
        __syncthreads();
        acc = 0.0;
        for (int i = lo; i < hi; ++i) {
            float x[D];
            load_row<D>(Sg + (size_t)i * D, x);
            const float v = sqdist<D>(x, L.Cs + jr * D);
            const float o = d2[i];
            const float nv = v < o ? v : o;
            d2[i] = nv;
            acc += nv;
        }
        __syncthreads();
    }
}

// Fold one wave's points into the per-cluster sums: for every distinct label
// present in the wave, a butterfly sum of each coordinate over the lanes
// holding that label, added by the leader lane to this wave's LDS copy.
template <int D>
__device__ __forceinline__ void wave_accumulate(const float (&x)[D], int am, bool valid, int d,
                                                double* __restrict__ pw, int* __restrict__ cw,
                                                bool atomic) {
    const int lane = threadIdx.x & (kWave - 1);
    unsigned long long act = __ballot(valid);
    while (act) {
        const int leader = __ffsll(act) - 1;
        const int j = __shfl(am, leader, kWave);
        const bool in = valid && am == j;
        const unsigned long long mask = __ballot(in);
#pragma unroll
        for (int t = 0; t < D; ++t) {
            if (t < d) {
                const float v = wave_sum(in ? x[t] : 0.f);
                if (lane == leader) {
                    if (atomic)
                        atomicAdd(&pw[j * D + t], (double)v);
                    else
                        pw[j * D + t] += (double)v;
                }
            }
        }
        if (lane == leader) {
            if (atomic)
                atomicAdd(&cw[j], (int)__popcll(mask));
            else
                cw[j] += (int)__popcll(mask);
        }
        act &= ~mask;
    }
}

template <int D, int NT>
__global__ __launch_bounds__(NT) void k_lloyd_resident(LloydArgs a) {
    extern __shared__ __align__(16) char smem[];
    Smem<D, NT> L(smem, a.kmax, a.n_copies);
    constexpr int NW = Smem<D, NT>::NW;
    const int tid = threadIdx.x, wid = tid / kWave;
    const int d = a.d;

    for (;;) {
        if (tid == 0) L.ints[15] = atomicAdd(a.queue, 1);
        __syncthreads();
        const int slot = L.ints[15];
        __syncthreads();
        if (slot >= a.n_samples) break;
        const int b = a.order ? a.order[slot] : slot;
        const hpc_sample_desc ds = a.desc[b];
        const int s = ds.s, k = ds.k;
        float* Sg = a.sbuf + (size_t)ds.idx_offset * D;
        float* d2 = a.d2buf + ds.idx_offset;

        // gather the sample rows (zero padded to D)
        for (int i = tid; i < s; i += NT) {
            const int64_t row = a.idx[ds.idx_offset + i];
            const bool in_range = row >= 0 && row < a.m;  // out-of-range rows read as zeros
            const float* src = a.X + (in_range ? row : 0) * d;
            float* dst = Sg + (size_t)i * D;
#pragma unroll
            for (int t = 0; t < D; ++t) dst[t] = (t < d && in_range) ? src[t] : 0.f;
        }
        for (int e = tid; e < k * D; e += NT) {
            const int j = e / D, t = e % D;
            L.Cs[e] = t < d ? a.C[ds.c_offset + (int64_t)j * d + t] : 0.f;
        }
        __syncthreads();

        if (a.seed_only) {
            if (a.chosen)
                for (int j = tid; j < k; j += NT) a.chosen[j] = -1;
            __syncthreads();
            kmeanspp_wg<D, NT>(Sg, s, k, a.n_cand, d2, ds.seed, kTagSeed, ds.sample_id, a.call_id,
                               a.chosen, L);
        } else {
            double f_prev = __builtin_huge_val(), f = 0.0;
            int it = 0;
            const int copies = a.n_copies;
            const bool atomic = copies < NW;
            double* pw = L.psum + (size_t)(wid % copies) * k * D;
            int* cw = L.pcnt + (wid % copies) * k;
            for (;;) {
                kmeanspp_wg<D, NT>(Sg, s, k, 3, d2, ds.seed, kTagReseed, ds.sample_id,
                                   (uint64_t)it, nullptr, L);
                // (re)pointer after the union region was used by seeding
                for (int e = tid; e < copies * k * D; e += NT) L.psum[e] = 0.0;
                for (int e = tid; e < copies * k; e += NT) L.pcnt[e] = 0;
                __syncthreads();
                pw = L.psum + (size_t)(wid % copies) * k * D;
                cw = L.pcnt + (wid % copies) * k;
                double fl = 0.0;
                for (int base = 0; base < s; base += NT) {
                    const int i = base + tid;
                    const bool valid = i < s;
                    float x[D];
                    if (valid) {
                        load_row<D>(Sg + (size_t)i * D, x);
                    } else {
#pragma unroll
                        for (int t = 0; t < D; ++t) x[t] = 0.f;
                    }
                    float best = __builtin_huge_valf();
                    int am = 0;
                    for (int j = 0; j < k; ++j) {
                        const float v = sqdist<D>(x, L.Cs + j * D);
                        if (v < best) {
                            best = v;
                            am = j;
                        }
                    }
                    if (valid) {
                        fl += (double)best;
                        if (a.labels_out) a.labels_out[ds.idx_offset + i] = am;
                    }
                    wave_accumulate<D>(x, am, valid, d, pw, cw, atomic);
                }
                f = block_sum<NT>(fl, L.red);
                ++it;
                if (it >= a.max_iter || f == 0.0 || (f_prev - f) < a.rel_tol * f_prev) break;
                f_prev = f;
                for (int e = tid; e < k * D; e += NT) {
                    const int j = e / D, t = e % D;
                    double sum = 0.0;
                    int n = 0;
                    for (int g = 0; g < copies; ++g) {
                        sum += L.psum[(size_t)g * k * D + e];
                        n += L.pcnt[g * k + j];
                    }
                    float v = 0.f;
                    if (t < d) v = n > 0 ? (float)(sum / (double)n) : __builtin_nanf("");
                    L.Cs[e] = v;
                }
                __syncthreads();
            }
            if (tid == 0) {
                a.f_out[b] = f;
                a.iters_out[b] = it;
            }
        }
        for (int e = tid; e < k * d; e += NT) {
            const int j = e / d, t = e % d;
            a.C[ds.c_offset + e] = L.Cs[j * D + t];
        }
        __syncthreads();
    }
}

}  // namespace hpc

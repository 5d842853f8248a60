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
// Arithmetic: the assignment screens all centroids in FP32 and certifies the
// winner with a rigorous error bound (screen_certified); the rare point that
// is not certified is re-decided in FP64.  The distance that enters the
// objective, the K-means++ weights D^2, the potentials, the centroid sums
// and the centroids themselves are FP64.  Every index the method decides is
// therefore the one an FP64 evaluation decides.
//
// Layout per sample: the gathered rows live in a scratch buffer (row stride
// D floats, zero padded) that stays hot in L2/MALL across passes; centroids
// sit in LDS as FP64 plus an FP32 copy for the screening; per-wave FP64
// partial sums of the update live in LDS; D^2 lives in scratch, each element
// owned by one thread.
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
    float* sbuf;    // gathered samples, indexed by idx_offset, stride D
    double* d2buf;  // D^2, indexed by idx_offset
    int32_t* queue;
    int32_t kmax;
    int32_t n_copies;  // partial-sum copies in LDS (== waves: private per wave)
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
    double* C64;   // kmax x D centroids (FP64)
    float* C32;    // kmax x D centroids rounded to FP32 (screening)
    double* crow;  // 4 x D candidate rows
    double* psum;  // n_copies x kmax x D update sums   (union with seeding scan)
    int* pcnt;     // n_copies x kmax counts
    double* incl;  // NT inclusive scan of chunk sums   (seeding)
    double* red;   // 4 x NW wave partials
    double* cn;    // kmax squared centroid norms
    int* deg;      // kmax degenerate-row list
    int* ints;     // 16 scalars

    static __host__ __device__ size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

    static __host__ __device__ size_t union_bytes(int kmax, int copies) {
        size_t lloyd = (size_t)copies * kmax * D * 8 + align_up((size_t)copies * kmax * 4, 16);
        size_t seed = (size_t)NT * 8;
        return lloyd > seed ? lloyd : seed;
    }
    static __host__ __device__ size_t bytes(int kmax, int copies) {
        size_t b = (size_t)kmax * D * 8 + align_up((size_t)kmax * D * 4, 16) + 4 * D * 8;
        b += union_bytes(kmax, copies);
        b += 4 * NW * 8 + align_up((size_t)kmax * 8, 16);
        b += align_up((size_t)kmax * 4, 16) + 16 * 4;
        return b;
    }
    __device__ Smem(char* base, int kmax, int copies) {
        char* p = base;
        C64 = reinterpret_cast<double*>(p);
        p += (size_t)kmax * D * 8;
        C32 = reinterpret_cast<float*>(p);
        p += align_up((size_t)kmax * D * 4, 16);
        crow = reinterpret_cast<double*>(p);
        p += 4 * D * 8;
        psum = reinterpret_cast<double*>(p);
        pcnt = reinterpret_cast<int*>(p + (size_t)copies * kmax * D * 8);
        incl = reinterpret_cast<double*>(p);
        p += union_bytes(kmax, copies);
        red = reinterpret_cast<double*>(p);
        p += 4 * NW * 8;
        cn = reinterpret_cast<double*>(p);
        p += align_up((size_t)kmax * 8, 16);
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

// Copy sample row i (FP32, padded) into centroid row j (FP64 and FP32).
template <int D, int NT>
__device__ __forceinline__ void set_row_from_sample(double* dst64, float* dst32,
                                                    const float* __restrict__ Sg, int i) {
    for (int t = threadIdx.x; t < D; t += NT) {
        const float v = Sg[(size_t)i * D + t];
        dst64[t] = (double)v;
        dst32[t] = v;
    }
}

// ---------------------------------------------------------------------------
// K-means++ on the gathered sample for every degenerate row of L.C64, in
// FP64 (weights, prefix sums, potentials).  Sg: s x D rows; d2: s doubles
// of scratch.  Stream (seed, tag) / (block, sid, call, 0).  Thread t owns
// the contiguous chunk [t*cs, (t+1)*cs) of the sample; the inverse-CDF
// search is a workgroup scan of the chunk sums followed by a sequential
// scan inside the one chunk that holds the target, so the prefix order is
// the sample's index order.  chosen (nullable, global) receives the picked
// sample-local indices.  Seeded rows are written to C64 and C32.
// ---------------------------------------------------------------------------
template <int D, int NT>
__device__ void kmeanspp_wg(const float* __restrict__ Sg, int s, int k, int n_cand,
                            double* __restrict__ d2, uint64_t seed, uint64_t tag, uint64_t sid,
                            uint64_t call, int32_t* __restrict__ chosen, Smem<D, NT>& L) {
    const int tid = threadIdx.x;
    if (tid == 0) {
        int nd = 0, nv = 0;
        for (int j = 0; j < k; ++j) {
            if (L.C64[j * D] != L.C64[j * D])
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
        const Words4 w0 = philox_block(seed, tag, 0, sid, call);
        const int i0 = (int)bounded_index(w0.w[0], (uint64_t)s);
        const int j0 = L.deg[0];
        if (tid == 0 && chosen) chosen[j0] = i0;
        set_row_from_sample<D, NT>(L.C64 + j0 * D, L.C32 + j0 * D, Sg, i0);
        __syncthreads();
        for (int i = lo; i < hi; ++i) {
            float x[D];
            load_row<D>(Sg + (size_t)i * D, x);
            const double v = sqdist64<D>(x, L.C64 + j0 * D);
            d2[i] = v;
            acc += v;
        }
        first = 1;
    } else {
        for (int i = lo; i < hi; ++i) {
            float x[D];
            load_row<D>(Sg + (size_t)i * D, x);
            double best = __builtin_huge_val();
            for (int j = 0; j < k; ++j) {
                if (L.C64[j * D] != L.C64[j * D]) continue;
                const double v = sqdist64<D>(x, L.C64 + j * D);
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
                        run += d2[i];
                        if (run > target) {
                            found = i;
                            break;
                        }
                    }
                    if (found < 0)
                        for (int i = hi - 1; i >= lo; --i)
                            if (d2[i] > 0.0) {
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
                        if (d2[i] > 0.0) found = i;
                    L.ints[4 + t] = found < 0 ? 0 : found;
                }
            }
            __syncthreads();
            for (int e = tid; e < n_cand * D; e += NT)
                L.crow[e] = (double)Sg[(size_t)L.ints[4 + e / D] * D + (e % D)];
            __syncthreads();
            // one candidate at a time keeps a single FP64 row live
            double p[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                if (t >= n_cand) continue;
                double pt = 0.0;
                for (int i = lo; i < hi; ++i) {
                    float x[D];
                    load_row<D>(Sg + (size_t)i * D, x);
                    const double dd = d2[i];
                    const double v = sqdist64<D>(x, L.crow + t * D);
                    pt += v < dd ? v : dd;
                }
                p[t] = pt;
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
        set_row_from_sample<D, NT>(L.C64 + jr * D, L.C32 + jr * D, Sg, pick);
        __syncthreads();
        acc = 0.0;
        for (int i = lo; i < hi; ++i) {
            float x[D];
            load_row<D>(Sg + (size_t)i * D, x);
            const double v = sqdist64<D>(x, L.C64 + jr * D);
            const double o = d2[i];
            const double nv = v < o ? v : o;
            d2[i] = nv;
            acc += nv;
        }
        __syncthreads();
    }
}

// Rounding radius of the FP32 centroid copy: 2^-24 * max_j |c_j| (rounded
// up slightly so that its FP32 use stays conservative).  Two barriers.
template <int D, int NT>
__device__ __forceinline__ float centroid_round_radius(Smem<D, NT>& L, int k, int d) {
    for (int j = threadIdx.x; j < k; j += NT) {
        double n2 = 0.0;
        for (int t = 0; t < d; ++t) n2 += L.C64[j * D + t] * L.C64[j * D + t];
        L.cn[j] = n2;
    }
    __syncthreads();
    double mx = 0.0;
    for (int j = 0; j < k; ++j) mx = L.cn[j] > mx ? L.cn[j] : mx;
    __syncthreads();
    return (float)(sqrt(mx) * 0x1.0p-24 * 1.0001) + 1e-30f;
}

template <int D, int NT>
__global__ __launch_bounds__(NT) void k_lloyd_resident(LloydArgs a) {
    extern __shared__ __align__(16) char smem[];
    Smem<D, NT> L(smem, a.kmax, a.n_copies);
    constexpr int NW = Smem<D, NT>::NW;
    const int tid = threadIdx.x, wid = tid / kWave;
    const int d = a.d;
    const float tau = 4.f * (float)(d + 8) * 0x1.0p-24f;

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
        double* d2 = a.d2buf + ds.idx_offset;

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
            const float v = t < d ? a.C[ds.c_offset + (int64_t)j * d + t] : 0.f;
            L.C32[e] = v;
            L.C64[e] = (double)v;
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
            const bool shared_copy = copies < NW;
            for (;;) {
                kmeanspp_wg<D, NT>(Sg, s, k, 3, d2, ds.seed, kTagReseed, ds.sample_id,
                                   (uint64_t)it, nullptr, L);
                const float rmax = centroid_round_radius<D, NT>(L, k, d);
                for (int e = tid; e < copies * k * D; e += NT) L.psum[e] = 0.0;
                for (int e = tid; e < copies * k; e += NT) L.pcnt[e] = 0;
                __syncthreads();
                double* pw = L.psum + (size_t)(wid % copies) * k * D;
                int* cw = L.pcnt + (wid % copies) * k;
                double fl = 0.0;
                for (int base = 0; base < s; base += NT) {
                    const int i = base + tid;
                    if (i < s) {
                        float x[D];
                        load_row<D>(Sg + (size_t)i * D, x);
                        // FP32 screening: best and runner-up
                        float b1 = __builtin_huge_valf(), b2 = __builtin_huge_valf();
                        int am = 0;
                        for (int j = 0; j < k; ++j) {
                            const float v = sqdist<D>(x, L.C32 + j * D);
                            if (v < b1) {
                                b2 = b1;
                                b1 = v;
                                am = j;
                            } else if (v < b2) {
                                b2 = v;
                            }
                        }
                        double dm;
                        if (screen_certified(b1, b2, tau, rmax)) {
                            dm = sqdist64<D>(x, L.C64 + am * D);
                        } else {  // re-decide in FP64 (lowest index on ties)
                            dm = __builtin_huge_val();
                            for (int j = 0; j < k; ++j) {
                                const double v = sqdist64<D>(x, L.C64 + j * D);
                                if (v < dm) {
                                    dm = v;
                                    am = j;
                                }
                            }
                        }
                        fl += dm;
                        if (a.labels_out) a.labels_out[ds.idx_offset + i] = am;
                        double* ps = pw + am * D;
                        (void)shared_copy;
#pragma unroll
                        for (int t = 0; t < D; ++t)
                            if (t < d) atomicAdd(ps + t, (double)x[t]);
                        atomicAdd(cw + am, 1);
                    }
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
                    double v = 0.0;
                    if (t < d) v = n > 0 ? sum / (double)n : __builtin_nan("");
                    L.C64[e] = v;
                    L.C32[e] = (float)v;
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
            a.C[ds.c_offset + e] = (float)L.C64[j * D + t];
        }
        __syncthreads();
    }
}

}  // namespace hpc

// Workgroup-resident sample processing for gfx950.
//
// One workgroup owns one sample at a time and runs the whole per-sample
// method on it without leaving the kernel: gather of the sample rows,
// K-means++ seeding of degenerate centroids (Section 3; three candidates,
// Section 6.5), and the K-means passes (Algorithm 1) with the stop rule of
// Section 6.5.  A persistent grid pulls samples from a queue in
// longest-first order, so hundreds of samples of uneven size share one
// launch.  When samples are few (at least twice as many resident
// workgroups as samples), each sample is P consecutive queue tasks and a
// warm sample is worked by P workgroups, each on every P-th tile, with one
// exchange of partial sums per pass (see the pass loop); otherwise there is
// no inter-workgroup synchronisation at all.
//
// Arithmetic: the assignment screens all centroids on the matrix cores
// (FP32, BF16 or BF16x3 MFMA, mfma_screen.hpp) and certifies the winner
// with a rigorous error bound; a point that is not certified is re-decided
// in FP64.  The distance that enters the
// objective, the K-means++ weights D^2, the potentials, the centroid sums
// and the centroids themselves are FP64.  Every index the method decides is
// therefore the one an FP64 evaluation decides.
//
// Layout per sample: the gathered rows live in a scratch buffer (row stride
// D floats, zero padded) that stays hot in L2/MALL across passes; centroids
// sit in LDS as FP64 plus the MFMA A operands (-2c) and |c|^2; per-wave FP64
// partial sums of the update live in LDS; D^2 lives in scratch, each element
// owned by one thread.  Warm samples read their rows straight from X through
// their indices until a gathered copy pays (kDirectPasses).
#pragma once

#include "common.hpp"
#include "mfma_screen.hpp"

namespace hpc {

// Passes a warm sample reads straight from X before it gathers its rows.
constexpr int kDirectPasses = 15;

// Smallest objective, relative to the sample's scatter Q about its
// reference point, that is taken from the running sums (below it the
// points are summed directly; see the pass loop).
constexpr double kSumsObjectiveMin = 1e-2;

// A row of zeros in global memory, read in place of a row whose index lies
// outside [0, m) (never written).
__device__ float g_zero_row[128];

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
    double* d2buf;  // per sample, at 5 * idx_offset: D^2 (s) and the
                    // distances to the K-means++ candidates of a step (4 x s)
    int32_t* lbuf;  // label of each sample point in the previous pass, by idx_offset
    int32_t* queue;
    int32_t kmax;
    int32_t n_copies;  // partial-sum copies in LDS (== waves: private per wave)
    // seeding-only mode (the order of these fields moves the d <= 32 forms'
    // scalar register allocation: keep it)
    int32_t seed_only;
    int32_t n_cand;
    uint32_t call_id;
    int32_t* chosen;
    int32_t vec4;  // rows of X are 16-byte aligned (d % 4 == 0, aligned base)
    // shared samples: with split == P > 1 every sample is P queue tasks,
    // and a warm sample read straight from X is worked by P workgroups,
    // each on every P-th tile, which exchange their partial sums once per
    // pass
    int32_t split;
    double* xbuf;     // per sample, part and pass parity: xstride doubles
    int32_t* xflag;   // per sample four ints, zeroed per launch (parts_barrier)
    int32_t xstride;  // kmax * Lay<D>::CS + 8
};

// Workgroups per shared sample at most.
constexpr int kMaxParts = 16;

// Spin limit of a shared sample's per-pass wait for its partners (about a
// second); past it the sample is abandoned with f = NaN rather than waiting
// for ever.
constexpr int kPairSpinLimit = 1 << 20;

// A shared sample's flags (four ints, zeroed per launch): the passes counted
// by all its workgroups together, and the first workgroup's decision.
enum : int { kPairShared = 1, kPairAlone = 2 };

// The first workgroup's decision for its sample, as seen by the others
// (kPairAlone if it is not published within the spin limit).  One thread.
// Nothing the decision guards is read from the first workgroup's stores, so
// a relaxed load suffices.
__device__ inline int pair_decision(int32_t* flags) {
    for (int spin = 0; spin < kPairSpinLimit; ++spin) {
        const int v = __hip_atomic_load(flags + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (v != 0) return v;
        __builtin_amdgcn_s_sleep(1);
    }
    return kPairAlone;
}

// Count one more shared pass of this workgroup and wait until all `parts`
// workgroups of the sample have counted `target` passes each.  Called by one
// thread once every wave's slot stores (device-coherent, see store_dev) have
// completed; relaxed device-scope atomics, so no cache is written back or
// invalidated.  False if a partner did not arrive within the spin limit.
__device__ inline bool parts_barrier(int32_t* flags, int parts, int target) {
    __hip_atomic_fetch_add(flags, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int spin = 0;
         __hip_atomic_load(flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < parts * target;
         ++spin) {
        if (spin >= kPairSpinLimit) return false;
        __builtin_amdgcn_s_sleep(1);
    }
    return true;
}

// Rows of one gathered sample (stride D, zero padded).
template <int D>
struct SampleView {
    const float* base;
    __device__ __forceinline__ const float* row(int i) const { return base + (size_t)i * D; }
};

// Carving of the dynamic LDS allocation; the host computes the same size.
template <int D, int NT, int PREC>
struct Smem {
    static constexpr int NW = NT / kWave;
    static_assert(NW <= 16, "the per-wave flags of block_any take ints[16, 16 + NW)");
    double* C64;   // kmax rows of FP64 centroids, stride Lay<D>::CS
    void* aop;     // MFMA A operands, nblk x ... (see mfma_screen.hpp)
    float* nrm;    // nblk*16 score biases |c|^2
    double* crow;  // 4 x D candidate rows
    double* ref;   // D coordinates of the sample's reference point r
    double* psum;  // n_copies x kmax rows (stride CS) of running update sums
                   // of x - r; slot D of a row (the stride's padding) holds
                   // the count
    double* red;   // 4 x NW wave partials
    double* cn;    // kmax squared centroid norms
    int* deg;      // kmax degenerate-row list
    int* ints;     // 32 scalars; [16, 16 + NW) are block_any's per-wave flags

    static __host__ __device__ size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
    static __host__ __device__ int nblk_of(int kmax) { return (kmax + 15) / 16; }

    static __host__ __device__ size_t union_bytes(int kmax, int copies) {
        return (size_t)copies * kmax * Lay<D>::CS * 8;
    }
    static __host__ __device__ size_t bytes(int kmax, int copies) {
        const int nb = nblk_of(kmax);
        size_t b = align_up((size_t)kmax * Lay<D>::CS * 8, 16) + align_up(aop_bytes<D, PREC>(nb), 16) +
                   (size_t)nb * 64;
        b += 4 * D * 8 + D * 8;
        b += union_bytes(kmax, copies);
        b += 4 * NW * 8 + align_up((size_t)kmax * 8, 16);
        b += align_up((size_t)kmax * 4, 16) + 32 * 4;
        return b;
    }
    __device__ Smem(char* base, int kmax, int copies) {
        const int nb = nblk_of(kmax);
        char* p = base;
        C64 = reinterpret_cast<double*>(p);
        p += align_up((size_t)kmax * Lay<D>::CS * 8, 16);
        aop = p;
        p += align_up(aop_bytes<D, PREC>(nb), 16);
        nrm = reinterpret_cast<float*>(p);
        p += (size_t)nb * 64;
        crow = reinterpret_cast<double*>(p);
        p += 4 * D * 8;
        ref = reinterpret_cast<double*>(p);
        p += D * 8;
        psum = reinterpret_cast<double*>(p);
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

// Whether v holds on any thread of the workgroup (every thread gets the
// answer).  Two barriers; the first NT / 64 ints of `slots` are scratch.
template <int NT>
__device__ __forceinline__ bool block_any(bool v, int* slots) {
    constexpr int NW = NT / kWave;
    const bool w = __ballot(v) != 0ull;
    if ((threadIdx.x & (kWave - 1)) == 0) slots[threadIdx.x / kWave] = w ? 1 : 0;
    __syncthreads();
    int r = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) r |= slots[i];
    __syncthreads();
    return r != 0;
}

// Copy sample row i (FP32, padded) into an FP64 centroid row.
template <int D, int NT>
__device__ __forceinline__ void set_row_from_sample(double* dst64, const SampleView<D>& sv, int i) {
    const float* r = sv.row(i);
    for (int t = threadIdx.x; t < D; t += NT) dst64[t] = (double)r[t];
}

// ---------------------------------------------------------------------------
// K-means++ on the gathered sample for every degenerate row of L.C64, in
// FP64 (weights, prefix sums, potentials).  sv: the sample's rows; d2: s
// doubles of scratch.  Stream (seed, tag) / (block, sid, call, 0).
//
// Layout: wave w owns the contiguous chunk [w*cw, (w+1)*cw) of the sample
// (cw a multiple of 16) and walks it in tiles of 16 points; within a tile a
// lane holds a quarter of a point's coordinates, as in the assignment pass
// (mfma_screen.hpp), so a distance is four partial FP64 sums and two
// shuffles.  Weights D^2 of chunk w are read and written by wave w only.
// The inverse-CDF search locates the chunk from the chunk totals, then the
// owning wave scans its tiles in index order, four per step, each with a
// 16-lane FP64 prefix scan, so the prefix order is the sample's index order.  chosen
// (nullable, global) receives the picked sample-local indices.  Seeded rows
// are written to C64.
// ---------------------------------------------------------------------------
template <int D, int NT, int PREC>
__device__ void kmeanspp_wg(const SampleView<D>& sv, int s, int k, int n_cand,
                            double* __restrict__ d2, uint64_t seed, uint64_t tag, uint64_t sid,
                            uint64_t call, int32_t* __restrict__ chosen, Smem<D, NT, PREC>& L) {
    constexpr int NW = NT / kWave;
    constexpr int DL = Lay<D>::DL, CS = Lay<D>::CS;
    // the wave index is wave-uniform: kept in scalar registers, and with it
    // every LDS address derived from it
    const int tid = threadIdx.x, wid = __builtin_amdgcn_readfirstlane(tid / kWave),
              lane = tid & 63;
    const int g = lane >> 4, p = lane & 15;
    if (tid == 0) {
        int nd = 0, nv = 0;
        for (int j = 0; j < k; ++j) {
            if (L.C64[j * CS] != L.C64[j * CS])
                L.deg[nd++] = j;
            else
                ++nv;
        }
        L.ints[0] = nd;
        L.ints[1] = nv;
    }
    __syncthreads();
    const int n_deg = __builtin_amdgcn_readfirstlane(L.ints[0]),
              n_valid = __builtin_amdgcn_readfirstlane(L.ints[1]);
    if (n_deg == 0) return;

    const int cw = (((s + NW - 1) / NW) + 15) / 16 * 16;
    const int lo = min(s, wid * cw), hi = min(s, lo + cw);
    double* __restrict__ vc = d2 + s;  // candidate distances, n_cand x s
    auto load_pt = [&](int i, float (&xq)[DL]) {
        if (i < hi) {
            load_quarter<D>(sv.row(i), g, xq);
        } else {
#pragma unroll
            for (int t = 0; t < DL; ++t) xq[t] = 0.f;
        }
    };

    int first = 0;
    double acc = 0.0;  // this lane's share of the wave's chunk total (g == 0 lanes)
    if (n_valid == 0) {
        const Words4 w0 = philox_block(seed, tag, 0, sid, call);
        const int i0 = (int)bounded_index(w0.w[0], (uint64_t)s);
        const int j0 = L.deg[0];
        if (tid == 0 && chosen) chosen[j0] = i0;
        set_row_from_sample<D, NT>(L.C64 + j0 * CS, sv, i0);
        __syncthreads();
        for (int b0 = lo; b0 < hi; b0 += 16) {
            const int i = b0 + p;
            float xq[DL];
            load_pt(i, xq);
            const double v = quarter_dist64<D>(xq, L.C64 + j0 * CS);
            if (i < hi && g == 0) {
                d2[i] = v;
                acc += v;
            }
        }
        first = 1;
    } else {
        for (int b0 = lo; b0 < hi; b0 += 16) {
            const int i = b0 + p;
            float xq[DL];
            load_pt(i, xq);
            double best = __builtin_huge_val();
            for (int j = 0; j < k; ++j) {
                if (L.C64[j * CS] != L.C64[j * CS]) continue;
                const double v = quarter_dist64<D>(xq, L.C64 + j * CS);
                best = v < best ? v : best;
            }
            if (i < hi && g == 0) {
                d2[i] = best;
                acc += best;
            }
        }
    }

    for (int r = first; r < n_deg; ++r) {
        // chunk totals and their inclusive prefix over waves (index order)
        const double wsum = wave_sum(acc);
        if (lane == 0) L.red[wid] = wsum;
        __syncthreads();
        double c_lo = 0.0, W = 0.0;
        for (int w = 0; w < NW; ++w) {
            if (w == wid) c_lo = W;
            W += L.red[w];
        }
        const double c_hi = c_lo + L.red[wid];
        const uint64_t q = (uint64_t)(r + (n_valid > 0 ? 1 : 0));
        const Words4 w = philox_block(seed, tag, q, sid, call);
        int pick, tsel = -1;
        if (!(W > 0.0)) {
            pick = (int)bounded_index(w.w[0], (uint64_t)s);
            __syncthreads();
        } else {
            if (tid < 4) L.ints[4 + tid] = -1;
            __syncthreads();
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const double target = unit_double(w.w[t]) * W;
                if (t < n_cand && c_lo <= target && target < c_hi) {  // wave-uniform
                    // four tiles per step, one per group of 16 lanes; the
                    // running total passes the tiles in index order, one
                    // addition per tile, so every comparison is the one a
                    // tile-by-tile walk makes
                    double run = c_lo;
                    int found = -1;
                    for (int b0 = lo; b0 < hi && found < 0; b0 += 64) {
                        const int i = b0 + 16 * g + p;
                        double v = i < hi ? d2[i] : 0.0;
#pragma unroll
                        for (int o = 1; o < 16; o <<= 1) {
                            const double u = __shfl_up(v, o, 16);
                            if (p >= o) v += u;
                        }
                        double acc = run, rg = run;
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            if (q == g) rg = acc;
                            acc += __shfl(v, 16 * q + 15);
                        }
                        const bool hit = i < hi && rg + v > target;
                        const unsigned long long mk = __ballot(hit);
                        if (mk)
                            found = b0 + __ffsll(mk) - 1;  // lane 16 g + p is point b0 + 16 g + p
                        else
                            run = acc;
                    }
                    if (found < 0) {  // rounding: last point of positive weight in the chunk
                        for (int b0 = (hi - 1 - lo) / 16 * 16 + lo; b0 >= lo && found < 0; b0 -= 16) {
                            const int i = b0 + p;
                            const bool pos = i < hi && d2[i] > 0.0;
                            const unsigned long long m16 = __ballot(pos) & 0xFFFFull;
                            if (m16) found = b0 + 63 - __clzll(m16);
                        }
                    }
                    if (lane == 0) L.ints[4 + t] = found;
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
                L.crow[e] = (double)sv.row(L.ints[4 + e / D])[e % D];
            __syncthreads();
            // the potentials of all candidates in one stream over the chunk
            double pt[4] = {0.0, 0.0, 0.0, 0.0};
            for (int b0 = lo; b0 < hi; b0 += 16) {
                const int i = b0 + p;
                float xq[DL];
                load_pt(i, xq);
                const double dd = i < hi ? d2[i] : 0.0;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    if (t >= n_cand) continue;
                    const double v = quarter_dist64<D>(xq, L.crow + t * D);
                    if (i < hi && g == 0) {
                        pt[t] += v < dd ? v : dd;
                        vc[(size_t)t * s + i] = v;  // the D^2 update reads it back
                    }
                }
            }
            block_sum_n<NT, 4>(pt, L.red);
            int tb = 0;
            double pb = pt[0];
#pragma unroll
            for (int t = 1; t < 4; ++t)
                if (t < n_cand && pt[t] < pb) {
                    pb = pt[t];
                    tb = t;
                }
            pick = L.ints[4 + tb];
            tsel = tb;
        }
        const int jr = L.deg[r];
        if (tid == 0 && chosen) chosen[jr] = pick;
        set_row_from_sample<D, NT>(L.C64 + jr * CS, sv, pick);
        __syncthreads();
        acc = 0.0;
        if (tsel >= 0) {
            // the chosen candidate's distances were stored by the lanes
            // that read them back: no second pass over the rows
            const double* vt = vc + (size_t)tsel * s;
            for (int b0 = lo; b0 < hi; b0 += 16) {
                const int i = b0 + p;
                if (i < hi && g == 0) {
                    const double v = vt[i], o = d2[i];
                    const double nv = v < o ? v : o;
                    d2[i] = nv;
                    acc += nv;
                }
            }
        } else {
            for (int b0 = lo; b0 < hi; b0 += 16) {
                const int i = b0 + p;
                float xq[DL];
                load_pt(i, xq);
                const double v = quarter_dist64<D>(xq, L.C64 + jr * CS);
                if (i < hi && g == 0) {
                    const double o = d2[i];
                    const double nv = v < o ? v : o;
                    d2[i] = nv;
                    acc += nv;
                }
            }
        }
        __syncthreads();
    }
}

// Largest centroid norm max_j |c_j| over valid rows.  Two barriers.
template <int D, int NT, int PREC>
__device__ __forceinline__ double centroid_max_norm(Smem<D, NT, PREC>& L, int k, int d) {
    constexpr int CS = Lay<D>::CS;
    for (int j = threadIdx.x; j < k; j += NT) {
        double n2 = 0.0;
        if (L.C64[j * CS] == L.C64[j * CS])
            for (int t = 0; t < d; ++t) n2 = __fma_rn(L.C64[j * CS + t], L.C64[j * CS + t], n2);
        L.cn[j] = n2;
    }
    __syncthreads();
    double mx = 0.0;
    for (int j = 0; j < k; ++j) mx = L.cn[j] > mx ? L.cn[j] : mx;
    __syncthreads();
    return sqrt(mx);
}

// Up to d = 32 the kernel without shared samples is held to 128 VGPRs (four
// waves per SIMD): the tile loop then runs at twice the occupancy, at the
// price of a few spilled values in the seeding and gather paths.  SHARE
// compiles the shared-sample paths (always for d > 32; up to d = 32 a
// separate form for batches of few samples, at two waves per SIMD).
template <int D, int NT, int PREC, bool SHARE>
__global__ __launch_bounds__(NT, (D <= 32 && !SHARE) ? 4 : 2) void k_lloyd_resident(LloydArgs a) {
    extern __shared__ __align__(16) char smem[];
    using S = Smem<D, NT, PREC>;
    constexpr int DL = Lay<D>::DL, CS = Lay<D>::CS;
    S L(smem, a.kmax, a.n_copies);
    constexpr int NW = S::NW;
    const int tid = threadIdx.x, wid = __builtin_amdgcn_readfirstlane(tid / kWave),
              lane = tid & 63;
    const int g = lane >> 4, pl = lane & 15;
    const int d = a.d;
    double alpha, beta;
    screen_coeffs<PREC>(d, &alpha, &beta);

    // shared samples exist in the SHARE forms only (up to d = 32 the other
    // form has no scalar or vector registers to spare for them)
    const int NP = SHARE ? a.split : 1;
    const bool two = SHARE && NP > 1;
    // every workgroup's first task is its own index (no atomic on one
    // address from the whole grid at once); later ones come from the queue
    bool first_task = true;
    for (;;) {
        if (tid == 0)
            L.ints[15] = first_task ? (int)blockIdx.x : (int)gridDim.x + atomicAdd(a.queue, 1);
        first_task = false;
        __syncthreads();
        // uniform across the workgroup: the sample's descriptor, sizes and
        // base pointers then live in scalar registers
        const int task = __builtin_amdgcn_readfirstlane(L.ints[15]);
        __syncthreads();
        if (task >= NP * a.n_samples) break;
        // with shared samples the P tasks of a sample are consecutive: they
        // are handed out one after another, so a workgroup never waits for a
        // partner that no workgroup will take
        const int slot = two ? task / NP : task, half = two ? task % NP : 0;
        const int b = a.order ? a.order[slot] : slot;
        const hpc_sample_desc ds = a.desc[b];
        const int s = ds.s, k = ds.k;
        const int nblk = (k + 15) / 16;
        float* Sg = a.sbuf + (size_t)ds.idx_offset * D;
        double* d2 = a.d2buf + 5 * (size_t)ds.idx_offset;
        int32_t* lprev = a.lbuf + ds.idx_offset;
        int32_t* lab_out = a.labels_out ? a.labels_out + ds.idx_offset : nullptr;
        const SampleView<D> sv{Sg};

        // gather the sample rows (zero padded to D): consecutive threads
        // copy consecutive 16-byte chunks of a row; eight chunks per thread
        // are loaded before any is stored, so the random-row loads overlap
        auto gather = [&]() {
            constexpr int NCH = D / 4;
            const int total = s * NCH;
            for (int base = tid; base < total; base += 8 * NT) {
                float4 v[8];
                int dst[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int e = base + u * NT;
                    dst[u] = -1;
                    v[u] = make_float4(0.f, 0.f, 0.f, 0.f);
                    if (e < total) {
                        const int i = e / NCH, col = (e % NCH) * 4;
                        const int64_t row = a.idx[ds.idx_offset + i];
                        const bool in_range = row >= 0 && row < a.m;  // else a zero row
                        dst[u] = i * D + col;
                        if (in_range && col < d) {
                            const float* src = a.X + row * d + col;
                            if (a.vec4) {
                                v[u] = *reinterpret_cast<const float4*>(src);
                            } else {
                                v[u].x = src[0];
                                v[u].y = col + 1 < d ? src[1] : 0.f;
                                v[u].z = col + 2 < d ? src[2] : 0.f;
                                v[u].w = col + 3 < d ? src[3] : 0.f;
                            }
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (dst[u] >= 0) *reinterpret_cast<float4*>(Sg + dst[u]) = v[u];
            }
            __syncthreads();
        };
        // the second workgroup of a sample takes no decision of its own: it
        // waits for the first one's (the centroids it would judge by are
        // rewritten when the first workgroup finishes a sample alone)
        int32_t* const pflags = two ? a.xflag + 4 * slot : nullptr;
        if (half > 0) {
            if (tid == 0) L.ints[14] = pair_decision(pflags);
            __syncthreads();
            const int dec = __builtin_amdgcn_readfirstlane(L.ints[14]);
            __syncthreads();
            if (dec != kPairShared) continue;
        }
        for (int e = tid; e < k * CS; e += NT) {
            const int j = e / CS, t = e % CS;
            L.C64[e] = t < d ? (double)a.C[ds.c_offset + (int64_t)j * d + t] : 0.0;
        }
        __syncthreads();
        // a sample that starts with every centroid valid is read straight
        // from X through its indices (rows of exactly D floats, 16-byte
        // aligned); the gathered copy is made when K-means++ needs the
        // sample (a degenerate row at the start or after an update) or when
        // the sample runs long
        auto any_degenerate = [&]() {
            int deg = 0;
            for (int j = tid; j < k; j += NT) deg |= L.C64[j * CS] != L.C64[j * CS];
            return block_any<NT>(deg != 0, L.ints + 16);
        };
        // seeding only: a block with no degenerate row (seeded already by
        // the team kernel, or all valid) is left as it is
        const bool direct_ok = !a.seed_only && a.vec4 && d == D;
        bool gathered = !direct_ok || any_degenerate();
        // a sample is shared only while it reads its rows straight from X
        // with every centroid valid; both workgroups take this decision
        // (and every later one) from identical data.  (Where samples can be
        // shared, the flags are read through readfirstlane: wave-uniform,
        // so the tile mapping derived from them stays in scalar registers.)
        if (two) gathered = __builtin_amdgcn_readfirstlane(gathered);
        bool paired = two && !gathered;
        if (two && half == 0 && tid == 0)
            __hip_atomic_store(pflags + 2, paired ? kPairShared : kPairAlone, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        if (half > 0 && !paired) continue;  // (same data as the first: does not happen)
        if (gathered) gather();

        if (a.seed_only) {
            if (a.chosen)
                for (int j = tid; j < k; j += NT) a.chosen[j] = -1;
            __syncthreads();
            kmeanspp_wg<D, NT, PREC>(sv, s, k, a.n_cand, d2, ds.seed, kTagSeed, ds.sample_id,
                                     a.call_id, a.chosen, L);
        } else {
            double f_prev = __builtin_huge_val(), f = 0.0, Qr = 0.0;
            int it = 0;
            const int copies = a.n_copies;
            unsigned kmask;
            float qscale;
            key_params(nblk, &kmask, &qscale);
            // the exchange slot of part hh of a shared sample, for the parity
            // of pass p; slot NP holds the totals over the parts
            auto xslot = [&](int hh, int p) {
                return a.xbuf + (((size_t)slot * (NP + 1) + hh) * 2 + (p & 1)) * a.xstride;
            };
            // leaving a shared sample (a reseed, the gathered copy or the
            // direct-sum objective is needed): the other workgroups stop; the
            // first adds their partial sums of pass p, the last exchange, to
            // its own and continues alone.  True if this workgroup leaves.
            // The partners' previous labels (lprev) of their tiles were
            // written device-coherently; this workgroup's caches may still
            // hold lines of them from its own tiles' accesses, so it
            // invalidates them once before reading every tile.
            // the sum over parts [h0, NP) of the sample (part order, identical
            // in every part) of element e of the pass-p slots; every load is
            // issued before the first is used
            auto parts_sum = [&](int p, int e, int h0) {
                double v[kMaxParts];
#pragma unroll
                for (int hh = 0; hh < kMaxParts; ++hh)
                    v[hh] = hh >= h0 && hh < NP ? load_dev(xslot(hh, p) + e) : 0.0;
                double sum = 0.0;
#pragma unroll
                for (int hh = 0; hh < kMaxParts; ++hh)
                    if (hh >= h0 && hh < NP) sum += v[hh];
                return sum;
            };
            auto unpair = [&](int p) {
                paired = false;
                if (half > 0) return true;
                for (int e = tid; e < k * CS; e += NT) L.psum[e] += parts_sum(p, e, 1);
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                __syncthreads();
                return false;
            };
            bool left = false;
            for (;;) {
                // reading rows through the indices costs more per pass than
                // reading the gathered copy (scattered 128-byte rows against
                // contiguous ones; measured at about a fifteenth of the
                // copy's cost): a sample still running after kDirectPasses
                // passes makes the copy, which bounds the loss to about twice
                // the better choice made in hindsight
                const bool deg = __builtin_amdgcn_readfirstlane(any_degenerate());
                if (!gathered && it > 0 && (it >= kDirectPasses || deg)) {
                    if (paired && unpair(it - 1)) {
                        left = true;
                        break;
                    }
                    gather();
                    gathered = true;
                }
                // the flags are set under branches on workgroup-wide values
                // the compiler cannot see are uniform: restate that they are
                if (two) {
                    gathered = __builtin_amdgcn_readfirstlane(gathered);
                    paired = __builtin_amdgcn_readfirstlane(paired);
                }
                if (deg)
                    kmeanspp_wg<D, NT, PREC>(sv, s, k, 3, d2, ds.seed, kTagReseed, ds.sample_id,
                                             (uint64_t)it, nullptr, L);
                const double cmax = centroid_max_norm<D, NT, PREC>(L, k, d);
                const float ea = (float)(alpha * cmax), eb = (float)(beta * cmax * cmax);
                build_operands<D, PREC, NT>(L.C64, k, d, nblk, L.aop, L.nrm);
                // the sums and counts run across passes: the first pass adds
                // every point, later passes only the points whose label
                // changed.  They are sums of x - r for a reference point r
                // fixed per sample (the mean of the first pass's centroids,
                // rounded to FP32 so that x - r is exact in FP64), which keeps
                // them and the objective below free of cancellation.
                const bool first = it == 0;
                if (first) {
                    for (int e = tid; e < copies * k * CS; e += NT) L.psum[e] = 0.0;
                    for (int t = tid; t < D; t += NT) {
                        double sum = 0.0;
                        int nv = 0;
                        for (int j = 0; j < k; ++j)
                            if (L.C64[j * CS] == L.C64[j * CS]) {
                                sum += L.C64[j * CS + t];
                                ++nv;
                            }
                        L.ref[t] = t < d && nv > 0 ? (double)(float)(sum / nv) : 0.0;
                    }
                }
                __syncthreads();
                lds_f64* pw = as_lds(L.psum + (size_t)(wid % copies) * k * CS);
                // tiles in pass order: a shared sample's workgroup takes every
                // P-th one (tile v of this workgroup is tile P v + part)
                const int tmul = paired ? NP : 1, toff = paired ? half : 0;
                auto TI = [&](int v) { return v * tmul + toff; };
                double fl = 0.0;
                // tiles of 16 points per wave, software pipelined over three
                // register buffers: the rows of the next two tiles are in
                // flight while one tile is processed (unrolled by three so
                // that no buffer with a load in flight is ever copied)
                float xa[DL], xb[DL], xc[DL];
                int la, lb, lc;
                // branch-free: rows past the end re-read the last row (their
                // lanes are masked in process), which keeps the memory
                // counters exact for the compiler's wait placement
                auto fetch = [&](int tile, float (&dst)[DL], int& old) {
                    const int i = min(TI(tile) * 16 + pl, s - 1);
                    load_quarter<D>(Sg + (size_t)i * D, g, dst);
                    old = lprev[(unsigned)i];
                };
                auto process = [&](int tile, const float (&xq)[DL], int old) {
                    const int i = TI(tile) * 16 + pl;
                    const bool valid = i < s;
                    const float xn2 = point_norm2<D>(xq);
                    const float xn = cert_norm(xn2);
                    const float h = screen_shift(xn2, xn, ea, eb);
                    // (rows of 64 and more run at two waves per SIMD, with
                    // the registers to interleave two blocks' MFMA chains)
                    const Top3 t3 = screen_tile<D, PREC, (D >= 64)>(xq, L.aop, L.nrm, nblk, h, kmask);
                    const bool ok = certified(t3, kmask, qscale, xn, ea, eb) || !valid;
                    const int a1 = (int)key_index(t3.t1, kmask), a2 = (int)key_index(t3.t2, kmask);
                    const int am = redecide64<D, PREC>(
                        xq, t3, !ok, top2_suffices(t3, kmask, qscale, xn, ea, eb), a1,
                        a2 < k ? a2 : a1, L.C64, L.aop, L.nrm, nblk, h, kmask, qscale, xn, ea, eb);
                    if (valid) {
                        // a point that changed cluster moves x - r between the
                        // running sums (padded coordinates of x and r are
                        // zero, so their sums stay exactly zero); in the first
                        // pass every point does, and adds its share of
                        // Q = sum |x - r|^2
                        const int prev = first ? -1 : old;
                        if (am != prev) {
                            const double* rq = L.ref + g * DL;
                            double xr[DL];
#pragma unroll
                            for (int t = 0; t < DL; ++t) xr[t] = (double)xq[t] - rq[t];
                            if (first) {
                                double part = 0.0;
#pragma unroll
                                for (int t = 0; t < DL; ++t) part = __fma_rn(xr[t], xr[t], part);
                                fl += part;
                            }
                            lds_f64* pn = pw + (am * CS + g * DL);
#pragma unroll
                            for (int t = 0; t < DL; ++t) lds_add(pn + t, xr[t]);
                            if (prev >= 0) {
                                lds_f64* po = pn + (prev - am) * CS;
#pragma unroll
                                for (int t = 0; t < DL; ++t) lds_add(po + t, -xr[t]);
                            }
                            if (g == 0) {
                                // counts are small integers, exact in FP64
                                lds_add(pw + (am * CS + D), 1.0);
                                if (prev >= 0) lds_add(pw + (prev * CS + D), -1.0);
                                // read by the first workgroup if a shared
                                // sample ends: device-coherent while shared
                                if (SHARE && paired)
                                    store_dev(lprev + (unsigned)i, am);
                                else
                                    lprev[(unsigned)i] = am;
                            }
                        }
                        if (g == 0 && lab_out) {
                            // while shared, device-coherent as well: a plain
                            // store would leave this part's L2 line dirty,
                            // and its write-back could land after the labels
                            // the first workgroup writes for the same points
                            // once it continues alone (L2 lines span the
                            // tiles of several parts)
                            if (SHARE && paired)
                                store_dev(lab_out + (unsigned)i, am);
                            else
                                lab_out[(unsigned)i] = am;
                        }
                    }
                };
                if (gathered) {
                    fetch(wid, xa, la);
                    fetch(wid + NW, xb, lb);
                    for (int tile = wid; TI(tile) * 16 < s; tile += 3 * NW) {
                        fetch(tile + 2 * NW, xc, lc);
                        process(tile, xa, la);
                        if (TI(tile + NW) * 16 >= s) break;
                        fetch(tile + 3 * NW, xa, la);
                        process(tile + NW, xb, lb);
                        if (TI(tile + 2 * NW) * 16 >= s) break;
                        fetch(tile + 4 * NW, xb, lb);
                        process(tile + 2 * NW, xc, lc);
                    }
                } else {
                    // rows straight from X: each tile's indices are loaded
                    // two tiles before its rows, so a row load never waits
                    // on rows still in flight
                    const int64_t* ix = a.idx + ds.idx_offset;
                    auto IDX = [&](int tile) -> int64_t {
                        return ix[(unsigned)min(TI(tile) * 16 + pl, s - 1)];
                    };
                    // an index outside [0, m) reads a row of zeros, as the
                    // gather does (a pointer select: nothing touches the
                    // loaded registers before they are used)
                    auto ROW = [&](int tile, int64_t r, float (&dst)[DL], int& old) {
                        const float* src = (r >= 0 && r < a.m) ? a.X + r * D : g_zero_row;
                        load_quarter<D>(src, g, dst);
                        old = lprev[(unsigned)min(TI(tile) * 16 + pl, s - 1)];
                    };
                    // the prologue issues its loads in the order the loop
                    // body does (the scheduling barriers stop the compiler
                    // from sinking the third tile's indices, which would make
                    // the loop head wait for every load in flight)
                    int64_t ia = IDX(wid), ib = IDX(wid + NW), ic = IDX(wid + 2 * NW);
                    __builtin_amdgcn_sched_barrier(0);
                    ROW(wid, ia, xa, la);
                    __builtin_amdgcn_sched_barrier(0);
                    ROW(wid + NW, ib, xb, lb);
                    __builtin_amdgcn_sched_barrier(0);
                    ia = IDX(wid + 3 * NW);
                    ib = IDX(wid + 4 * NW);
                    __builtin_amdgcn_sched_barrier(0);
                    // no early exit inside the body (the loads past the end
                    // are clamped and cheap; skipped tiles are not processed)
                    for (int tile = wid; TI(tile) * 16 < s; tile += 3 * NW) {
                        ROW(tile + 2 * NW, ic, xc, lc);
                        ic = IDX(tile + 5 * NW);
                        process(tile, xa, la);
                        ROW(tile + 3 * NW, ia, xa, la);
                        ia = IDX(tile + 6 * NW);
                        if (TI(tile + NW) * 16 < s) process(tile + NW, xb, lb);
                        ROW(tile + 4 * NW, ib, xb, lb);
                        ib = IDX(tile + 7 * NW);
                        if (TI(tile + 2 * NW) * 16 < s) process(tile + 2 * NW, xc, lc);
                    }
                }
                // The pass objective from the sums: with S_j the sum of x - r
                // and n_j the count over the points now labelled j, and c_j
                // this pass's centroids, sum_i |x_i - c_a(i)|^2 = Q +
                // sum_j (n_j |c_j - r|^2 - 2 (c_j - r).S_j).  Where the
                // clustering leaves less than kSumsObjectiveMin of Q, the
                // cancellation would cost digits, and the points' FP64
                // distances are summed directly instead (which also keeps an
                // exact zero exact).
                __syncthreads();
                // A shared sample's workgroups exchange their partial sums
                // (in the first pass also their shares of Q) through
                // device-coherent stores and loads: every part publishes its
                // running sums; after a first barrier part h adds up the h-th
                // P-th of the elements over all parts (in part order),
                // publishes these totals and its share of the objective's
                // centroid term; after a second barrier every part reads the
                // totals.  Every part then holds the same objective and
                // centroids.
                bool xch = false;  // this pass's totals come from the exchange
                const int E = k * CS;
                double* const tot = xslot(NP, it);
                auto arrive = [&](int target) {
                    if (tid == 0) L.ints[14] = parts_barrier(pflags, NP, target);
                    __syncthreads();
                    return __builtin_amdgcn_readfirstlane(L.ints[14]) != 0;
                };
                if (paired) {
                    double* mine = xslot(half, it);
                    for (int e = tid; e < E; e += NT) {
                        double S = 0.0;
                        for (int gg = 0; gg < copies; ++gg) S += L.psum[(size_t)gg * E + e];
                        store_dev(mine + e, S);
                    }
                    if (first) {
                        fl = block_sum<NT>(fl, L.red);  // this workgroup's share of Q
                        if (tid == 0) store_dev(mine + E, fl);
                    }
                    wait_stores();
                    __syncthreads();
                    bool arrived = arrive(2 * it + 1);
                    if (arrived) {
                        const int lo = (int)((int64_t)E * half / NP);
                        const int hi = (int)((int64_t)E * (half + 1) / NP);
                        double fph = 0.0;
                        for (int e = lo + tid; e < hi; e += NT) {
                            const int j = e / CS, t = e % CS;
                            const double S = parts_sum(it, e, 0);
                            store_dev(tot + e, S);
                            if (t < d) {
                                const double n = parts_sum(it, j * CS + D, 0);
                                if (n > 0.0) {
                                    const double dc = L.C64[e] - L.ref[t];
                                    fph = __fma_rn(dc, __fma_rn(n, dc, -2.0 * S), fph);
                                }
                            }
                        }
                        fph = block_sum<NT>(fph, L.red);
                        if (tid == 0) store_dev(mine + E + 1, fph);
                        wait_stores();
                        __syncthreads();
                        arrived = arrive(2 * it + 2);
                    }
                    if (!arrived) {
                        // a partner never came: abandon the sample
                        // (f = NaN, passes = -1)
                        f = __builtin_nan("");
                        it = -1;
                        paired = false;
                        left = half > 0;
                        break;
                    }
                    xch = true;
                }
                double fp = 0.0;
                if (xch) {
                    // (the same loads in every thread: a uniform value)
                    fp = parts_sum(it, E + 1, 0);
                    if (first) Qr = parts_sum(it, E, 0);
                } else {
                    for (int e = tid; e < E; e += NT) {
                        const int j = e / CS, t = e % CS;
                        if (t >= d) continue;
                        double S = 0.0, n = 0.0;
                        for (int gg = 0; gg < copies; ++gg) {
                            S += L.psum[(size_t)gg * E + e];
                            n += L.psum[(size_t)gg * E + j * CS + D];
                        }
                        if (n > 0.0) {
                            const double dc = L.C64[e] - L.ref[t];
                            fp = __fma_rn(dc, __fma_rn(n, dc, -2.0 * S), fp);
                        }
                    }
                    if (first) {
                        double v2[2] = {fl, fp};
                        block_sum_n<NT, 2>(v2, L.red);
                        Qr = v2[0];
                        fp = v2[1];
                    } else {
                        fp = block_sum<NT>(fp, L.red);
                    }
                }
                f = Qr + fp;
                if (!(f > kSumsObjectiveMin * Qr)) {
                    if (paired) {
                        if (unpair(it)) {
                            left = true;
                            break;
                        }
                        xch = false;
                    }
                    const int64_t* ixs = a.idx + ds.idx_offset;
                    double fe = 0.0;
                    for (int tile = wid; tile * 16 < s; tile += NW) {
                        const int i = tile * 16 + pl, ic = min(i, s - 1);
                        float xq[DL];
                        if (gathered) {
                            load_quarter<D>(Sg + (size_t)ic * D, g, xq);
                        } else {
                            const int64_t r = ixs[(unsigned)ic];
                            load_quarter<D>((r >= 0 && r < a.m) ? a.X + r * D : g_zero_row, g,
                                            xq);
                        }
                        const int lab = lprev[(unsigned)ic];
                        if (i < s) fe += quarter_part64<D>(xq, L.C64 + lab * CS);
                    }
                    f = block_sum<NT>(fe, L.red);
                }
                ++it;
                if (it >= a.max_iter || f == 0.0 || (f_prev - f) < a.rel_tol * f_prev) break;
                f_prev = f;
                if (xch) {
                    // the totals of pass it - 1, four elements per thread at
                    // a time with their loads in flight together
                    for (int e0 = tid; e0 < E; e0 += 4 * NT) {
                        double sv[4], nv[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int e = min(e0 + u * NT, E - 1);
                            sv[u] = load_dev(tot + e);
                            nv[u] = load_dev(tot + (e / CS) * CS + D);
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int e = e0 + u * NT, t = e % CS;
                            if (e >= E) break;
                            double v = 0.0;
                            if (t < d) v = nv[u] > 0.0 ? L.ref[t] + sv[u] / nv[u] : __builtin_nan("");
                            L.C64[e] = v;
                        }
                    }
                } else {
                    for (int e = tid; e < E; e += NT) {
                        const int j = e / CS, t = e % CS;
                        double sum = 0.0, n = 0.0;
                        for (int gg = 0; gg < copies; ++gg) {
                            sum += L.psum[(size_t)gg * E + e];
                            n += L.psum[(size_t)gg * E + j * CS + D];
                        }
                        double v = 0.0;
                        if (t < d) v = n > 0.0 ? L.ref[t] + sum / n : __builtin_nan("");
                        L.C64[e] = v;
                    }
                }
                __syncthreads();
            }
            // the first workgroup of a shared sample writes its results
            if (tid == 0 && half == 0) {
                a.f_out[b] = f;
                a.iters_out[b] = it;
            }
            if (__builtin_amdgcn_readfirstlane(left)) continue;
        }
        if (half == 0)
            for (int e = tid; e < k * d; e += NT) {
                const int j = e / d, t = e % d;
                a.C[ds.c_offset + e] = (float)L.C64[j * CS + t];
            }
        __syncthreads();
    }
}

}  // namespace hpc

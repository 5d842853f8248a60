// K-means++ seeding of cold samples (Section 3: the first sample's centroids
// come from K-means++; Section 6.5: three candidate points per new centroid)
// by teams of workgroups.
//
// A cold sample (every centroid row degenerate) is split over a team of T
// workgroups, each owning a contiguous slice of the sample's points in
// index order (whole groups of 256 points).  Each of the k - 1 greedy steps
// then costs one pass over the slice per workgroup plus one exchange
// between the team's workgroups:
//
//   1. every workgroup knows every slice's total weight W_b = sum of D^2 and
//      its group sums, so all of them compute the same D^2-weighted targets
//      and find each target's slice and group; the point inside the group
//      comes from the owner's 256 weights in global memory (written before
//      the owner arrived at the last exchange);
//   2. every workgroup computes, for its slice and each candidate t, the
//      would-be weights min(|x - c_t|^2, D^2), their sums per group of 256
//      points and over the slice, and publishes the sums;  -- the exchange
//   3. every workgroup adds the slice sums (in the same order in all of
//      them), keeps the candidate of smallest potential (lowest t on ties)
//      and adopts that candidate's weights: its slice and group sums are
//      the next W_b and group sums.
//
// With T = 1 there is no exchange and the workgroup runs the same steps
// alone (batches of many cold samples).  Everything a decision depends on
// is FP64: distances (FP32 coordinates, exact FP64 differences), weights,
// sums, potentials, targets; the decisions are then those of an FP64
// evaluation up to the order of the sums.
//
// Layout: the slice's rows are read from the gathered copy of the sample
// (stride D, zero padded), D / 8 lanes per point with 8 coordinates each,
// in groups of 256 points (see kpp_stream); the candidates' coordinates
// are FP64 in registers for the whole pass.  D^2 lives in five rotating
// buffers of s doubles per sample: the weights of
// the step's candidates go to the four buffers not read, and the kept
// candidate's buffer becomes the current one, so no pass updates D^2.
// Group sums live in LDS, one array per buffer, and guide the inverse-CDF
// search to one group of 256 weights.
//
// Exchanges: per team a monotonic arrival counter and per workgroup a slot
// (two step parities); a workgroup publishes its slot, waits for its stores
// to complete, counts its arrival and waits for the whole team, within a
// bounded spin.  Everything one workgroup reads from another (slots, the
// weights of a group) is stored and loaded as relaxed device-scope atomics,
// which are coherent across the XCDs' caches without fences: a device-scope
// fence writes back or invalidates a whole L2, which at every exchange of
// every team would cost all workgroups on that XCD their cached data.  A team that runs out of the spin (not
// expected: the host launches a team form only when every workgroup of the
// grid is resident at once) gives up: its workgroups leave the kernel and
// the rows of the samples it has not finished stay degenerate, which the
// Lloyd kernel then seeds itself from the same random stream.
#pragma once

#include "common.hpp"

namespace hpc {

constexpr int kKppGroup = 256;            // points per group sum (four tiles of 64)
constexpr int kKppBuffers = 5;            // rotating D^2 buffers per sample
constexpr int kTeamSpinLimit = 1 << 20;   // about a second of waiting per exchange

struct KppArgs {
    const float* X;
    int64_t m;
    int32_t d;
    const int64_t* idx;
    const hpc_sample_desc* desc;
    const int32_t* order;  // processing order (longest first); may be null
    int32_t n_samples;
    float* C;              // centroid blocks; a sample is cold when all its rows are degenerate
    int32_t n_cand;        // candidates per step, 1..4
    uint32_t tag;          // stream tag (kTagSeed for the seeding call, kTagReseed in Lloyd)
    uint32_t call_id;
    int32_t* chosen;       // nullable: picked sample-local index per row (first sample)
    int32_t vec4;          // rows of X are 16-byte aligned (d % 4 == 0, aligned base)
    float* sbuf;           // gathered rows, by idx_offset, stride D
    double* d2buf;         // kKppBuffers * s doubles per sample at kKppBuffers * idx_offset
    int32_t team;          // workgroups per sample (T)
    int32_t n_teams;       // grid = n_teams * team
    int32_t ngmax;         // group sums per buffer in LDS (largest slice / 256)
    int32_t kmax;
    int32_t* queue;        // next task for T == 1 (zeroed per launch)
    int32_t* tflag;        // per team: arrivals, abort (zeroed per launch)
    double* tx;            // per team 2 * T slots of kpp_slot_doubles(ngmax) doubles
};

constexpr int kMaxTeam = 64;               // workgroups per team at most

// Team barrier number e (every workgroup of the team calls it with the same
// e, from one thread, once the workgroup's exchanged data -- written with
// device-coherent stores -- has completed).  The arrival count and the wait
// are relaxed device-scope atomics, so no cache is written back or
// invalidated.  False if the team gave up (abort flag) or the wait ran
// out, which then sets the flag.
__device__ inline bool team_barrier(int32_t* flags, int T, int e) {
    __hip_atomic_fetch_add(flags, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int target = T * (e + 1);
    for (int spin = 0;; ++spin) {
        if (__hip_atomic_load(flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target)
            return true;
        if (__hip_atomic_load(flags + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
            return false;
        if (spin >= kTeamSpinLimit) {
            __hip_atomic_store(flags + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// Inclusive prefix sum over the 64 lanes (lane order).
__device__ __forceinline__ double wave_incl_scan(double v) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const double u = __shfl_up(v, o, kWave);
        if (lane >= o) v += u;
    }
    return v;
}

// The inverse-CDF step of K-means++ inside one slice, by one whole wave:
// the first point i of [lo, hi) (index order) at which carry plus the
// running weight exceeds x.  gt: the slice's group sums (LDS), w: the
// sample's weights.  Returns -1 if no group's running sum exceeds x, -2 if
// a group does but, by rounding, none of its points (every lane gets the
// same answer).
__device__ inline int kpp_find(const double* gt, int ngroups, const double* __restrict__ w, int lo,
                               int hi, double carry, double x, bool coh) {
    const int lane = threadIdx.x & (kWave - 1);
    int q = -1;
    for (int base = 0; base < ngroups; base += kWave) {
        const int gi = base + lane;
        const double v = gi < ngroups ? gt[gi] : 0.0;
        const double inc = wave_incl_scan(v);
        const double run = carry + inc;
        const unsigned long long hit = __ballot(gi < ngroups && run > x);
        if (hit) {
            const int l = __ffsll((long long)hit) - 1;
            const double ex = __shfl(inc - v, l, kWave);  // before group base + l
            carry = carry + ex;
            q = base + l;
            break;
        }
        carry = __shfl(run, kWave - 1, kWave);
    }
    if (q < 0) return -1;
    const int g0 = lo + q * kKppGroup;
    // the group's weights, all four tiles' loads in flight at once
    constexpr int U = kKppGroup / kWave;
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int i = min(g0 + u * kWave + lane, hi - 1);
        v[u] = coh ? load_dev(w + i) : w[i];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int i = g0 + u * kWave + lane;
        const double vi = i < hi ? v[u] : 0.0;
        const double run = carry + wave_incl_scan(vi);
        const unsigned long long hit = __ballot(i < hi && run > x);
        if (hit) return g0 + u * kWave + __ffsll((long long)hit) - 1;
        carry = __shfl(run, kWave - 1, kWave);
    }
    return -2;
}

// Last point of positive weight in [lo, hi), or -1 (one whole wave).
__device__ inline int kpp_last_positive(const double* __restrict__ w, int lo, int hi, bool coh) {
    const int lane = threadIdx.x & (kWave - 1);
    for (int top = hi; top > lo; top -= kWave) {
        const int i = top - kWave + lane;
        const bool pos = i >= lo && (coh ? load_dev(w + i) : w[i]) > 0.0;
        const unsigned long long mk = __ballot(pos);
        if (mk) return top - kWave + 63 - __clzll((long long)mk);
    }
    return -1;
}

// Last point of positive weight in group q of a slice, or -1.
__device__ inline int kpp_last_positive_group(const double* __restrict__ w, int lo, int hi, int q,
                                              bool coh) {
    const int g0 = lo + q * kKppGroup;
    return kpp_last_positive(w, g0, min(hi, g0 + kKppGroup), coh);
}

// Sum over the LP lanes of a point, which sit 64 / LP lanes apart (lane =
// j * (64 / LP) + p for point p and dimension chunk j): rotations by 4 and 8
// within rows of 16 lanes (DPP) and the row swaps by 16 and 32 (permlane),
// all VALU.  The lanes of a point may differ in the last bit; the value of
// chunk 0's lane is the one used.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
template <int LP>
__device__ __forceinline__ double point_sum(double v) {
    static_assert(LP == 1 || LP == 2 || LP == 4 || LP == 8 || LP == 16, "lanes per point");
    if constexpr (LP == 16) v += dpp_f64<0x124>(v);  // row_ror:4
    if constexpr (LP >= 8) v += dpp_f64<0x128>(v);   // row_ror:8
    if constexpr (LP >= 4) v = pair_sum<16>(v);
    if constexpr (LP >= 2) v = pair_sum<32>(v);
    return v;
}

// One pass over the slice [lo, hi) of a sample (rows sg, stride D): for each
// point and candidate t < NC the would-be weight nd_t = min(|x - c_t|^2, D^2)
// (D^2 from `in`; without `in` the distance itself) goes to out[t]; the sums
// of nd_t per group of 256 points go to gto[t] (LDS) and this thread's share
// of the slice sums is added to pot[t].
//
// Layout: LP = D / 8 lanes per point, each with 8 coordinates; a tile is
// 64 / LP consecutive points, a group TPG tiles.  A lane holds its 8
// coordinates of every candidate (FP64) in registers for the whole pass, so
// the pass reads no LDS; the tiles go in batches whose loads are all in
// flight at once.  A slice of at least NW groups gives each wave whole
// groups (group q to wave q mod NW).  A smaller slice -- a team's slices
// of one cold sample -- would leave waves idle and one wave's chain of
// TPG dependent tiles per group on the critical path: there every group is
// shared by all waves (tile u of a group to wave u mod NW), each wave's
// share of a group sum goes to `part` (LDS, 4 x NW x NW doubles) and the
// shares are added in wave order.  Every thread of the workgroup calls it.
template <int D, int NT, int NC>
__device__ void kpp_stream(const float* __restrict__ sg, int lo, int hi, const double* crow,
                           const double* __restrict__ in, bool first, bool coh,
                           double* const (&out)[4], double* const (&gto)[4], double (&pot)[4],
                           double* part) {
    constexpr int NW = NT / kWave;
    constexpr int LP = D / 8, PPT = kWave / LP, TPG = kKppGroup / PPT;
    static_assert(TPG % NW == 0, "a group's tiles split evenly over the waves");
    constexpr int TPW = TPG / NW;  // tiles of a shared group per wave
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int p = lane % PPT, j = lane / PPT;  // point within the tile, dimension chunk
    const int ng = (hi - lo + kKppGroup - 1) / kKppGroup;
    const bool shared = ng < NW;
    if (ng == 0 || (!shared && wid >= ng)) return;  // (uniform over the workgroup)
    double cr[NC][8];
#pragma unroll
    for (int t = 0; t < NC; ++t)
#pragma unroll
        for (int u = 0; u < 8; ++u) cr[t][u] = crow[t * D + 8 * j + u];
    // the wave's tiles in order.  Whole groups: tile f is tile f % TPG of
    // group wid + NW * (f / TPG).  Shared groups: tile f is tile
    // wid + NW * (f % TPW) of group f / TPW.
    const int per_group = shared ? TPW : TPG;
    const int nt = shared ? ng * TPW : ((ng - 1 - wid) / NW + 1) * TPG;
    auto group_of = [&](int f) { return shared ? f / per_group : wid + NW * (f / per_group); };
    auto point = [&](int f) {
        const int u = f % per_group;
        return lo + group_of(f) * kKppGroup + (shared ? wid + NW * u : u) * PPT + p;
    };
    // branch-free loads (tiles past the wave's last and points past the
    // slice end re-read the last ones), so that the compiler's wait for a
    // tile's rows leaves the next tiles' loads in flight
    auto fetch = [&](int f, float4 (&x)[2], double& dd) {
        const int i = point(min(f, nt - 1));
        const int ic = min(i, hi - 1);
        const float4* r = reinterpret_cast<const float4*>(sg + (size_t)ic * D + 8 * j);
        x[0] = r[0];
        x[1] = r[1];
        dd = in[ic];
    };
    double gp[NC];
#pragma unroll
    for (int t = 0; t < NC; ++t) gp[t] = 0.0;
    // the would-be weights of tile f (every lane of a point gets them)
    auto dist = [&](const float4 (&x)[2], double dd, double (&nd)[NC]) {
        if (first) dd = __builtin_huge_val();  // the first centre: D^2 is the distance
        const double xv[8] = {x[0].x, x[0].y, x[0].z, x[0].w, x[1].x, x[1].y, x[1].z, x[1].w};
#pragma unroll
        for (int t = 0; t < NC; ++t) {
            double acc = 0.0;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const double e = xv[u] - cr[t][u];
                acc = __fma_rn(e, e, acc);
            }
            acc = point_sum<LP>(acc);
            // every lane of the point holds the same sum (up to 8 lanes the
            // pairwise sums take their operands in lane order); with 16 the
            // first lane's is taken
            if constexpr (LP == 16) acc = __shfl(acc, p, kWave);
            nd[t] = acc < dd ? acc : dd;
        }
    };
    // tile f's weights into the group sums, which are complete when f ends
    // the wave's share of a group; tiles past the wave's last (f >= nt),
    // computed on re-read rows, count nothing
    auto account = [&](int f, const double (&nd)[NC]) {
        const bool valid = f < nt;
        const bool mine = valid && point(f) < hi && j == 0;  // the lane that counts the point
#pragma unroll
        for (int t = 0; t < NC; ++t) gp[t] += mine ? nd[t] : 0.0;
        if (valid && f % per_group == per_group - 1) {
            const int q = group_of(f);
#pragma unroll
            for (int t = 0; t < NC; ++t) {
                const double gs = wave_sum(gp[t]);
                if (lane == 0) {
                    if (shared)
                        part[(t * NW + q) * NW + wid] = gs;
                    else
                        gto[t][q] = gs;
                }
                pot[t] += lane == 0 ? gs : 0.0;
                gp[t] = 0.0;
            }
        }
    };
    // every lane stores, without a branch: the lanes of a point, points past
    // the slice end and tiles past the wave's last write the same values to
    // the same (clamped) places as the lanes that own them, so that the
    // compiler's count of memory operations in flight stays exact
    auto store = [&](int f, const double (&nd)[NC]) {
        const int ic = min(point(min(f, nt - 1)), hi - 1);
#pragma unroll
        for (int t = 0; t < NC; ++t) {
            // read by the other workgroups of a team: device-coherent
            if (coh)
                store_dev(out[t] + ic, nd[t]);
            else
                out[t][ic] = nd[t];
        }
    };
    // batches of KB tiles, software pipelined: a batch's rows and weights
    // are all in flight before its first tile is computed, and its results
    // are stored only after the next batch's loads are issued, so that no
    // load waits behind a store (vector memory operations complete in order)
    constexpr int KB = NC <= 3 ? 4 : 2;  // (within 256 registers: two waves per SIMD)
    float4 xs[KB][2];
    double dv[KB];
#pragma unroll
    for (int u = 0; u < KB; ++u) fetch(u, xs[u], dv[u]);
    for (int f0 = 0; f0 < nt; f0 += KB) {
        // the batch's distances first (no branch between its tiles, so that
        // their FP64 chains interleave), then the sums
        double nd[KB][NC];
#pragma unroll
        for (int u = 0; u < KB; ++u) dist(xs[u], dv[u], nd[u]);
#pragma unroll
        for (int u = 0; u < KB; ++u) account(f0 + u, nd[u]);
        // (unconditional: past the wave's last tile the loads re-read it)
#pragma unroll
        for (int u = 0; u < KB; ++u) fetch(f0 + KB + u, xs[u], dv[u]);
#pragma unroll
        for (int u = 0; u < KB; ++u) store(f0 + u, nd[u]);
    }
    if (shared) {
        __syncthreads();
        const int tid = threadIdx.x;
        if (tid < NC * ng) {
            const int t = tid / ng, q = tid % ng;
            double acc = 0.0;
#pragma unroll
            for (int w = 0; w < NW; ++w) acc += part[(t * NW + q) * NW + w];
            gto[t][q] = acc;
        }
        __syncthreads();
    }
}

// kpp_stream with the candidate count as a compile-time constant.
template <int D, int NT>
__device__ __forceinline__ void kpp_stream_n(int nc, const float* __restrict__ sg, int lo, int hi,
                                             const double* crow, const double* __restrict__ in,
                                             bool coh, double* const (&out)[4],
                                             double* const (&gto)[4], double (&pot)[4],
                                             double* part) {
    switch (nc) {
        case 1: kpp_stream<D, NT, 1>(sg, lo, hi, crow, in, false, coh, out, gto, pot, part); break;
        case 2: kpp_stream<D, NT, 2>(sg, lo, hi, crow, in, false, coh, out, gto, pot, part); break;
        case 3: kpp_stream<D, NT, 3>(sg, lo, hi, crow, in, false, coh, out, gto, pot, part); break;
        default: kpp_stream<D, NT, 4>(sg, lo, hi, crow, in, false, coh, out, gto, pot, part); break;
    }
}

// Doubles of one workgroup's exchange slot (per parity): the candidates'
// slice sums, then per candidate the slice's group sums.
__host__ __device__ inline int kpp_slot_doubles(int ngmax) { return 4 + 4 * ngmax; }

// Dynamic LDS of the seeding kernel for teams of T with ngmax group sums per
// slice and at most kmax centroids.
template <int D, int NT>
__host__ __device__ inline size_t kpp_lds_bytes(int ngmax, int kmax, int T) {
    const size_t dbl = (size_t)4 * ngmax           // the stream's group sums per candidate
                       + (size_t)T * ngmax         // every slice's group sums (current weights)
                       + 4 * (size_t)D             // candidate rows
                       + 4 * (NT / kWave)          // workgroup sums
                       + 4 * (NT / kWave) * (NT / kWave)  // shared groups' wave shares
                       + (size_t)T                 // every slice's weight
                       + (size_t)T * kpp_slot_doubles(ngmax)  // one exchange, gathered
                       + 8;                        // potentials
    return dbl * 8 + ((size_t)kmax * 4 + 15) / 16 * 16 + 64 * 4;
}

// Cold samples of a batch, one per team of `team` workgroups (see above).
//
// One exchange per step: every workgroup publishes, for each candidate, its
// slice's sum and group sums of the would-be weights.  After the exchange
// every workgroup knows the kept candidate, hence every slice's weight and
// group sums, and finds all the next step's candidates itself: the owner
// slice and group from the sums (LDS), the point from the owner's 256
// weights of that group in global memory (written before the owner arrived).
template <int D, int NT>
__global__ __launch_bounds__(NT) void k_kmeanspp_team(KppArgs a) {
    constexpr int NW = NT / kWave;
    static_assert(NW >= 4, "one wave per candidate in the search");
    extern __shared__ __align__(16) char smem[];
    const int T = a.team, ngmax = a.ngmax, SD = kpp_slot_doubles(ngmax);
    double* gtmp = reinterpret_cast<double*>(smem);  // 4 x ngmax: this slice's group sums
    double* ggs = gtmp + 4 * ngmax;                  // T x ngmax: every slice's, current weights
    double* crow = ggs + (size_t)T * ngmax;          // 4 x D
    double* red = crow + 4 * D;                      // 4 x NW
    double* part = red + 4 * NW;                     // 4 x NW x NW: shared groups' wave shares
    double* wts = part + 4 * NW * NW;                // T: every slice's weight
    double* tsl = wts + T;                           // T x SD: one exchange's slots
    double* pv = tsl + (size_t)T * SD;               // 8
    int* picks = reinterpret_cast<int*>(pv + 8);     // kmax
    int* ints = picks + ((size_t)a.kmax * 4 + 15) / 16 * 4;  // 64

    const int tid = threadIdx.x, lane = tid & (kWave - 1);
    const int wid = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int tau = blockIdx.x % a.n_teams, b = blockIdx.x / a.n_teams;
    int32_t* const flags = a.tflag + 4 * tau;
    double* const xs = a.tx + (size_t)tau * 2 * T * SD;
    const int d = a.d;
    int ebar = 0;  // team barriers passed

    // every wave's device-coherent stores complete, then arrive and wait;
    // every thread returns whether the team is still alive
    const bool coh = T > 1;
    auto team_sync = [&]() -> bool {
        wait_stores();
        __syncthreads();
        if (tid == 0) ints[1] = team_barrier(flags, T, ebar) ? 1 : 0;
        __syncthreads();
        ++ebar;
        return __builtin_amdgcn_readfirstlane(ints[1]) != 0;
    };
    auto slot = [&](int par, int member) { return xs + ((size_t)par * T + member) * SD; };

    for (int it = 0;; ++it) {
        int task;
        if (T == 1) {
            if (tid == 0) ints[0] = it == 0 ? (int)blockIdx.x : (int)gridDim.x + atomicAdd(a.queue, 1);
            __syncthreads();
            task = __builtin_amdgcn_readfirstlane(ints[0]);
            __syncthreads();
        } else {
            task = tau + it * a.n_teams;
        }
        if (task >= a.n_samples) break;
        const int sidx = a.order ? a.order[task] : task;
        const hpc_sample_desc ds = a.desc[sidx];
        const int s = ds.s, k = ds.k;
        // cold: every row degenerate (the same answer in every workgroup)
        int warm = 0;
        for (int j = tid; j < k; j += NT) {
            const float v = a.C[ds.c_offset + (int64_t)j * d];
            warm |= v == v;
        }
        if (__syncthreads_or(warm)) continue;

        // the slices: whole groups of 256 points, in team order
        const int per = ((s + T - 1) / T + kKppGroup - 1) / kKppGroup * kKppGroup;
        auto slice_lo = [&](int q) { return min(s, q * per); };
        auto slice_hi = [&](int q) { return min(s, q * per + per); };
        auto slice_ng = [&](int q) {
            return (slice_hi(q) - slice_lo(q) + kKppGroup - 1) / kKppGroup;
        };
        const int lo = slice_lo(b), hi = slice_hi(b), ngr = slice_ng(b);
        float* const sg = a.sbuf + (size_t)ds.idx_offset * D;
        double* const wb = a.d2buf + (size_t)kKppBuffers * ds.idx_offset;
        auto buf = [&](int j) { return wb + (size_t)j * s; };
        const int64_t* const ix = a.idx + ds.idx_offset;

        // gather the slice's rows (zero padded to D); an index outside
        // [0, m) reads a row of zeros
        {
            constexpr int NCH = D / 4;
            const int total = (hi - lo) * NCH;
            for (int base = tid; base < total; base += 8 * NT) {
                float4 v[8];
                int dst[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int e = base + u * NT;
                    dst[u] = -1;
                    v[u] = make_float4(0.f, 0.f, 0.f, 0.f);
                    if (e < total) {
                        const int i = lo + e / NCH, col = (e % NCH) * 4;
                        const int64_t row = ix[i];
                        dst[u] = i * D + col;
                        if (row >= 0 && row < a.m && col < d) {
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
                    if (dst[u] >= 0) *reinterpret_cast<float4*>(sg + dst[u]) = v[u];
            }
        }

        // candidate rows into LDS as FP64, from X through the sample's
        // indices (X is never written, so every workgroup reads them
        // without an exchange)
        auto load_rows = [&](const int (&cand)[4], int nc) {
            for (int e = tid; e < 4 * D; e += NT) {
                const int t = e / D, col = e % D;
                double v = 0.0;
                if (t < nc && col < d) {
                    const int ct = t == 0 ? cand[0] : t == 1 ? cand[1] : t == 2 ? cand[2] : cand[3];
                    const int64_t row = ix[ct];
                    if (row >= 0 && row < a.m) v = (double)a.X[row * d + col];
                }
                crow[e] = v;
            }
        };
        // the first centre: uniform over the sample (block 0, word 0)
        const Words4 w0 = philox_block(ds.seed, a.tag, 0, ds.sample_id, a.call_id);
        const int i0 = (int)bounded_index(w0.w[0], (uint64_t)s);
        if (tid == 0) picks[0] = i0;
        {
            const int c0[4] = {i0, i0, i0, i0};
            load_rows(c0, 1);
        }
        __syncthreads();
        auto block_pot = [&](double (&v)[4]) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const double ws = wave_sum(v[t]);
                if (lane == 0) red[t * NW + wid] = ws;
            }
            __syncthreads();
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                double acc = 0.0;
#pragma unroll
                for (int w = 0; w < NW; ++w) acc += red[t * NW + w];
                v[t] = acc;
            }
            __syncthreads();
        };
        // publish this slice's sums of nc candidates, exchange, keep the
        // candidate of smallest potential (lowest index on ties) and adopt
        // its weights and group sums for every slice; returns the kept
        // candidate, or -1 if the team gave up
        int par = 0;
        auto exchange = [&](const double (&pt)[4], int nc) -> int {
            if (T > 1) {
                par ^= 1;
                double* my = slot(par, b);
                for (int e = tid; e < SD; e += NT) {
                    double v = 0.0;
                    if (e < 4) {
                        v = e < nc ? pt[e] : 0.0;
                    } else {
                        const int t = (e - 4) / ngmax, q = (e - 4) % ngmax;
                        v = (t < nc && q < ngr) ? gtmp[t * ngmax + q] : 0.0;
                    }
                    store_dev(my + e, v);
                }
                if (!team_sync()) return -1;
                for (int e = tid; e < T * SD; e += NT) tsl[e] = load_dev(slot(par, e / SD) + e % SD);
                __syncthreads();
                if (wid < 4) {  // wave t adds candidate t's slice sums
                    const double v = lane < T ? tsl[lane * SD + wid] : 0.0;
                    const double acc = wave_sum(v);
                    if (lane == 0) pv[wid] = acc;
                }
            } else if (tid < 4) {
                pv[tid] = pt[tid];
            }
            __syncthreads();
            int tb = 0;
#pragma unroll
            for (int t = 1; t < 4; ++t)
                if (t < nc && pv[t] < pv[tb]) tb = t;
            if (T > 1) {
                for (int e = tid; e < T; e += NT) wts[e] = tsl[e * SD + tb];
                for (int e = tid; e < T * ngmax; e += NT) {
                    const int q = e / ngmax, g = e % ngmax;
                    ggs[e] = tsl[q * SD + 4 + tb * ngmax + g];
                }
            } else {
                if (tid == 0) wts[0] = pv[tb];
                for (int e = tid; e < ngmax; e += NT) ggs[e] = e < ngr ? gtmp[tb * ngmax + e] : 0.0;
            }
            __syncthreads();
            return tb;
        };
        // D^2 from the first centre: the weights in buffer 0
        double pot[4] = {0.0, 0.0, 0.0, 0.0};
        {
            double* const o[4] = {buf(0), buf(0), buf(0), buf(0)};
            double* const g[4] = {gtmp, gtmp, gtmp, gtmp};
            kpp_stream<D, NT, 1>(sg, lo, hi, crow, buf(0), true, coh, o, g, pot, part);
        }
        block_pot(pot);
        int cur = 0;
        bool alive = exchange(pot, 1) >= 0;
        for (int r = 1; r < k && alive; ++r) {
            const Words4 w = philox_block(ds.seed, a.tag, (uint64_t)r, ds.sample_id, a.call_id);
            // every slice's running end in team order, one slice per lane (a
            // team has at most 64 workgroups), and W, the last one: the same
            // values in every workgroup
            const double wq = lane < T ? wts[lane] : 0.0;
            const double wend = wave_incl_scan(wq);
            const double W = __shfl(wend, kWave - 1, kWave);
            int pick;
            if (!(W > 0.0)) {
                pick = (int)bounded_index(w.w[0], (uint64_t)s);
            } else {
                // wave t finds candidate t: the slice whose running end first
                // exceeds the target (or, the target rounded up to W, the last
                // slice of positive weight), then the group and the point
                const int nc = a.n_cand;
                const double* const wcur = buf(cur);
                if (wid < nc) {
                    const double x = unit_double(w.w[wid]) * W;
                    const unsigned long long over = __ballot(lane < T && wend > x);
                    const unsigned long long pos = __ballot(lane < T && wq > 0.0);
                    int owner = over ? __ffsll((long long)over) - 1 : -1;
                    const int last_pos = pos ? 63 - __clzll((long long)pos) : -1;
                    // the running end of the slices before the owner
                    const double prev = __shfl_up(wend, 1, kWave);
                    double off = 0.0;
                    if (owner > 0) off = __shfl(prev, owner, kWave);
                    int found = -1;
                    const bool rounded_up = owner < 0;
                    if (rounded_up) owner = last_pos;
                    const int olo = slice_lo(owner), ohi = slice_hi(owner), ong = slice_ng(owner);
                    const double* og = ggs + (size_t)owner * ngmax;
                    if (!rounded_up) {
                        found = kpp_find(og, ong, wcur, olo, ohi, off, x, coh);
                        if (found == -2) {
                            // in a group by its sum, in none of its points by
                            // theirs: the group's last point of positive weight
                            double c2 = off;
                            int q2 = 0;
                            for (; q2 < ong; ++q2) {
                                if (c2 + og[q2] > x) break;
                                c2 += og[q2];
                            }
                            found = kpp_last_positive_group(wcur, olo, ohi, min(q2, ong - 1), coh);
                        }
                    }
                    if (found < 0) found = kpp_last_positive(wcur, olo, ohi, coh);
                    found = found < 0 ? 0 : found;
                    if (lane == 0) ints[8 + wid] = found;
                    // the candidate's row into LDS (FP64), read by this wave
                    const int64_t row = ix[found];
                    const bool in_range = row >= 0 && row < a.m;
                    for (int col = lane; col < D; col += kWave)
                        crow[wid * D + col] =
                            (in_range && col < d) ? (double)a.X[row * d + col] : 0.0;
                }
                __syncthreads();
                const int cand[4] = {ints[8], ints[9], ints[10], ints[11]};
                // the candidates' would-be weights into the four buffers
                // other than the current one
                double* o[4];
                double* const g[4] = {gtmp, gtmp + ngmax, gtmp + 2 * ngmax, gtmp + 3 * ngmax};
#pragma unroll
                for (int t = 0; t < 4; ++t) o[t] = buf((cur + 1 + t) % kKppBuffers);
                double pt[4] = {0.0, 0.0, 0.0, 0.0};
                kpp_stream_n<D, NT>(nc, sg, lo, hi, crow, wcur, coh, o, g, pt, part);
                block_pot(pt);
                const int tb = exchange(pt, nc);
                alive = tb >= 0;
                if (!alive) break;
                pick = cand[tb];
                cur = (cur + 1 + tb) % kKppBuffers;
            }
            if (tid == 0) picks[r] = pick;
        }
        __syncthreads();
        if (!alive) return;  // the team gave up: its remaining samples stay cold
        // the first workgroup writes the seeded rows (copies of sample rows)
        if (b == 0) {
            for (int e = tid; e < k * d; e += NT) {
                const int j = e / d, col = e % d;
                const int64_t row = ix[picks[j]];
                a.C[ds.c_offset + e] = (row >= 0 && row < a.m) ? a.X[row * d + col] : 0.f;
            }
            if (a.chosen)
                for (int j = tid; j < k; j += NT) a.chosen[j] = picks[j];
        }
        __syncthreads();
    }
}

}  // namespace hpc

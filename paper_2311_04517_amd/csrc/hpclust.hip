// Host side of the C ABI declared in include/hpclust.h: argument
// validation, per-(device, stream) scratch workspaces, launch shapes, and
// dispatch of the gfx950 kernels on the padded dimension D.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "../../include/hpclust.h"
#include "assign_misc.hpp"
#include "common.hpp"
#include "host_util.hpp"
#include "kmeanspp_team.hpp"
#include "lloyd_resident.hpp"

namespace {
thread_local std::string g_last_error = "";
}  // namespace

namespace hpc_host {
int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}
}  // namespace hpc_host

namespace {

using hpc_host::fail;

constexpr int kMaxD = 128;
constexpr int kNT = 512;  // threads per workgroup of the resident kernels

int pad_dim(int d) {
    if (d <= 8) return 8;
    if (d <= 16) return 16;
    if (d <= 32) return 32;
    if (d <= 64) return 64;
    return 128;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Pinned host slots through which descriptor tables reach the device: a
// slot is refilled only after the copy out of it has run, so an upload
// waits on the host only when every slot's copy is still queued.
constexpr int kStageSlots = 8;

struct StageSlot {
    void* host = nullptr;
    size_t cap = 0;
    hipEvent_t copied = nullptr;  // the copy out of this slot
};

// Grow-only device scratch plus the pinned staging slots, one per (device,
// stream).
struct Workspace {
    void* dev = nullptr;
    size_t dev_cap = 0;
    StageSlot stage[kStageSlots];
    int next_slot = 0;
    hipStream_t stream = nullptr;
    int device = 0;
};

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, Workspace*> g_ws;

int get_ws(hipStream_t stream, Workspace** out) {
    int dev = 0;
    HPC_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_mu);
    auto key = std::make_pair(dev, stream);
    auto it = g_ws.find(key);
    if (it == g_ws.end()) {
        Workspace* w = new Workspace();
        w->stream = stream;
        w->device = dev;
        for (auto& sl : w->stage) HPC_HIP(hipEventCreateWithFlags(&sl.copied, hipEventDisableTiming));
        it = g_ws.emplace(key, w).first;
    }
    *out = it->second;
    return HPC_OK;
}

// Make sure the device scratch holds `bytes`.  Growing frees the old buffer
// only after the stream has drained, so queued kernels never see it vanish.
int ws_reserve_dev(Workspace* w, size_t bytes) {
    if (bytes <= w->dev_cap) return HPC_OK;
    size_t cap = std::max(bytes, w->dev_cap + w->dev_cap / 2);
    cap = align_up(cap, 1 << 20);
    if (w->dev) {
        HPC_HIP(hipStreamSynchronize(w->stream));
        HPC_HIP(hipFree(w->dev));
        w->dev = nullptr;
        w->dev_cap = 0;
    }
    hipError_t e = hipMalloc(&w->dev, cap);
    if (e != hipSuccess) {
        w->dev = nullptr;
        return fail(HPC_ERR_NO_MEMORY, "scratch allocation of %zu bytes failed: %s", cap,
                    hipGetErrorString(e));
    }
    w->dev_cap = cap;
    return HPC_OK;
}

// Copy `bytes` of host data to device scratch at `dst` on the stream through
// the next pinned slot.  The host waits only if that slot's previous copy
// has not run yet (more than kStageSlots uploads queued on the stream).
int ws_upload(Workspace* w, void* dst, const void* src, size_t bytes) {
    StageSlot& sl = w->stage[w->next_slot];
    w->next_slot = (w->next_slot + 1) % kStageSlots;
    const hipError_t q = hipEventQuery(sl.copied);
    if (q == hipErrorNotReady)
        HPC_HIP(hipEventSynchronize(sl.copied));
    else if (q != hipSuccess)
        return fail(HPC_ERR_HIP, "hipEventQuery failed: %s", hipGetErrorString(q));
    if (bytes > sl.cap) {
        if (sl.host) HPC_HIP(hipHostFree(sl.host));
        sl.host = nullptr;
        sl.cap = 0;
        const size_t cap = align_up(std::max(bytes, (size_t)4096), 4096);
        HPC_HIP(hipHostMalloc(&sl.host, cap, hipHostMallocDefault));
        sl.cap = cap;
    }
    memcpy(sl.host, src, bytes);
    HPC_HIP(hipMemcpyAsync(dst, sl.host, bytes, hipMemcpyHostToDevice, w->stream));
    HPC_HIP(hipEventRecord(sl.copied, w->stream));
    return HPC_OK;
}

struct Carve {
    char* base;
    size_t off = 0;
    explicit Carve(void* b) : base(static_cast<char*>(b)) {}
    void* take(size_t bytes) {
        void* p = base + off;
        off = align_up(off + bytes, 256);
        return p;
    }
    static size_t need(std::initializer_list<size_t> parts) {
        size_t t = 0;
        for (size_t p : parts) t = align_up(t + p, 256);
        return t;
    }
};

int device_cus(int* cus) {
    int dev = 0;
    HPC_HIP(hipGetDevice(&dev));
    HPC_HIP(hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, dev));
    return HPC_OK;
}

int max_dyn_lds(int* bytes) {
    int dev = 0;
    HPC_HIP(hipGetDevice(&dev));
    HPC_HIP(hipDeviceGetAttribute(bytes, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    return HPC_OK;
}

bool precision_ok(int32_t p) {
    return p == HPC_PREC_FP32 || p == HPC_PREC_BF16_MFMA || p == HPC_PREC_BF16X3_MFMA;
}

// Call f(integral_constant<int, D>, integral_constant<int, PREC>) for the
// padded dimension D and the precision mode.
template <class F>
int with_dp(int D, int prec, F&& f) {
    using std::integral_constant;
#define HPC_DP(DD)                                                                            \
    case DD:                                                                                  \
        if (prec == HPC_PREC_BF16_MFMA)                                                       \
            return f(integral_constant<int, DD>{}, integral_constant<int, hpc::kPrecBF16>{});   \
        if (prec == HPC_PREC_BF16X3_MFMA)                                                     \
            return f(integral_constant<int, DD>{}, integral_constant<int, hpc::kPrecBF16x3>{}); \
        return f(integral_constant<int, DD>{}, integral_constant<int, hpc::kPrecF32>{})
    switch (D) {
        HPC_DP(8);
        HPC_DP(16);
        HPC_DP(32);
        HPC_DP(64);
        HPC_DP(128);
    }
#undef HPC_DP
    return fail(HPC_ERR_UNSUPPORTED, "padded dimension %d", D);
}

// --------------------------------------------------------------------------
// Resident Lloyd / seeding launch.
// --------------------------------------------------------------------------
struct ResGeo {
    int grid = 1;        // workgroups launched
    int copies = 1;      // private partial-sum copies per workgroup
    size_t lds = 0;      // dynamic LDS bytes
    int per_cu_max = 0;  // occupancy limit at this LDS size
    int split = 1;       // workgroups per sample (P > 1: shared warm samples)
    bool share = false;  // the kernel form with the shared-sample paths
};

// Doubles of the exchange buffer for n samples of `parts` workgroups: per
// part and for the totals two pass parities, and per slot the partial sums
// (kmax rows of D + 1), Q and the part's share of the objective.
size_t xbuf_doubles(int n, int parts, int kmax, int D) {
    return (size_t)n * (parts + 1) * 2 * ((size_t)kmax * (D + 1) + 8);
}

// Points a part of a shared sample keeps at least (eight tiles per wave).
constexpr int kMinPartPoints = 1024;

// The resident kernel's form: up to d = 32 the shared-sample paths live in
// a separate form; wider rows always have them.
template <int D>
constexpr bool share_form(bool shared) {
    return D >= 64 ? true : shared;
}

// Parts per sample a batch can use at most (s_min points in its smallest
// sample).
int parts_limit(int s_min) {
    return std::max(1, std::min(hpc::kMaxParts, s_min / kMinPartPoints));
}

// Launch geometry for a batch of n_wg samples (at most kmax centroids, the
// smallest s_min points).  copies_req 0 = as many private copies as fit in
// 64 KiB; wg_per_cu 0 = as many workgroups per CU as the occupancy allows.
// parts_req 0: with max_parts > 1 and at least twice as many resident
// workgroups (of the shared form) as samples, every sample gets P =
// min(resident / samples, max_parts, parts_limit) workgroups (warm samples
// are then shared).  parts_req > 0 asks for P = min(parts_req, max_parts,
// parts_limit, resident) whatever the number of samples: samples beyond
// the resident grid then wait in the queue, and the grid is a whole number
// of samples' parts.
template <int D, int PREC>
int resident_geometry(int kmax, int n_wg, int s_min, int wg_per_cu, int copies_req,
                      int max_parts, int parts_req, ResGeo* out) {
    using S = hpc::Smem<D, kNT, PREC>;
    constexpr int NW = kNT / hpc::kWave;
    int lds_max = 0;
    int rc = max_dyn_lds(&lds_max);
    if (rc) return rc;
    int copies = NW;
    if (copies_req > 0) {
        copies = std::min(copies_req, NW);
    } else {
        const size_t soft = 64 * 1024;
        while (copies > 1 && S::bytes(kmax, copies) > soft) --copies;
    }
    const size_t lds = S::bytes(kmax, copies);
    if (lds > (size_t)lds_max)
        return fail(HPC_ERR_UNSUPPORTED,
                    "k=%d with padded d=%d and %d partial copies needs %zu bytes of LDS per "
                    "workgroup (limit %d)",
                    kmax, D, copies, lds, lds_max);
    int cus = 0;
    rc = device_cus(&cus);
    if (rc) return rc;
    // resident workgroups of one form
    auto capacity = [&](auto kern, int* per_cu_out, int64_t* cap) -> int {
        if (lds > 64 * 1024)
            HPC_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        int per_cu = 0;
        HPC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kNT, lds));
        per_cu = std::max(1, per_cu);
        *per_cu_out = per_cu;
        *cap = (int64_t)cus * (wg_per_cu > 0 ? std::min(per_cu, wg_per_cu) : per_cu);
        return HPC_OK;
    };
    int per_s = 0;
    int64_t cap_s = 0;
    rc = capacity(hpc::k_lloyd_resident<D, kNT, PREC, true>, &per_s, &cap_s);
    if (rc) return rc;
    int parts = 1;
    if (max_parts > 1) {
        const int64_t lim = std::min(max_parts, parts_limit(s_min));
        parts = (int)std::max<int64_t>(
            1, parts_req > 0 ? std::min<int64_t>({(int64_t)parts_req, lim, cap_s})
                             : std::min<int64_t>(cap_s / n_wg, lim));
    }
    int per_cu = per_s;
    int64_t cap = cap_s;
    const bool share = share_form<D>(parts > 1);
    if (!share) {
        rc = capacity(hpc::k_lloyd_resident<D, kNT, PREC, share_form<D>(false)>, &per_cu, &cap);
        if (rc) return rc;
    }
    out->split = parts;
    out->share = share;
    out->grid = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)n_wg * parts, cap / parts * parts));
    out->copies = copies;
    out->lds = lds;
    out->per_cu_max = per_cu;
    return HPC_OK;
}

// Enqueue the queue reset and the resident kernel (kernel launches only).
template <int D, int PREC>
int launch_resident(hpc::LloydArgs a, const ResGeo& g, hipStream_t st) {
    a.n_copies = g.copies;
    a.split = g.split;
    a.xstride = a.kmax * (D + 1) + 8;
    if (g.split > 1 && (!a.xbuf || !a.xflag))
        return fail(HPC_ERR_INVALID_ARG, "shared samples without an exchange buffer");
    hipLaunchKernelGGL(hpc::k_fill_i32, dim3(1), dim3(64), 0, st, a.queue, (int64_t)1, 0);
    if (g.split > 1)
        hipLaunchKernelGGL(hpc::k_fill_i32, dim3((4 * a.n_samples + 255) / 256), dim3(256), 0, st,
                           a.xflag, (int64_t)4 * a.n_samples, 0);
    if (g.share)
        hipLaunchKernelGGL((hpc::k_lloyd_resident<D, kNT, PREC, true>), dim3(g.grid), dim3(kNT),
                           g.lds, st, a);
    else
        hipLaunchKernelGGL((hpc::k_lloyd_resident<D, kNT, PREC, share_form<D>(false)>),
                           dim3(g.grid), dim3(kNT), g.lds, st, a);
    HPC_HIP(hipGetLastError());
    return HPC_OK;
}

int resident_geo(int D, int prec, int kmax, int n_wg, int s_min, int max_parts, ResGeo* g) {
    return with_dp(D, prec, [&](auto Dc, auto Pc) {
        return resident_geometry<decltype(Dc)::value, decltype(Pc)::value>(kmax, n_wg, s_min, 0, 0,
                                                                           max_parts, 0, g);
    });
}

int dispatch_resident(int D, int prec, const hpc::LloydArgs& a, const ResGeo& g, hipStream_t st) {
    return with_dp(D, prec, [&](auto Dc, auto Pc) {
        return launch_resident<decltype(Dc)::value, decltype(Pc)::value>(a, g, st);
    });
}

// --------------------------------------------------------------------------
// K-means++ seeding of cold samples by teams of workgroups.
// --------------------------------------------------------------------------
constexpr int kKppNT = 256;        // threads per workgroup of the seeding kernel
constexpr int kKppMinSlice = 256;  // points per workgroup of a team at least (one group)
constexpr int kKppMaxTeam = hpc::kMaxTeam;
constexpr int kKppMaxWgPerCu = 8;  // bound on resident seeding workgroups per CU (buffers)

struct KppGeo {
    int team = 1;     // workgroups per sample
    int n_teams = 0;  // 0: no launch (the Lloyd kernel seeds every sample itself)
    int grid = 0;
    int ngmax = 0;
    size_t lds = 0;
};

// Launch shape of the seeding kernel for n samples (largest s smax, largest
// k kmax).  team_req 0 picks the team size from the free capacity: as many
// workgroups per sample as the resident grid allows for all samples at once,
// at most one per kKppMinSlice points (rounded up) and kKppMaxTeam.  inflight_req caps the teams working
// at once (0: as many as are resident; fewer keep the samples' rows and
// weights within the last-level cache).  The grid is always resident at
// once, which the teams' exchanges rely on (they wait on each other); a team
// takes its samples in turn from the processing order.
template <int D>
int kpp_geometry(int n, int smax, int kmax, int team_req, int inflight_req, KppGeo* g) {
    *g = KppGeo{};
    int lds_max = 0, cus = 0;
    int rc = max_dyn_lds(&lds_max);
    if (rc) return rc;
    rc = device_cus(&cus);
    if (rc) return rc;
    auto kern = hpc::k_kmeanspp_team<D, kKppNT>;
    auto shape = [&](int T, int* ngmax, size_t* lds, int64_t* cap) -> int {
        const int64_t per = ((smax + (int64_t)T - 1) / T + hpc::kKppGroup - 1) / hpc::kKppGroup;
        *ngmax = (int)std::max<int64_t>(1, per);
        *lds = hpc::kpp_lds_bytes<D, kKppNT>(*ngmax, kmax, T);
        *cap = 0;
        if (*lds > (size_t)lds_max) return HPC_OK;
        if (*lds > 64 * 1024)
            HPC_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)*lds));
        int per_cu = 0;
        HPC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kKppNT, *lds));
        *cap = (int64_t)cus * std::min(std::max(per_cu, 0), kKppMaxWgPerCu);
        return HPC_OK;
    };
    int ngmax = 0;
    size_t lds = 0;
    int64_t cap = 0;
    rc = shape(1, &ngmax, &lds, &cap);
    if (rc) return rc;
    int T = 1;
    if (team_req > 0) {
        T = std::min(team_req, kKppMaxTeam);
    } else if (cap > 0) {
        const int64_t by_cap = cap / n;
        const int64_t by_size = std::max<int64_t>(1, (smax + kKppMinSlice - 1) / kKppMinSlice);
        T = (int)std::max<int64_t>(1, std::min<int64_t>({by_cap, by_size, (int64_t)kKppMaxTeam}));
    }
    if (T > 1) {
        rc = shape(T, &ngmax, &lds, &cap);
        if (rc) return rc;
        if (cap < T) {  // not even one team resident
            T = 1;
            rc = shape(1, &ngmax, &lds, &cap);
            if (rc) return rc;
        }
    }
    if (cap == 0) return HPC_OK;  // the slices do not fit in LDS: seeded in the Lloyd kernel
    int64_t teams = cap / T;
    if (inflight_req > 0) teams = std::min<int64_t>(teams, inflight_req);
    g->team = T;
    g->n_teams = (int)std::min<int64_t>(n, teams);
    g->grid = g->n_teams * T;
    g->ngmax = ngmax;
    g->lds = lds;
    return HPC_OK;
}

int kpp_geo(int D, int n, int smax, int kmax, int team_req, int inflight_req, KppGeo* g) {
    switch (D) {
        case 8: return kpp_geometry<8>(n, smax, kmax, team_req, inflight_req, g);
        case 16: return kpp_geometry<16>(n, smax, kmax, team_req, inflight_req, g);
        case 32: return kpp_geometry<32>(n, smax, kmax, team_req, inflight_req, g);
        case 64: return kpp_geometry<64>(n, smax, kmax, team_req, inflight_req, g);
        case 128: return kpp_geometry<128>(n, smax, kmax, team_req, inflight_req, g);
    }
    return fail(HPC_ERR_UNSUPPORTED, "seeding: padded dimension %d", D);
}

// Bytes of the seeding kernel's team flags (four ints per team, at most one
// team per workgroup) and exchange slots (two parities per workgroup).
size_t kpp_flag_bytes(int64_t grid) { return (size_t)grid * 16; }
size_t kpp_slot_bytes(const KppGeo& g) {
    return g.team > 1 ? (size_t)g.grid * 2 * hpc::kpp_slot_doubles(g.ngmax) * 8 : 0;
}

// Enqueue the flag resets and the seeding kernel (kernel launches only).
int launch_kpp(int D, hpc::KppArgs a, const KppGeo& g, hipStream_t st) {
    if (g.grid == 0) return HPC_OK;
    a.team = g.team;
    a.n_teams = g.n_teams;
    a.ngmax = g.ngmax;
    hipLaunchKernelGGL(hpc::k_fill_i32, dim3(1), dim3(64), 0, st, a.queue, (int64_t)1, 0);
    hipLaunchKernelGGL(hpc::k_fill_i32, dim3((4 * g.n_teams + 255) / 256), dim3(256), 0, st,
                       a.tflag, (int64_t)4 * g.n_teams, 0);
#define HPC_KPP(DD)                                                                           \
    case DD:                                                                                  \
        hipLaunchKernelGGL((hpc::k_kmeanspp_team<DD, kKppNT>), dim3(g.grid), dim3(kKppNT), g.lds, \
                           st, a);                                                            \
        break
    switch (D) {
        HPC_KPP(8);
        HPC_KPP(16);
        HPC_KPP(32);
        HPC_KPP(64);
        HPC_KPP(128);
        default: return fail(HPC_ERR_UNSUPPORTED, "seeding: padded dimension %d", D);
    }
#undef HPC_KPP
    HPC_HIP(hipGetLastError());
    return HPC_OK;
}

// Resident waves per CU of k_assign_sse<D, NT, PREC> with `lds` bytes of
// LDS per workgroup (0 if it does not fit); sets the attribute allowing
// more than 64 KiB.
template <int D, int NT, int PREC>
int assign_waves_per_cu(size_t lds, int lds_max, int* waves) {
    *waves = 0;
    if (lds > (size_t)lds_max) return HPC_OK;
    auto kern = hpc::k_assign_sse<D, NT, PREC>;
    if (lds > 64 * 1024)
        HPC_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int per_cu = 0;
    HPC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, NT, lds));
    *waves = per_cu * (NT / hpc::kWave);
    return HPC_OK;
}

// Where the assignment's per-workgroup partial sums go: the calling
// stream's workspace (grown as needed), or a fixed device buffer of `cap`
// doubles (the no-allocation entry point), which then bounds the grid.
struct PartialsDst {
    Workspace* ws = nullptr;
    double* fixed = nullptr;
    int64_t cap = 0;
};

template <int D, int NT, int PREC>
int launch_assign_nt(const float* X, int64_t m, int d, const float* C, int k, int32_t* labels,
                     int64_t* counts, double* sse, const PartialsDst& pd, hipStream_t st,
                     int waves_cu) {
    constexpr int NW = NT / hpc::kWave;
    const size_t lds = hpc::assign_lds_bytes<D, PREC>(k, NT);
    int cus = 0;
    int rc = device_cus(&cus);
    if (rc) return rc;
    // four workgroup slots per resident workgroup (grid-stride over tiles of
    // 16 rows per wave), at most one workgroup per NW tiles
    const int64_t want = (m + 16 * NW - 1) / (16 * NW);
    const int64_t slots = (int64_t)cus * std::max(1, waves_cu / NW) * 4;
    int64_t g64 = std::max<int64_t>(1, std::min<int64_t>(want, slots));
    double* partials = nullptr;
    if (pd.ws) {
        rc = ws_reserve_dev(pd.ws, Carve::need({(size_t)g64 * 8}));
        if (rc) return rc;
        Carve cv(pd.ws->dev);
        partials = static_cast<double*>(cv.take((size_t)g64 * 8));
    } else {
        g64 = std::min<int64_t>(g64, pd.cap);
        partials = pd.fixed;
    }
    const int grid = (int)g64;
    if (counts)
        hipLaunchKernelGGL(hpc::k_fill_u64, dim3((k + 255) / 256), dim3(256), 0, st,
                           reinterpret_cast<unsigned long long*>(counts), (int64_t)k, 0ull);
    const bool vec = (d == D) && (reinterpret_cast<uintptr_t>(X) % 16 == 0);
    hipLaunchKernelGGL((hpc::k_assign_sse<D, NT, PREC>), dim3(grid), dim3(NT), lds, st, X, m, d,
                       C, k, labels, reinterpret_cast<unsigned long long*>(counts), partials, vec);
    hipLaunchKernelGGL(hpc::k_reduce_partials<256>, dim3(1), dim3(256), 0, st, partials, grid,
                       sse);
    HPC_HIP(hipGetLastError());
    return HPC_OK;
}

// The full assignment on 32-point tiles (rows of up to 32 coordinates):
// 256-thread workgroups, four workgroup slots per resident one.
template <int D, int PREC>
int launch_assign32(const float* X, int64_t m, int d, const float* C, int k, int32_t* labels,
                    int64_t* counts, double* sse, const PartialsDst& pd, hipStream_t st,
                    int lds_max) {
    constexpr int NT = 256, NW = NT / hpc::kWave;
    const size_t lds = hpc::assign32_lds_bytes<D, PREC>(k, NT);
    if (lds > (size_t)lds_max)
        return fail(HPC_ERR_UNSUPPORTED, "k=%d, padded d=%d: centroids exceed LDS", k, D);
    auto kern = hpc::k_assign_sse32<D, NT, PREC>;
    if (lds > 64 * 1024)
        HPC_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int per_cu = 0;
    HPC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, NT, lds));
    int cus = 0;
    int rc = device_cus(&cus);
    if (rc) return rc;
    const int64_t want = (m + 32 * NW - 1) / (32 * NW);
    const int64_t slots = (int64_t)cus * std::max(1, per_cu) * 4;
    int64_t g64 = std::max<int64_t>(1, std::min<int64_t>(want, slots));
    double* partials = nullptr;
    if (pd.ws) {
        rc = ws_reserve_dev(pd.ws, Carve::need({(size_t)g64 * 8}));
        if (rc) return rc;
        Carve cv(pd.ws->dev);
        partials = static_cast<double*>(cv.take((size_t)g64 * 8));
    } else {
        g64 = std::min<int64_t>(g64, pd.cap);
        partials = pd.fixed;
    }
    const int grid = (int)g64;
    if (counts)
        hipLaunchKernelGGL(hpc::k_fill_u64, dim3((k + 255) / 256), dim3(256), 0, st,
                           reinterpret_cast<unsigned long long*>(counts), (int64_t)k, 0ull);
    const bool vec = (d == D) && (reinterpret_cast<uintptr_t>(X) % 16 == 0);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(NT), lds, st, X, m, d, C, k, labels,
                       reinterpret_cast<unsigned long long*>(counts), partials, vec);
    hipLaunchKernelGGL(hpc::k_reduce_partials<256>, dim3(1), dim3(256), 0, st, partials, grid,
                       sse);
    HPC_HIP(hipGetLastError());
    return HPC_OK;
}

// Full assignment: up to d = 32 on 32-point tiles; wider rows on 16-point
// tiles with 256-thread workgroups, or (d <= 64) 768- or 1,024-thread ones
// when the centroid tables leave room for more resident waves that way.
template <int D, int PREC>
int launch_assign(const float* X, int64_t m, int d, const float* C, int k, int32_t* labels,
                  int64_t* counts, double* sse, const PartialsDst& w, hipStream_t st) {
    int lds_max = 0;
    int rc = max_dyn_lds(&lds_max);
    if (rc) return rc;
    if constexpr (D <= 32)
        return launch_assign32<D, PREC>(X, m, d, C, k, labels, counts, sse, w, st, lds_max);
    int w256 = 0, w768 = 0, w1024 = 0;
    rc = assign_waves_per_cu<D, 256, PREC>(hpc::assign_lds_bytes<D, PREC>(k, 256), lds_max, &w256);
    if (rc) return rc;
    if constexpr (D <= 64) {
        rc = assign_waves_per_cu<D, 768, PREC>(hpc::assign_lds_bytes<D, PREC>(k, 768), lds_max,
                                               &w768);
        if (rc) return rc;
        rc = assign_waves_per_cu<D, 1024, PREC>(hpc::assign_lds_bytes<D, PREC>(k, 1024), lds_max,
                                                &w1024);
        if (rc) return rc;
        if (w1024 > w256 && w1024 > w768)
            return launch_assign_nt<D, 1024, PREC>(X, m, d, C, k, labels, counts, sse, w, st,
                                                   w1024);
        if (w768 > w256)
            return launch_assign_nt<D, 768, PREC>(X, m, d, C, k, labels, counts, sse, w, st,
                                                  w768);
    }
    if (w256 == 0)
        return fail(HPC_ERR_UNSUPPORTED, "k=%d, padded d=%d: centroids exceed LDS", k, D);
    return launch_assign_nt<D, 256, PREC>(X, m, d, C, k, labels, counts, sse, w, st, w256);
}

bool sizes_ok(int32_t d, int32_t k) { return d >= 1 && d <= kMaxD && k >= 1 && k <= 512; }

// Validate a batch descriptor table against the array lengths; also checks
// that no two samples share idx or centroid storage.
int check_desc(const hpc_sample_desc* desc, int32_t n, int64_t idx_len, int64_t c_len, int32_t d,
               int* kmax) {
    *kmax = 0;
    std::vector<std::pair<int64_t, int64_t>> ir, cr;
    ir.reserve(n);
    cr.reserve(n);
    for (int32_t b = 0; b < n; ++b) {
        const hpc_sample_desc& s = desc[b];
        if (s.k < 1 || s.k > 512)
            return fail(HPC_ERR_INVALID_ARG, "sample %d: k=%d outside [1, 512]", b, s.k);
        if (s.s < s.k) return fail(HPC_ERR_INVALID_ARG, "sample %d: s=%d < k=%d", b, s.s, s.k);
        if (s.idx_offset < 0 || s.idx_offset + s.s > idx_len)
            return fail(HPC_ERR_INVALID_ARG, "sample %d: idx range [%lld, %lld) outside idx_len %lld",
                        b, (long long)s.idx_offset, (long long)(s.idx_offset + s.s),
                        (long long)idx_len);
        if (c_len >= 0 && (s.c_offset < 0 || s.c_offset + (int64_t)s.k * d > c_len))
            return fail(HPC_ERR_INVALID_ARG, "sample %d: centroid block outside c_len %lld", b,
                        (long long)c_len);
        ir.emplace_back(s.idx_offset, s.idx_offset + s.s);
        cr.emplace_back(s.c_offset, s.c_offset + (int64_t)s.k * d);
        *kmax = std::max(*kmax, s.k);
    }
    auto overlap = [](std::vector<std::pair<int64_t, int64_t>>& v) {
        std::sort(v.begin(), v.end());
        for (size_t i = 1; i < v.size(); ++i)
            if (v[i].first < v[i - 1].second) return true;
        return false;
    };
    if (overlap(ir)) return fail(HPC_ERR_INVALID_ARG, "samples share idx entries");
    if (c_len >= 0 && overlap(cr)) return fail(HPC_ERR_INVALID_ARG, "samples share centroid blocks");
    return HPC_OK;
}

// Longest-first processing order (work ~ s * k), ties by descriptor order.
std::vector<int32_t> longest_first(const hpc_sample_desc* desc, int32_t n) {
    std::vector<int32_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return (int64_t)desc[a].s * desc[a].k > (int64_t)desc[b].s * desc[b].k;
    });
    return order;
}

// Arguments of the seeding kernel for the batch of a resident launch.
hpc::KppArgs kpp_args(const hpc::LloydArgs& a, uint32_t tag, uint32_t call_id, int n_cand,
                      int32_t* queue, int32_t* tflag, double* tx) {
    hpc::KppArgs k{};
    k.X = a.X;
    k.m = a.m;
    k.d = a.d;
    k.idx = a.idx;
    k.desc = a.desc;
    k.order = a.order;
    k.n_samples = a.n_samples;
    k.C = a.C;
    k.n_cand = n_cand;
    k.tag = tag;
    k.call_id = call_id;
    k.chosen = a.chosen;
    k.vec4 = a.vec4;
    k.sbuf = a.sbuf;
    k.d2buf = a.d2buf;
    k.kmax = a.kmax;
    k.queue = queue;
    k.tflag = tflag;
    k.tx = tx;
    return k;
}

// Run the resident kernel over a batch (Lloyd, or seeding only).
int run_resident(const float* X, int64_t m, int32_t d, const int64_t* idx, int64_t idx_len,
                 const hpc_sample_desc* desc, int32_t n, float* C, int32_t max_iter,
                 double rel_tol, int32_t precision, double* f_out, int32_t* iters_out,
                 int32_t* labels_out, int seed_only, int n_cand, uint32_t call_id,
                 int32_t* chosen, int kmax, hipStream_t st) {
    Workspace* w = nullptr;
    int rc = get_ws(st, &w);
    if (rc) return rc;
    const int D = pad_dim(d);
    ResGeo g;
    int s_min = INT32_MAX;
    for (int32_t b = 0; b < n; ++b) s_min = std::min(s_min, desc[b].s);
    rc = resident_geo(D, precision, kmax, n, s_min, seed_only ? 1 : hpc::kMaxParts, &g);
    if (rc) return rc;
    const std::vector<int32_t> order = longest_first(desc, n);
    const size_t desc_b = (size_t)n * sizeof(hpc_sample_desc);
    const size_t order_b = (size_t)n * 4;
    const size_t sbuf_b = (size_t)idx_len * D * 4;
    const size_t xbuf_b = g.split > 1 ? xbuf_doubles(n, g.split, kmax, D) * 8 : 0;
    const size_t xflag_b = g.split > 1 ? (size_t)n * 16 : 0;
    int smax = 0;
    for (int32_t b = 0; b < n; ++b) smax = std::max(smax, desc[b].s);
    KppGeo kg;
    rc = kpp_geo(D, n, smax, kmax, 0, 0, &kg);
    if (rc) return rc;
    const size_t kflag_b = kpp_flag_bytes(kg.grid), kslot_b = kpp_slot_bytes(kg);
    const size_t need = Carve::need({desc_b + order_b, 256, sbuf_b, (size_t)idx_len * 40,
                                     (size_t)idx_len * 4, xbuf_b, xflag_b, kflag_b, kslot_b,
                                     (size_t)kmax * 4});
    rc = ws_reserve_dev(w, need);
    if (rc) return rc;
    Carve cv(w->dev);
    char* tbl = static_cast<char*>(cv.take(desc_b + order_b));
    int32_t* queue = static_cast<int32_t*>(cv.take(256));
    float* sbuf = static_cast<float*>(cv.take(sbuf_b));
    double* d2 = static_cast<double*>(cv.take((size_t)idx_len * 40));
    int32_t* lbuf = static_cast<int32_t*>(cv.take((size_t)idx_len * 4));
    double* xbuf = static_cast<double*>(cv.take(xbuf_b));
    int32_t* xflag = static_cast<int32_t*>(cv.take(xflag_b));
    int32_t* kflag = static_cast<int32_t*>(cv.take(kflag_b));
    double* kslot = static_cast<double*>(cv.take(kslot_b));
    int32_t* chosen_tmp = static_cast<int32_t*>(cv.take((size_t)kmax * 4));
    std::vector<char> host(desc_b + order_b);
    memcpy(host.data(), desc, desc_b);
    memcpy(host.data() + desc_b, order.data(), order_b);
    rc = ws_upload(w, tbl, host.data(), host.size());
    if (rc) return rc;
    hpc::LloydArgs a{};
    a.X = X;
    a.m = m;
    a.d = d;
    a.idx = idx;
    a.desc = reinterpret_cast<const hpc_sample_desc*>(tbl);
    a.order = reinterpret_cast<const int32_t*>(tbl + desc_b);
    a.n_samples = n;
    a.C = C;
    a.max_iter = max_iter;
    a.rel_tol = rel_tol;
    a.f_out = f_out;
    a.iters_out = iters_out;
    a.labels_out = labels_out;
    a.sbuf = sbuf;
    a.d2buf = d2;
    a.lbuf = lbuf;
    a.queue = queue;
    a.kmax = kmax;
    a.seed_only = seed_only;
    a.n_cand = n_cand;
    a.call_id = call_id;
    a.chosen = chosen;
    a.vec4 = (d % 4 == 0) && (reinterpret_cast<uintptr_t>(X) % 16 == 0);
    a.xbuf = g.split > 1 ? xbuf : nullptr;
    a.xflag = g.split > 1 ? xflag : nullptr;
    // cold samples are seeded first by the team kernel (stream tag SEED and
    // the caller's call_id for the seeding call; RESEED and 0, the stream of
    // a Lloyd cold start, otherwise); the resident kernel then seeds only
    // what is left: partially valid blocks, or samples of a team that gave up
    // (the seeding call: the team kernel writes the caller's chosen for a
    // cold start; the resident kernel, which resets chosen to -1 for every
    // block it visits, writes a scratch copy that is merged afterwards)
    if (seed_only && chosen)
        hipLaunchKernelGGL(hpc::k_fill_i32, dim3(1), dim3(256), 0, st, chosen, (int64_t)kmax, -1);
    const hpc::KppArgs ka = kpp_args(a, seed_only ? hpc::kTagSeed : hpc::kTagReseed,
                                     seed_only ? call_id : 0u, n_cand, queue + 16, kflag, kslot);
    rc = launch_kpp(D, ka, kg, st);
    if (rc) return rc;
    if (seed_only && chosen) a.chosen = chosen_tmp;
    rc = dispatch_resident(D, precision, a, g, st);
    if (rc) return rc;
    if (seed_only && chosen) {
        hipLaunchKernelGGL(hpc::k_merge_chosen, dim3(1), dim3(256), 0, st, chosen,
                           (const int32_t*)chosen_tmp, (int32_t)kmax);
        HPC_HIP(hipGetLastError());
    }
    return HPC_OK;
}

int next_pow2(int64_t v) {
    int e = 0;
    while (((int64_t)1 << e) < v) ++e;
    return e;
}

}  // namespace

// A prepared batch (include/hpclust.h, "Batch plans").  All device buffers
// live in one allocation.
struct hpc_plan_s {
    int device = 0;
    int32_t d = 0, D = 0, prec = 0, n = 0, kmax = 0;
    int64_t idx_len = 0, c_len = 0;
    std::vector<hpc_sample_desc> desc;
    char* mem = nullptr;
    void* kmem = nullptr;  // the seeding teams' flags and exchange slots
    hpc_sample_desc* desc_dev = nullptr;   // live table (sample ids advance)
    hpc_sample_desc* desc_init = nullptr;  // table as created
    int32_t* order_dev = nullptr;          // [0, n): longest first; [n, 2n): given order
    int32_t* queue = nullptr;
    float* sbuf = nullptr;
    double* d2 = nullptr;
    int32_t* lbuf = nullptr;
    double* xbuf = nullptr;    // pair exchange (only when samples can be shared)
    int32_t* xflag = nullptr;
    float* tC = nullptr;  // autotuner scratch
    double* tf = nullptr;
    int32_t* tit = nullptr;
    int32_t* kflag = nullptr;  // seeding teams' flags and exchange slots
    double* kslot = nullptr;
    int64_t kgrid_max = 0;     // workgroups those buffers serve
    int smax = 0, smin = 0;
    int xparts = 1;            // workgroups per shared sample the exchange buffer serves
    hpc_tune tune{};
    ResGeo geo;
    KppGeo kgeo;
    hipStream_t cap = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

int plan_check(hpc_plan p, const char* where) {
    if (!p) return fail(HPC_ERR_INVALID_ARG, "%s: NULL plan", where);
    int dev = 0;
    HPC_HIP(hipGetDevice(&dev));
    if (dev != p->device)
        return fail(HPC_ERR_INVALID_ARG, "%s: plan was created on device %d, current is %d", where,
                    p->device, dev);
    return HPC_OK;
}

int plan_geometry(hpc_plan p, const hpc_tune& t, ResGeo* g, int max_parts) {
    return with_dp(p->D, p->prec, [&](auto Dc, auto Pc) {
        return resident_geometry<decltype(Dc)::value, decltype(Pc)::value>(
            p->kmax, p->n, p->smin, t.wg_per_cu, t.copies, max_parts, t.parts, g);
    });
}

// Geometry within the plan's exchange buffer (its parts per sample).
int plan_geometry(hpc_plan p, const hpc_tune& t, ResGeo* g) {
    return plan_geometry(p, t, g, p->xparts);
}

hpc::LloydArgs plan_args(hpc_plan p, const float* X, int64_t m, const int64_t* idx, float* C,
                         int32_t max_iter, double rel_tol, double* f_out, int32_t* iters_out,
                         int32_t* labels_out, int order) {
    hpc::LloydArgs a{};
    a.X = X;
    a.m = m;
    a.d = p->d;
    a.idx = idx;
    a.desc = p->desc_dev;
    a.order = p->order_dev + (order ? p->n : 0);
    a.n_samples = p->n;
    a.C = C;
    a.max_iter = max_iter;
    a.rel_tol = rel_tol;
    a.f_out = f_out;
    a.iters_out = iters_out;
    a.labels_out = labels_out;
    a.sbuf = p->sbuf;
    a.d2buf = p->d2;
    a.lbuf = p->lbuf;
    a.queue = p->queue;
    a.kmax = p->kmax;
    a.n_cand = 3;
    a.vec4 = (p->d % 4 == 0) && (reinterpret_cast<uintptr_t>(X) % 16 == 0);
    a.xbuf = p->xbuf;
    a.xflag = p->xflag;
    return a;
}

// Seeding of the cold samples (team kernel), then the resident Lloyd kernel.
int plan_launch(hpc_plan p, const hpc::LloydArgs& a, const ResGeo& g, hipStream_t st) {
    const hpc::KppArgs ka =
        kpp_args(a, hpc::kTagReseed, 0u, 3, p->queue + 16, p->kflag, p->kslot);
    int rc = launch_kpp(p->D, ka, p->kgeo, st);
    if (rc) return rc;
    return with_dp(p->D, p->prec, [&](auto Dc, auto Pc) {
        return launch_resident<decltype(Dc)::value, decltype(Pc)::value>(a, g, st);
    });
}

// The seeding kernel's launch shape for a plan and a team request (the
// buffers allocated with the plan bound the grid).
int plan_kpp_geometry(hpc_plan p, int team_req, int inflight_req, KppGeo* g) {
    int rc = kpp_geo(p->D, p->n, p->smax, p->kmax, team_req, inflight_req, g);
    if (rc) return rc;
    if (g->grid > p->kgrid_max)
        return fail(HPC_ERR_UNSUPPORTED, "seeding grid of %d workgroups exceeds the plan's %lld",
                    g->grid, (long long)p->kgrid_max);
    return HPC_OK;
}

int lloyd_opts_ok(const char* where, const float* X, int64_t m, const void* idx, const void* C,
                  int32_t max_iter, double rel_tol, const void* f_out, const void* iters_out) {
    if (!X || !idx || !C || !f_out || !iters_out)
        return fail(HPC_ERR_INVALID_ARG, "%s: NULL pointer", where);
    if (m < 1) return fail(HPC_ERR_INVALID_ARG, "%s: m < 1", where);
    if (max_iter < 1 || !(rel_tol >= 0.0) || std::isinf(rel_tol))
        return fail(HPC_ERR_INVALID_ARG, "%s: need max_iter>=1 and finite rel_tol>=0", where);
    return HPC_OK;
}

void plan_draw(hpc_plan p, int64_t m, int64_t* idx, hipStream_t st) {
    int64_t max_s = 0;
    for (const auto& ds : p->desc) max_s = std::max<int64_t>(max_s, ds.s);
    const int64_t nq = (max_s + 3) / 4;
    const unsigned gx = (unsigned)std::min<int64_t>((nq + 255) / 256, 1024);
    hipLaunchKernelGGL(hpc::k_draw_batch, dim3(gx, p->n), dim3(256), 0, st, m,
                       (const hpc_sample_desc*)p->desc_dev, idx);
}

void plan_advance(hpc_plan p, uint64_t id_stride, hipStream_t st) {
    hipLaunchKernelGGL(hpc::k_advance_ids, dim3((p->n + 255) / 256), dim3(256), 0, st, p->desc_dev,
                       p->n, id_stride);
}

// Enqueue one worker-loop round (kernel launches only).
int plan_enqueue_round(hpc_plan p, const float* X, int64_t m, int64_t* idx, float* C,
                       float* C_inc, double* f_inc, int32_t max_iter, double rel_tol,
                       double* f_out, int32_t* iters_out, uint64_t id_stride, hipStream_t st) {
    plan_draw(p, m, idx, st);
    const unsigned cx = (unsigned)std::min<int64_t>(((int64_t)p->kmax * p->d + 255) / 256, 64);
    hipLaunchKernelGGL(hpc::k_copy_blocks, dim3(cx, p->n), dim3(256), 0, st,
                       (const hpc_sample_desc*)p->desc_dev, p->d, (const float*)C_inc, C);
    const hpc::LloydArgs a =
        plan_args(p, X, m, idx, C, max_iter, rel_tol, f_out, iters_out, nullptr, p->tune.order);
    int rc = plan_launch(p, a, p->geo, st);
    if (rc) return rc;
    hipLaunchKernelGGL(hpc::k_keep_best_desc, dim3(p->n), dim3(256), 0, st,
                       (const hpc_sample_desc*)p->desc_dev, p->d, (const float*)C,
                       (const double*)f_out, C_inc, f_inc);
    if (id_stride) plan_advance(p, id_stride, st);
    HPC_HIP(hipGetLastError());
    return HPC_OK;
}

// The no-allocation form of the full assignment keeps its per-workgroup
// partial sums in this fixed array: each GPU the library runs on holds one
// copy until the process ends.  Host code never passes the array's name to
// a kernel (in host code it is a stand-in, not a device address); it uses
// the device address looked up once per device below.
constexpr int kStaticPartials = 8192;
static __device__ __align__(256) double scratch[kStaticPartials];

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
double* g_static_partials[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up with that
// device current on its first use, then cached).
int static_partials(double** out) {
    int dev = 0;
    HPC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(HPC_ERR_UNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_partials[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(HPC_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d failed: %s", dev,
                        hipGetErrorString(e));
        g_static_partials[dev] = static_cast<double*>(ptr);
    }
    *out = g_static_partials[dev];
    return HPC_OK;
}

int assign_args_ok(const char* where, const float* X, int64_t m, int32_t d, const float* C,
                   int32_t k, int32_t precision, const double* sse) {
    if (!X || !C || !sse) return fail(HPC_ERR_INVALID_ARG, "%s: NULL pointer", where);
    if (m < 1 || !sizes_ok(d, k))
        return fail(HPC_ERR_INVALID_ARG, "%s: need m>=1, 1<=d<=%d, 1<=k<=512", where, kMaxD);
    if (!precision_ok(precision))
        return fail(HPC_ERR_INVALID_ARG, "%s: unknown precision %d", where, precision);
    return HPC_OK;
}

int dispatch_assign(const float* X, int64_t m, int32_t d, const float* C, int32_t k,
                    int32_t precision, int32_t* labels, int64_t* counts, double* sse,
                    const PartialsDst& pd, hipStream_t st) {
#define HPC_ASSIGN(DD)                                                                          \
    if (precision == HPC_PREC_BF16_MFMA)                                                        \
        return launch_assign<DD, hpc::kPrecBF16>(X, m, d, C, k, labels, counts, sse, pd, st);   \
    if (precision == HPC_PREC_BF16X3_MFMA)                                                      \
        return launch_assign<DD, hpc::kPrecBF16x3>(X, m, d, C, k, labels, counts, sse, pd, st); \
    return launch_assign<DD, hpc::kPrecF32>(X, m, d, C, k, labels, counts, sse, pd, st)
    switch (pad_dim(d)) {
        case 8: HPC_ASSIGN(8);
        case 16: HPC_ASSIGN(16);
        case 32: HPC_ASSIGN(32);
        case 64: HPC_ASSIGN(64);
        case 128: HPC_ASSIGN(128);
    }
#undef HPC_ASSIGN
    return fail(HPC_ERR_UNSUPPORTED, "assignment: d=%d", d);
}

}  // namespace


extern "C" {

const char* hpc_version(void) { return "hpclust-gfx950 0.1.0"; }

const char* hpc_last_error(void) { return g_last_error.c_str(); }

int hpc_device_count(void) {
    int n = 0;
    HPC_HIP(hipGetDeviceCount(&n));
    return n;
}

int hpc_release(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    int prev = 0;
    HPC_HIP(hipGetDevice(&prev));
    for (auto& kv : g_ws) {
        Workspace* w = kv.second;
        HPC_HIP(hipSetDevice(w->device));
        HPC_HIP(hipStreamSynchronize(w->stream));
        if (w->dev) HPC_HIP(hipFree(w->dev));
        for (auto& sl : w->stage) {
            if (sl.host) HPC_HIP(hipHostFree(sl.host));
            if (sl.copied) HPC_HIP(hipEventDestroy(sl.copied));
        }
        delete w;
    }
    g_ws.clear();
    HPC_HIP(hipSetDevice(prev));
    return HPC_OK;
}

int hpc_draw_sample(int64_t m, int32_t s, uint64_t seed, uint64_t sample_id, int64_t* idx,
                    void* hip_stream) {
    if (m < 1 || s < 1 || !idx)
        return fail(HPC_ERR_INVALID_ARG, "hpc_draw_sample: need m >= 1, s >= 1, idx != NULL");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const int64_t nq = ((int64_t)s + 3) / 4;
    const int bs = 256;
    hipLaunchKernelGGL(hpc::k_draw_one, dim3((unsigned)((nq + bs - 1) / bs)), dim3(bs), 0, st, m,
                       s, seed, sample_id, idx);
    HPC_HIP(hipGetLastError());
    return HPC_OK;
}

int hpc_draw_samples(int64_t m, const hpc_sample_desc* desc, int32_t n_samples, int64_t* idx,
                     int64_t idx_len, void* hip_stream) {
    if (m < 1 || !desc || n_samples < 1 || n_samples > 65535 || !idx)
        return fail(HPC_ERR_INVALID_ARG,
                    "hpc_draw_samples: need m>=1, 1<=n_samples<=65535, idx != NULL");
    int64_t max_s = 0;
    for (int32_t b = 0; b < n_samples; ++b) {
        if (desc[b].s < 1 || desc[b].idx_offset < 0 || desc[b].idx_offset + desc[b].s > idx_len)
            return fail(HPC_ERR_INVALID_ARG, "hpc_draw_samples: sample %d outside idx", b);
        max_s = std::max<int64_t>(max_s, desc[b].s);
    }
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    Workspace* w = nullptr;
    int rc = get_ws(st, &w);
    if (rc) return rc;
    const size_t bytes = (size_t)n_samples * sizeof(hpc_sample_desc);
    rc = ws_reserve_dev(w, Carve::need({bytes}));
    if (rc) return rc;
    rc = ws_upload(w, w->dev, desc, bytes);
    if (rc) return rc;
    const int bs = 256;
    const int64_t nq = (max_s + 3) / 4;
    const unsigned gx = (unsigned)std::min<int64_t>((nq + bs - 1) / bs, 1024);
    hipLaunchKernelGGL(hpc::k_draw_batch, dim3(gx, n_samples), dim3(bs), 0, st, m,
                       static_cast<const hpc_sample_desc*>(w->dev), idx);
    HPC_HIP(hipGetLastError());
    return HPC_OK;
}

int hpc_seed_kmeanspp(const float* X, int64_t m, int32_t d, const int64_t* idx, int32_t s,
                      int32_t k, int32_t n_candidates, uint64_t seed, uint64_t sample_id,
                      uint32_t call_id, float* C, int32_t* chosen, void* hip_stream) {
    if (!X || !idx || !C) return fail(HPC_ERR_INVALID_ARG, "hpc_seed_kmeanspp: NULL pointer");
    if (m < 1 || !sizes_ok(d, k) || s < k)
        return fail(HPC_ERR_INVALID_ARG, "hpc_seed_kmeanspp: need m>=1, 1<=d<=%d, 1<=k<=512, s>=k",
                    kMaxD);
    if (n_candidates < 1 || n_candidates > 4)
        return fail(HPC_ERR_INVALID_ARG, "hpc_seed_kmeanspp: n_candidates must be in [1, 4]");
    hpc_sample_desc ds{};
    ds.idx_offset = 0;
    ds.c_offset = 0;
    ds.s = s;
    ds.k = k;
    ds.seed = seed;
    ds.sample_id = sample_id;
    return run_resident(X, m, d, idx, s, &ds, 1, C, 1, 0.0, HPC_PREC_FP32, nullptr, nullptr,
                        nullptr, 1, n_candidates, call_id, chosen, k,
                        static_cast<hipStream_t>(hip_stream));
}

int hpc_lloyd_batch(const float* X, int64_t m, int32_t d, const int64_t* idx, int64_t idx_len,
                    const hpc_sample_desc* desc, int32_t n_samples, float* C, int64_t c_len,
                    int32_t max_iter, double rel_tol, int32_t precision, double* f_out,
                    int32_t* iters_out, int32_t* labels_out, void* hip_stream) {
    if (!X || !idx || !desc || !C || !f_out || !iters_out)
        return fail(HPC_ERR_INVALID_ARG, "hpc_lloyd_batch: NULL pointer");
    if (m < 1 || d < 1 || d > kMaxD || n_samples < 1 || idx_len < 1 || c_len < 1)
        return fail(HPC_ERR_INVALID_ARG, "hpc_lloyd_batch: need m>=1, 1<=d<=%d, n_samples>=1",
                    kMaxD);
    if (max_iter < 1 || !(rel_tol >= 0.0) || std::isinf(rel_tol))
        return fail(HPC_ERR_INVALID_ARG, "hpc_lloyd_batch: need max_iter>=1 and finite rel_tol>=0");
    if (!precision_ok(precision))
        return fail(HPC_ERR_INVALID_ARG, "hpc_lloyd_batch: unknown precision %d", precision);
    int kmax = 0;
    int rc = check_desc(desc, n_samples, idx_len, c_len, d, &kmax);
    if (rc) return rc;
    return run_resident(X, m, d, idx, idx_len, desc, n_samples, C, max_iter, rel_tol, precision,
                        f_out, iters_out, labels_out, 0, 3, 0, nullptr, kmax,
                        static_cast<hipStream_t>(hip_stream));
}

int hpc_keep_best(const float* C_new, const double* f_new, float* C_inc, double* f_inc,
                  int32_t n_workers, int32_t k, int32_t d, int32_t* updated, void* hip_stream) {
    if (!C_new || !f_new || !C_inc || !f_inc || n_workers < 1 || k < 1 || d < 1)
        return fail(HPC_ERR_INVALID_ARG, "hpc_keep_best: bad arguments");
    hipLaunchKernelGGL(hpc::k_keep_best, dim3(n_workers), dim3(256), 0,
                       static_cast<hipStream_t>(hip_stream), C_new, f_new, C_inc, f_inc,
                       (int64_t)k * d, updated);
    HPC_HIP(hipGetLastError());
    return HPC_OK;
}

int hpc_select_best(const float* C_inc, const double* f_inc, int32_t n_workers, int32_t k,
                    int32_t d, float* C_best, double* f_best, int32_t* w_best, void* hip_stream) {
    if (!C_inc || !f_inc || !C_best || !f_best || n_workers < 1 || k < 1 || d < 1)
        return fail(HPC_ERR_INVALID_ARG, "hpc_select_best: bad arguments");
    hipLaunchKernelGGL(hpc::k_select_best<256>, dim3(1), dim3(256), 0,
                       static_cast<hipStream_t>(hip_stream), C_inc, f_inc, n_workers,
                       (int64_t)k * d, C_best, f_best, w_best);
    HPC_HIP(hipGetLastError());
    return HPC_OK;
}

int hpc_screen_bound(int32_t d, int32_t precision, double* alpha, double* beta) {
    if (!alpha || !beta) return fail(HPC_ERR_INVALID_ARG, "hpc_screen_bound: NULL pointer");
    if (d < 1 || d > kMaxD)
        return fail(HPC_ERR_INVALID_ARG, "hpc_screen_bound: need 1<=d<=%d", kMaxD);
    if (!precision_ok(precision))
        return fail(HPC_ERR_INVALID_ARG, "hpc_screen_bound: unknown precision %d", precision);
    if (precision == HPC_PREC_BF16_MFMA)
        hpc::screen_coeffs<hpc::kPrecBF16>(d, alpha, beta);
    else if (precision == HPC_PREC_BF16X3_MFMA)
        hpc::screen_coeffs<hpc::kPrecBF16x3>(d, alpha, beta);
    else
        hpc::screen_coeffs<hpc::kPrecF32>(d, alpha, beta);
    return HPC_OK;
}

int hpc_assign_sse(const float* X, int64_t m, int32_t d, const float* C, int32_t k,
                   int32_t precision, int32_t* labels, int64_t* counts, double* sse,
                   void* hip_stream) {
    int rc = assign_args_ok("hpc_assign_sse", X, m, d, C, k, precision, sse);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    PartialsDst pd;
    rc = get_ws(st, &pd.ws);
    if (rc) return rc;
    return dispatch_assign(X, m, d, C, k, precision, labels, counts, sse, pd, st);
}


int hpc_assign_sse_noalloc(const float* X, int64_t m, int32_t d, const float* C, int32_t k,
                           int32_t precision, int32_t* labels, int64_t* counts, double* sse,
                           void* hip_stream) {
    int rc = assign_args_ok("hpc_assign_sse_noalloc", X, m, d, C, k, precision, sse);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    PartialsDst pd;
    rc = static_partials(&pd.fixed);
    if (rc) return rc;
    pd.cap = kStaticPartials;
    return dispatch_assign(X, m, d, C, k, precision, labels, counts, sse, pd, st);
}


int hpc_plan_create(int32_t d, const hpc_sample_desc* desc, int32_t n_samples, int64_t idx_len,
                    int64_t c_len, int32_t precision, hpc_plan* out) {
    if (!out) return fail(HPC_ERR_INVALID_ARG, "hpc_plan_create: NULL out");
    *out = nullptr;
    if (!desc || d < 1 || d > kMaxD || n_samples < 1 || n_samples > 65535 || idx_len < 1 ||
        c_len < 1)
        return fail(HPC_ERR_INVALID_ARG,
                    "hpc_plan_create: need desc, 1<=d<=%d, 1<=n_samples<=65535, idx_len>=1, "
                    "c_len>=1",
                    kMaxD);
    if (!precision_ok(precision))
        return fail(HPC_ERR_INVALID_ARG, "hpc_plan_create: unknown precision %d", precision);
    int kmax = 0;
    int rc = check_desc(desc, n_samples, idx_len, c_len, d, &kmax);
    if (rc) return rc;
    auto* p = new hpc_plan_s();
    p->d = d;
    p->D = pad_dim(d);
    p->prec = precision;
    p->n = n_samples;
    p->kmax = kmax;
    p->idx_len = idx_len;
    p->c_len = c_len;
    p->desc.assign(desc, desc + n_samples);
    auto cleanup = [&](int code) {
        if (p->mem) (void)hipFree(p->mem);
        if (p->kmem) (void)hipFree(p->kmem);
        delete p;
        return code;
    };
    if (hipGetDevice(&p->device) != hipSuccess)
        return cleanup(fail(HPC_ERR_HIP, "hpc_plan_create: hipGetDevice failed"));
    // the exchange buffers serve the most parts per sample any configuration
    // of this plan can ask for (set by the smallest sample)
    p->smin = INT32_MAX;
    for (int32_t b = 0; b < n_samples; ++b) p->smin = std::min(p->smin, desc[b].s);
    p->xparts = parts_limit(p->smin);
    const bool shareable = p->xparts > 1;
    const size_t desc_b = (size_t)n_samples * sizeof(hpc_sample_desc);
    const size_t order_b = (size_t)n_samples * 8;
    const size_t sbuf_b = (size_t)idx_len * p->D * 4;
    const size_t d2_b = (size_t)idx_len * 40;  // D^2 and up to four candidate distances
    const size_t xbuf_b = shareable ? xbuf_doubles(n_samples, p->xparts, kmax, p->D) * 8 : 0;
    const size_t xflag_b = shareable ? (size_t)n_samples * 16 : 0;
    for (int32_t b = 0; b < n_samples; ++b) p->smax = std::max(p->smax, desc[b].s);
    int cus = 0;
    rc = device_cus(&cus);
    if (rc) return cleanup(rc);
    p->kgrid_max = (int64_t)cus * kKppMaxWgPerCu;
    // the seeding teams' exchange slots for the largest team form this plan
    // can be given (any seed_team), so a later set_tune never allocates
    size_t kslot_b = 0;
    for (int T = 2; T <= kKppMaxTeam; ++T) {
        KppGeo kg;
        rc = kpp_geo(p->D, n_samples, p->smax, kmax, T, 0, &kg);
        if (rc) return cleanup(rc);
        kslot_b = std::max(kslot_b, kpp_slot_bytes(kg));
    }
    const size_t kflag_b = kpp_flag_bytes(p->kgrid_max);
    // (in an allocation of their own: the layout of the rest is the one the
    // Lloyd kernels were measured with)
    const size_t need = Carve::need({desc_b, desc_b, order_b, 256, sbuf_b, d2_b, (size_t)idx_len * 4,
                                     (size_t)c_len * 4, (size_t)n_samples * 8,
                                     (size_t)n_samples * 4, xbuf_b, xflag_b});
    hipError_t e = hipMalloc(&p->mem, need);
    if (e != hipSuccess) {
        p->mem = nullptr;
        return cleanup(fail(HPC_ERR_NO_MEMORY, "hpc_plan_create: %zu bytes: %s", need,
                            hipGetErrorString(e)));
    }
    Carve cv(p->mem);
    p->desc_dev = static_cast<hpc_sample_desc*>(cv.take(desc_b));
    p->desc_init = static_cast<hpc_sample_desc*>(cv.take(desc_b));
    p->order_dev = static_cast<int32_t*>(cv.take(order_b));
    p->queue = static_cast<int32_t*>(cv.take(256));
    p->sbuf = static_cast<float*>(cv.take(sbuf_b));
    p->d2 = static_cast<double*>(cv.take(d2_b));
    p->lbuf = static_cast<int32_t*>(cv.take((size_t)idx_len * 4));
    p->tC = static_cast<float*>(cv.take((size_t)c_len * 4));
    p->tf = static_cast<double*>(cv.take((size_t)n_samples * 8));
    p->tit = static_cast<int32_t*>(cv.take((size_t)n_samples * 4));
    if (shareable) {
        p->xbuf = static_cast<double*>(cv.take(xbuf_b));
        p->xflag = static_cast<int32_t*>(cv.take(xflag_b));
    } else {
        (void)cv.take(xbuf_b);
        (void)cv.take(xflag_b);
    }
    e = hipMalloc(&p->kmem, Carve::need({kflag_b, kslot_b}));
    if (e != hipSuccess) {
        p->kmem = nullptr;
        return cleanup(fail(HPC_ERR_NO_MEMORY, "hpc_plan_create: seeding buffers: %s",
                            hipGetErrorString(e)));
    }
    Carve ck(p->kmem);
    p->kflag = static_cast<int32_t*>(ck.take(kflag_b));
    p->kslot = static_cast<double*>(ck.take(kslot_b));
    std::vector<int32_t> orders = longest_first(desc, n_samples);
    orders.resize((size_t)2 * n_samples);
    std::iota(orders.begin() + n_samples, orders.end(), 0);
    if (hipMemcpy(p->desc_dev, desc, desc_b, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->desc_init, desc, desc_b, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->order_dev, orders.data(), order_b, hipMemcpyHostToDevice) != hipSuccess)
        return cleanup(fail(HPC_ERR_HIP, "hpc_plan_create: descriptor upload failed"));
    rc = plan_geometry(p, p->tune, &p->geo);
    if (rc) return cleanup(rc);
    rc = plan_kpp_geometry(p, p->tune.seed_team, p->tune.seed_inflight, &p->kgeo);
    if (rc) return cleanup(rc);
    *out = p;
    return HPC_OK;
}

int hpc_plan_destroy(hpc_plan plan) {
    if (!plan) return HPC_OK;
    int prev = 0;
    HPC_HIP(hipGetDevice(&prev));
    HPC_HIP(hipSetDevice(plan->device));
    HPC_HIP(hipDeviceSynchronize());
    if (plan->exec) HPC_HIP(hipGraphExecDestroy(plan->exec));
    if (plan->cap) HPC_HIP(hipStreamDestroy(plan->cap));
    if (plan->mem) HPC_HIP(hipFree(plan->mem));
    if (plan->kmem) HPC_HIP(hipFree(plan->kmem));
    delete plan;
    HPC_HIP(hipSetDevice(prev));
    return HPC_OK;
}

int hpc_plan_set_tune(hpc_plan plan, const hpc_tune* tune) {
    int rc = plan_check(plan, "hpc_plan_set_tune");
    if (rc) return rc;
    if (!tune || tune->wg_per_cu < 0 || tune->copies < 0 || tune->copies > 4 || tune->order < 0 ||
        tune->order > 1 || tune->seed_team < 0 || tune->seed_team > kKppMaxTeam ||
        tune->seed_inflight < 0 || tune->parts < 0 || tune->parts > hpc::kMaxParts)
        return fail(HPC_ERR_INVALID_ARG,
                    "hpc_plan_set_tune: need wg_per_cu>=0, copies in [0,4], order in {0,1}, "
                    "seed_team in [0,%d], seed_inflight>=0, parts in [0,%d]",
                    kKppMaxTeam, hpc::kMaxParts);
    ResGeo g;
    rc = plan_geometry(plan, *tune, &g);
    if (rc) return rc;
    KppGeo kg;
    rc = plan_kpp_geometry(plan, tune->seed_team, tune->seed_inflight, &kg);
    if (rc) return rc;
    plan->tune = *tune;
    plan->geo = g;
    plan->kgeo = kg;
    return HPC_OK;
}

int hpc_plan_get_tune(hpc_plan plan, hpc_tune* tune) {
    if (!plan || !tune) return fail(HPC_ERR_INVALID_ARG, "hpc_plan_get_tune: NULL argument");
    *tune = plan->tune;
    return HPC_OK;
}

int hpc_plan_tune_key(hpc_plan plan, char* buf, int32_t len) {
    if (!plan || !buf || len < 1) return fail(HPC_ERR_INVALID_ARG, "hpc_plan_tune_key: bad argument");
    hipDeviceProp_t prop;
    HPC_HIP(hipGetDeviceProperties(&prop, plan->device));
    int64_t sum_s = 0;
    for (const auto& ds : plan->desc) sum_s += ds.s;
    const int n = snprintf(buf, (size_t)len, "%s|d%d|p%d|n2^%d|k2^%d|s2^%d", prop.gcnArchName,
                           plan->D, plan->prec, next_pow2(plan->n), next_pow2(plan->kmax),
                           next_pow2((sum_s + plan->n - 1) / plan->n));
    if (n < 0 || n >= len) return fail(HPC_ERR_INVALID_ARG, "hpc_plan_tune_key: buffer too short");
    return HPC_OK;
}

int hpc_plan_autotune(hpc_plan plan, const float* X, int64_t m, const int64_t* idx,
                      const float* C, int32_t max_iter, double rel_tol, hpc_tune* best,
                      double* best_ms, void* hip_stream) {
    int rc = plan_check(plan, "hpc_plan_autotune");
    if (rc) return rc;
    rc = lloyd_opts_ok("hpc_plan_autotune", X, m, idx, C, max_iter, rel_tol, plan->tf, plan->tit);
    if (rc) return rc;
    if (!best) return fail(HPC_ERR_INVALID_ARG, "hpc_plan_autotune: NULL best");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    bool uneven = false;
    for (const auto& ds : plan->desc)
        uneven |= (int64_t)ds.s * ds.k != (int64_t)plan->desc[0].s * plan->desc[0].k;
    // parts per sample: automatic, then every power of two the plan's
    // exchange buffers serve (each a distinct geometry)
    std::vector<int> parts_opts{0};
    for (int P = 1; P <= plan->xparts; P *= 2) parts_opts.push_back(P);
    std::vector<hpc_tune> cand;
    for (int P : parts_opts)
        for (int copies : {1, 2, 4}) {
            hpc_tune t{0, copies, 0, 0, 0, P};
            ResGeo g;
            if (plan_geometry(plan, t, &g) != HPC_OK) continue;  // does not fit: skip
            if (P > 0 && g.split != P) continue;                 // not a geometry of its own
            for (int w = 1; w <= g.per_cu_max; ++w)
                for (int o = 0; o <= (uneven ? 1 : 0); ++o)
                    cand.push_back(hpc_tune{w, copies, o, 0, 0, P});
        }
    if (cand.empty()) return fail(HPC_ERR_UNSUPPORTED, "hpc_plan_autotune: no configuration fits");
    hipEvent_t e0, e1;
    HPC_HIP(hipEventCreate(&e0));
    HPC_HIP(hipEventCreate(&e1));
    auto run = [&](const hpc_tune& t, float* ms) -> int {
        ResGeo g;
        int r = plan_geometry(plan, t, &g);
        if (r) return r;
        HPC_HIP(hipMemcpyAsync(plan->tC, C, (size_t)plan->c_len * 4, hipMemcpyDeviceToDevice, st));
        const hpc::LloydArgs a = plan_args(plan, X, m, idx, plan->tC, max_iter, rel_tol, plan->tf,
                                           plan->tit, nullptr, t.order);
        HPC_HIP(hipEventRecord(e0, st));
        r = plan_launch(plan, a, g, st);
        if (r) return r;
        HPC_HIP(hipEventRecord(e1, st));
        HPC_HIP(hipEventSynchronize(e1));
        HPC_HIP(hipEventElapsedTime(ms, e0, e1));
        return HPC_OK;
    };
    float warm = 0.f;
    rc = run(cand[0], &warm);
    double tbest = 1e300;
    hpc_tune tb = cand[0];
    for (size_t i = 0; rc == HPC_OK && i < cand.size(); ++i) {
        float a = 0.f, b = 0.f;
        rc = run(cand[i], &a);
        if (rc == HPC_OK) rc = run(cand[i], &b);
        const double t = std::min(a, b);
        if (rc == HPC_OK && t < tbest) {
            tbest = t;
            tb = cand[i];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    rc = hpc_plan_set_tune(plan, &tb);
    if (rc) return rc;
    *best = tb;
    if (best_ms) *best_ms = tbest;
    return HPC_OK;
}

int hpc_plan_lloyd(hpc_plan plan, const float* X, int64_t m, const int64_t* idx, float* C,
                   int32_t max_iter, double rel_tol, double* f_out, int32_t* iters_out,
                   int32_t* labels_out, void* hip_stream) {
    int rc = plan_check(plan, "hpc_plan_lloyd");
    if (rc) return rc;
    rc = lloyd_opts_ok("hpc_plan_lloyd", X, m, idx, C, max_iter, rel_tol, f_out, iters_out);
    if (rc) return rc;
    const hpc::LloydArgs a = plan_args(plan, X, m, idx, C, max_iter, rel_tol, f_out, iters_out,
                                       labels_out, plan->tune.order);
    return plan_launch(plan, a, plan->geo, static_cast<hipStream_t>(hip_stream));
}

int hpc_plan_draw(hpc_plan plan, int64_t m, int64_t* idx, void* hip_stream) {
    int rc = plan_check(plan, "hpc_plan_draw");
    if (rc) return rc;
    if (m < 1 || !idx) return fail(HPC_ERR_INVALID_ARG, "hpc_plan_draw: need m >= 1, idx");
    plan_draw(plan, m, idx, static_cast<hipStream_t>(hip_stream));
    HPC_HIP(hipGetLastError());
    return HPC_OK;
}

int hpc_plan_advance(hpc_plan plan, uint64_t id_stride, void* hip_stream) {
    int rc = plan_check(plan, "hpc_plan_advance");
    if (rc) return rc;
    plan_advance(plan, id_stride, static_cast<hipStream_t>(hip_stream));
    HPC_HIP(hipGetLastError());
    return HPC_OK;
}

int hpc_plan_round(hpc_plan plan, const float* X, int64_t m, int64_t* idx, float* C, float* C_inc,
                   double* f_inc, int32_t max_iter, double rel_tol, double* f_out,
                   int32_t* iters_out, uint64_t id_stride, void* hip_stream) {
    int rc = plan_check(plan, "hpc_plan_round");
    if (rc) return rc;
    rc = lloyd_opts_ok("hpc_plan_round", X, m, idx, C, max_iter, rel_tol, f_out, iters_out);
    if (rc) return rc;
    if (!C_inc || !f_inc) return fail(HPC_ERR_INVALID_ARG, "hpc_plan_round: NULL incumbents");
    return plan_enqueue_round(plan, X, m, idx, C, C_inc, f_inc, max_iter, rel_tol, f_out,
                              iters_out, id_stride, static_cast<hipStream_t>(hip_stream));
}

int hpc_plan_capture_round(hpc_plan plan, const float* X, int64_t m, int64_t* idx, float* C,
                           float* C_inc, double* f_inc, int32_t max_iter, double rel_tol,
                           double* f_out, int32_t* iters_out, uint64_t id_stride) {
    int rc = plan_check(plan, "hpc_plan_capture_round");
    if (rc) return rc;
    rc = lloyd_opts_ok("hpc_plan_capture_round", X, m, idx, C, max_iter, rel_tol, f_out, iters_out);
    if (rc) return rc;
    if (!C_inc || !f_inc)
        return fail(HPC_ERR_INVALID_ARG, "hpc_plan_capture_round: NULL incumbents");
    if (!plan->cap) HPC_HIP(hipStreamCreateWithFlags(&plan->cap, hipStreamNonBlocking));
    if (plan->exec) {
        HPC_HIP(hipGraphExecDestroy(plan->exec));
        plan->exec = nullptr;
    }
    HPC_HIP(hipStreamBeginCapture(plan->cap, hipStreamCaptureModeThreadLocal));
    rc = plan_enqueue_round(plan, X, m, idx, C, C_inc, f_inc, max_iter, rel_tol, f_out, iters_out,
                            id_stride, plan->cap);
    hipGraph_t graph = nullptr;
    const hipError_t ee = hipStreamEndCapture(plan->cap, &graph);
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (ee != hipSuccess)
        return fail(HPC_ERR_HIP, "hipStreamEndCapture failed: %s", hipGetErrorString(ee));
    const hipError_t ei = hipGraphInstantiate(&plan->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
        plan->exec = nullptr;
        return fail(HPC_ERR_HIP, "hipGraphInstantiate failed: %s", hipGetErrorString(ei));
    }
    return HPC_OK;
}

int hpc_plan_replay(hpc_plan plan, int32_t n_rounds, void* hip_stream) {
    int rc = plan_check(plan, "hpc_plan_replay");
    if (rc) return rc;
    if (!plan->exec) return fail(HPC_ERR_INVALID_ARG, "hpc_plan_replay: no captured round");
    if (n_rounds < 0) return fail(HPC_ERR_INVALID_ARG, "hpc_plan_replay: n_rounds < 0");
    for (int32_t r = 0; r < n_rounds; ++r)
        HPC_HIP(hipGraphLaunch(plan->exec, static_cast<hipStream_t>(hip_stream)));
    return HPC_OK;
}

int hpc_plan_reset_ids(hpc_plan plan, void* hip_stream) {
    int rc = plan_check(plan, "hpc_plan_reset_ids");
    if (rc) return rc;
    HPC_HIP(hipMemcpyAsync(plan->desc_dev, plan->desc_init, (size_t)plan->n * sizeof(hpc_sample_desc),
                           hipMemcpyDeviceToDevice, static_cast<hipStream_t>(hip_stream)));
    return HPC_OK;
}

}  // extern "C"

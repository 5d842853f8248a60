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
#include <utility>
#include <vector>

#include "../../include/hpclust.h"
#include "assign_misc.hpp"
#include "common.hpp"
#include "lloyd_resident.hpp"

namespace {

thread_local std::string g_last_error = "";

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define HPC_HIP(call)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(HPC_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_));      \
    } while (0)

constexpr int kMaxD = 128;
constexpr int kNT = 256;  // threads per workgroup of the resident kernels

int pad_dim(int d) {
    if (d <= 8) return 8;
    if (d <= 16) return 16;
    if (d <= 32) return 32;
    if (d <= 64) return 64;
    return 128;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Grow-only device scratch plus a pinned host staging area for descriptor
// uploads, one per (device, stream).
struct Workspace {
    void* dev = nullptr;
    size_t dev_cap = 0;
    void* pinned = nullptr;
    size_t pinned_cap = 0;
    hipEvent_t staged = nullptr;  // last copy out of the pinned area
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
        HPC_HIP(hipEventCreateWithFlags(&w->staged, hipEventDisableTiming));
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

// Copy `bytes` of host data to device scratch at `dst` on the stream via the
// pinned staging area (waits for the previous staged copy to have run).
int ws_upload(Workspace* w, void* dst, const void* src, size_t bytes) {
    HPC_HIP(hipEventSynchronize(w->staged));
    if (bytes > w->pinned_cap) {
        if (w->pinned) HPC_HIP(hipHostFree(w->pinned));
        w->pinned = nullptr;
        size_t cap = align_up(std::max(bytes, (size_t)4096), 4096);
        HPC_HIP(hipHostMalloc(&w->pinned, cap, hipHostMallocDefault));
        w->pinned_cap = cap;
    }
    memcpy(w->pinned, src, bytes);
    HPC_HIP(hipMemcpyAsync(dst, w->pinned, bytes, hipMemcpyHostToDevice, w->stream));
    HPC_HIP(hipEventRecord(w->staged, w->stream));
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

// --------------------------------------------------------------------------
// Resident Lloyd / seeding launch.
// --------------------------------------------------------------------------
template <int D, int PREC>
int launch_resident(hpc::LloydArgs a, int n_wg, hipStream_t st) {
    using S = hpc::Smem<D, kNT, PREC>;
    constexpr int NW = kNT / hpc::kWave;
    int lds_max = 0;
    int rc = max_dyn_lds(&lds_max);
    if (rc) return rc;
    // as many private partial-sum copies as fit (one per wave = no atomics)
    int copies = NW;
    const size_t soft = 64 * 1024;
    while (copies > 1 && S::bytes(a.kmax, copies) > soft) --copies;
    size_t lds = S::bytes(a.kmax, copies);
    if (lds > (size_t)lds_max)
        return fail(HPC_ERR_UNSUPPORTED,
                    "k=%d with padded d=%d needs %zu bytes of LDS per workgroup (limit %d)",
                    a.kmax, D, lds, lds_max);
    a.n_copies = copies;
    auto kern = hpc::k_lloyd_resident<D, kNT, PREC>;
    if (lds > 64 * 1024)
        HPC_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int per_cu = 0;
    HPC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kNT, lds));
    int cus = 0;
    rc = device_cus(&cus);
    if (rc) return rc;
    int grid = std::max(1, std::min(n_wg, cus * std::max(1, per_cu)));
    hipLaunchKernelGGL(hpc::k_fill_i32, dim3(1), dim3(64), 0, st, a.queue, (int64_t)1, 0);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kNT), lds, st, a);
    HPC_HIP(hipGetLastError());
    return HPC_OK;
}

int dispatch_resident(int D, int prec, const hpc::LloydArgs& a, int n_wg, hipStream_t st) {
    const bool bf = prec == HPC_PREC_BF16_MFMA;
    switch (D) {
        case 8: return bf ? launch_resident<8, hpc::kPrecBF16>(a, n_wg, st)
                          : launch_resident<8, hpc::kPrecF32>(a, n_wg, st);
        case 16: return bf ? launch_resident<16, hpc::kPrecBF16>(a, n_wg, st)
                           : launch_resident<16, hpc::kPrecF32>(a, n_wg, st);
        case 32: return bf ? launch_resident<32, hpc::kPrecBF16>(a, n_wg, st)
                           : launch_resident<32, hpc::kPrecF32>(a, n_wg, st);
        case 64: return bf ? launch_resident<64, hpc::kPrecBF16>(a, n_wg, st)
                           : launch_resident<64, hpc::kPrecF32>(a, n_wg, st);
        case 128: return bf ? launch_resident<128, hpc::kPrecBF16>(a, n_wg, st)
                            : launch_resident<128, hpc::kPrecF32>(a, n_wg, st);
    }
    return fail(HPC_ERR_UNSUPPORTED, "padded dimension %d", D);
}

template <int D, int PREC>
int launch_assign(const float* X, int64_t m, int d, const float* C, int k, int32_t* labels,
                  int64_t* counts, double* sse, Workspace* w, hipStream_t st) {
    constexpr int NT = 256;
    const size_t lds = hpc::assign_lds_bytes<D, PREC>(k, NT);
    int lds_max = 0;
    int rc = max_dyn_lds(&lds_max);
    if (rc) return rc;
    if (lds > (size_t)lds_max)
        return fail(HPC_ERR_UNSUPPORTED, "k=%d, padded d=%d: centroids exceed LDS", k, D);
    auto kern = hpc::k_assign_sse<D, NT, PREC>;
    if (lds > 64 * 1024)
        HPC_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int per_cu = 0, cus = 0;
    HPC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, NT, lds));
    rc = device_cus(&cus);
    if (rc) return rc;
    int64_t want = (m + 63) / 64;  // tiles of 16 rows per wave, 4 waves
    int grid = (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)cus * std::max(1, per_cu) * 4));
    rc = ws_reserve_dev(w, Carve::need({(size_t)grid * 8}));
    if (rc) return rc;
    Carve cv(w->dev);
    double* partials = static_cast<double*>(cv.take((size_t)grid * 8));
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
    // longest first: work ~ s * k
    std::vector<int32_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return (int64_t)desc[a].s * desc[a].k > (int64_t)desc[b].s * desc[b].k;
    });
    const size_t desc_b = (size_t)n * sizeof(hpc_sample_desc);
    const size_t order_b = (size_t)n * 4;
    const size_t sbuf_b = (size_t)idx_len * D * 4;
    const size_t need = Carve::need({desc_b + order_b, 256, sbuf_b, (size_t)idx_len * 8});
    rc = ws_reserve_dev(w, need);
    if (rc) return rc;
    Carve cv(w->dev);
    char* tbl = static_cast<char*>(cv.take(desc_b + order_b));
    int32_t* queue = static_cast<int32_t*>(cv.take(256));
    float* sbuf = static_cast<float*>(cv.take(sbuf_b));
    double* d2 = static_cast<double*>(cv.take((size_t)idx_len * 8));
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
    a.queue = queue;
    a.kmax = kmax;
    a.seed_only = seed_only;
    a.n_cand = n_cand;
    a.call_id = call_id;
    a.chosen = chosen;
    a.vec4 = (d % 4 == 0) && (reinterpret_cast<uintptr_t>(X) % 16 == 0);
    return dispatch_resident(D, precision, a, n, st);
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
        if (w->pinned) HPC_HIP(hipHostFree(w->pinned));
        if (w->staged) HPC_HIP(hipEventDestroy(w->staged));
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
    if (precision != HPC_PREC_FP32 && precision != HPC_PREC_BF16_MFMA)
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

int hpc_assign_sse(const float* X, int64_t m, int32_t d, const float* C, int32_t k,
                   int32_t precision, int32_t* labels, int64_t* counts, double* sse,
                   void* hip_stream) {
    if (!X || !C || !sse) return fail(HPC_ERR_INVALID_ARG, "hpc_assign_sse: NULL pointer");
    if (m < 1 || !sizes_ok(d, k))
        return fail(HPC_ERR_INVALID_ARG, "hpc_assign_sse: need m>=1, 1<=d<=%d, 1<=k<=512", kMaxD);
    if (precision != HPC_PREC_FP32 && precision != HPC_PREC_BF16_MFMA)
        return fail(HPC_ERR_INVALID_ARG, "hpc_assign_sse: unknown precision %d", precision);
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    Workspace* w = nullptr;
    int rc = get_ws(st, &w);
    if (rc) return rc;
    const bool bf = precision == HPC_PREC_BF16_MFMA;
#define HPC_ASSIGN(DD)                                                                       \
    return bf ? launch_assign<DD, hpc::kPrecBF16>(X, m, d, C, k, labels, counts, sse, w, st) \
              : launch_assign<DD, hpc::kPrecF32>(X, m, d, C, k, labels, counts, sse, w, st)
    switch (pad_dim(d)) {
        case 8: HPC_ASSIGN(8);
        case 16: HPC_ASSIGN(16);
        case 32: HPC_ASSIGN(32);
        case 64: HPC_ASSIGN(64);
        case 128: HPC_ASSIGN(128);
    }
#undef HPC_ASSIGN
    return fail(HPC_ERR_UNSUPPORTED, "hpc_assign_sse: d=%d", d);
}

}  // extern "C"

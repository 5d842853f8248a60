// Host side of the learned initializer (set encoder; include/hpclust.h,
// "Learned initializer"): the model object, its forward / backward / Adam
// entry points, and the proposal-or-K-means++ seeding of a batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/hpclust.h"
#include "host_util.hpp"
#include "setenc.hpp"

using hpc_host::fail;
namespace enc = hpc::enc;
using hpc::bf16x8;

struct hpc_setenc_s {
    int device = 0;
    int32_t d = 0, k = 0, kd = 0, n_enc = 0, max_batch = 0, chunks = 0;
    enc::Layout L{};
    int64_t step = 0;  // Adam steps taken
    // fixed allocation: parameters, gradients, Adam moments, operand tables,
    // training scratch (max_batch samples)
    char* mem = nullptr;
    float *theta = nullptr, *grad = nullptr, *m1 = nullptr, *m2 = nullptr;
    bf16x8 *W1s = nullptr, *W2Ts = nullptr, *W2s = nullptr;
    float* Whr = nullptr;
    float *g2 = nullptr, *dout = nullptr;
    double* loss_part = nullptr;
    float *sX = nullptr, *sH1 = nullptr, *sG2 = nullptr, *sG1 = nullptr, *wpart = nullptr;
    int wsplits = 0;
    // grow-only per-sample buffers (any batch size)
    char* imem = nullptr;
    int32_t icap = 0;
    float *stats = nullptr, *pooled_part = nullptr, *pooled = nullptr, *obuf = nullptr;
    int32_t* its = nullptr;
    hpc_sample_desc* desc_dev = nullptr;
    // pinned staging of descriptor uploads
    void* pinned = nullptr;
    size_t pinned_cap = 0;
    hipEvent_t staged = nullptr;
};

namespace {

size_t al(size_t v) { return (v + 255) / 256 * 256; }

int check_model(hpc_setenc s, const char* where) {
    if (!s) return fail(HPC_ERR_INVALID_ARG, "%s: NULL model", where);
    int dev = 0;
    HPC_HIP(hipGetDevice(&dev));
    if (dev != s->device)
        return fail(HPC_ERR_INVALID_ARG, "%s: model lives on device %d, current is %d", where,
                    s->device, dev);
    return HPC_OK;
}

int swizzle(hpc_setenc s, hipStream_t st) {
    hipLaunchKernelGGL(enc::k_enc_swizzle, dim3(256), dim3(256), 0, st, (const float*)s->theta,
                       s->d, s->kd, s->W1s, s->W2Ts, s->W2s, s->Whr);
    HPC_HIP(hipGetLastError());
    return HPC_OK;
}

// Per-sample buffers for n samples (grows; synchronises the device before
// freeing a smaller set).
int reserve_infer(hpc_setenc s, int32_t n) {
    if (n <= s->icap) return HPC_OK;
    const int32_t cap = std::max(n, s->icap * 2);
    if (s->imem) {
        HPC_HIP(hipDeviceSynchronize());
        HPC_HIP(hipFree(s->imem));
        s->imem = nullptr;
        s->icap = 0;
    }
    const size_t b_stats = al((size_t)cap * (enc::DIN + 2) * 4);
    const size_t b_part = al((size_t)cap * s->chunks * enc::H * 4);
    const size_t b_pool = al((size_t)cap * enc::H * 4);
    const size_t b_o = al((size_t)cap * s->kd * 4);
    const size_t b_its = al((size_t)cap * 4);
    const size_t b_desc = al((size_t)cap * sizeof(hpc_sample_desc));
    hipError_t e = hipMalloc(&s->imem, b_stats + b_part + b_pool + b_o + b_its + b_desc);
    if (e != hipSuccess) {
        s->imem = nullptr;
        return fail(HPC_ERR_NO_MEMORY, "set encoder: per-sample buffers for %d samples: %s", cap,
                    hipGetErrorString(e));
    }
    char* p = s->imem;
    s->stats = reinterpret_cast<float*>(p);
    p += b_stats;
    s->pooled_part = reinterpret_cast<float*>(p);
    p += b_part;
    s->pooled = reinterpret_cast<float*>(p);
    p += b_pool;
    s->obuf = reinterpret_cast<float*>(p);
    p += b_o;
    s->its = reinterpret_cast<int32_t*>(p);
    p += b_its;
    s->desc_dev = reinterpret_cast<hpc_sample_desc*>(p);
    s->icap = cap;
    return HPC_OK;
}

int upload_desc(hpc_setenc s, const hpc_sample_desc* desc, int32_t n, hipStream_t st) {
    const size_t bytes = (size_t)n * sizeof(hpc_sample_desc);
    HPC_HIP(hipEventSynchronize(s->staged));
    if (bytes > s->pinned_cap) {
        if (s->pinned) HPC_HIP(hipHostFree(s->pinned));
        s->pinned = nullptr;
        const size_t cap = std::max<size_t>(al(bytes), 4096);
        HPC_HIP(hipHostMalloc(&s->pinned, cap, hipHostMallocDefault));
        s->pinned_cap = cap;
    }
    memcpy(s->pinned, desc, bytes);
    HPC_HIP(hipMemcpyAsync(s->desc_dev, s->pinned, bytes, hipMemcpyHostToDevice, st));
    HPC_HIP(hipEventRecord(s->staged, st));
    return HPC_OK;
}

int check_batch(hpc_setenc s, const char* where, const int64_t* idx, int64_t idx_len,
                const hpc_sample_desc* desc, int32_t n, int64_t c_len) {
    if (!idx || !desc || n < 1 || n > 65535)
        return fail(HPC_ERR_INVALID_ARG, "%s: need idx, desc and 1 <= n <= 65535", where);
    for (int32_t b = 0; b < n; ++b) {
        const hpc_sample_desc& ds = desc[b];
        if (ds.k != s->k)
            return fail(HPC_ERR_INVALID_ARG, "%s: sample %d has k=%d, the model proposes k=%d",
                        where, b, ds.k, s->k);
        if (ds.s < ds.k || ds.idx_offset < 0 || ds.idx_offset + ds.s > idx_len)
            return fail(HPC_ERR_INVALID_ARG, "%s: sample %d: s=%d or idx range outside idx_len",
                        where, b, ds.s);
        if (ds.c_offset < 0 || ds.c_offset + (int64_t)s->kd > c_len)
            return fail(HPC_ERR_INVALID_ARG, "%s: sample %d: centroid block outside c_len", where,
                        b);
    }
    return HPC_OK;
}

enc::RowArgs row_args(hpc_setenc s, const float* X, int64_t m, const int64_t* idx) {
    enc::RowArgs a{};
    a.X = X;
    a.m = m;
    a.d = s->d;
    a.idx = idx;
    a.desc = s->desc_dev;
    a.n_enc = s->n_enc;
    a.stats = s->stats;
    a.W1s = s->W1s;
    a.W2Ts = s->W2Ts;
    a.W2s = s->W2s;
    a.b1 = s->theta + s->L.b1;
    a.b2 = s->theta + s->L.b2;
    a.pooled_part = s->pooled_part;
    a.chunks = s->chunks;
    a.g2 = s->g2;
    a.sX = s->sX;
    a.sH1 = s->sH1;
    a.sG2 = s->sG2;
    a.sG1 = s->sG1;
    return a;
}

// Normalisation, per-point layers, pooling and head for n samples (desc
// already on the device).  C nullable.
int forward(hpc_setenc s, const float* X, int64_t m, const int64_t* idx, int32_t n, float* C,
            hipStream_t st) {
    hipLaunchKernelGGL(enc::k_enc_stats, dim3(n), dim3(enc::NT), 0, st, X, m, s->d, idx,
                       (const hpc_sample_desc*)s->desc_dev, s->n_enc, s->stats);
    const enc::RowArgs a = row_args(s, X, m, idx);
    hipLaunchKernelGGL(enc::k_enc_rows<false>, dim3(s->chunks, n), dim3(enc::NT), 0, st, a);
    hipLaunchKernelGGL(enc::k_enc_pool, dim3(n), dim3(256), 0, st, (const float*)s->pooled_part,
                       s->chunks, (const hpc_sample_desc*)s->desc_dev, s->n_enc, s->pooled);
    hipLaunchKernelGGL(enc::k_enc_head, dim3((s->kd + 255) / 256, n), dim3(256), 0, st,
                       (const float*)s->pooled, (const float*)s->Whr,
                       (const float*)(s->theta + s->L.bh), s->kd, s->d, (const float*)s->stats,
                       (const hpc_sample_desc*)s->desc_dev, s->obuf, C);
    HPC_HIP(hipGetLastError());
    return HPC_OK;
}

// grad[off .. off + M*N) = A^T B over P rows (split partials, fixed order).
int wgrad(hpc_setenc s, const float* A, int lda, int M, const float* B, int ldb, int N, int64_t P,
          float* out, hipStream_t st) {
    const int splits = s->wsplits;
    const int64_t per = ((P + splits - 1) / splits + 31) / 32 * 32;
    hipLaunchKernelGGL(enc::k_wgrad, dim3((M + 63) / 64, (N + 63) / 64, splits), dim3(256), 0, st,
                       A, lda, M, B, ldb, N, P, per, s->wpart);
    hipLaunchKernelGGL(enc::k_sum_splits, dim3(256), dim3(256), 0, st, (const float*)s->wpart,
                       splits, (int64_t)M * N, out);
    HPC_HIP(hipGetLastError());
    return HPC_OK;
}

int colsum(hpc_setenc s, const float* B, int ldb, int N, int64_t P, float* out, hipStream_t st) {
    // about 128 rows per split (the partials buffer holds wsplits x H x
    // max(H, kd) floats, far more than splits x N)
    const int splits = (int)std::max<int64_t>(1, std::min<int64_t>(512, (P + 127) / 128));
    const int64_t per = (P + splits - 1) / splits;
    hipLaunchKernelGGL(enc::k_colsum, dim3((N + 255) / 256, splits), dim3(256), 0, st, B, ldb, N,
                       P, per, s->wpart);
    hipLaunchKernelGGL(enc::k_sum_splits, dim3(4), dim3(256), 0, st, (const float*)s->wpart,
                       splits, (int64_t)N, out);
    HPC_HIP(hipGetLastError());
    return HPC_OK;
}

__global__ void k_sum_loss(const double* __restrict__ part, int32_t n, double* __restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += part[i];
        *out = s;
    }
}

__global__ void k_fill_f32(float* __restrict__ p, int64_t n, float v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Keep the proposal where its sample objective is no larger than the
// K-means++ seeding's; otherwise copy the seeding.  One workgroup per sample.
__global__ void k_select_init(const hpc_sample_desc* __restrict__ desc, int32_t kd,
                              const double* __restrict__ f_prop, const double* __restrict__ f_kpp,
                              const float* __restrict__ C_kpp, float* __restrict__ C,
                              int32_t* __restrict__ accepted) {
    const int b = blockIdx.x;
    const bool take = f_prop[b] <= f_kpp[b];
    if (!take)
        for (int e = threadIdx.x; e < kd; e += blockDim.x)
            C[desc[b].c_offset + e] = C_kpp[desc[b].c_offset + e];
    if (threadIdx.x == 0 && accepted) accepted[b] = take ? 1 : 0;
}

}  // namespace

extern "C" {

int hpc_setenc_create(int32_t d, int32_t k, int32_t n_enc, int32_t max_batch, uint64_t seed,
                      hpc_setenc* out) {
    if (!out) return fail(HPC_ERR_INVALID_ARG, "hpc_setenc_create: NULL out");
    *out = nullptr;
    if (d < 1 || d > enc::DIN || k < 1 || k > 64 || n_enc < 16 || n_enc > (1 << 20) ||
        max_batch < 1 || max_batch > 65535)
        return fail(HPC_ERR_INVALID_ARG,
                    "hpc_setenc_create: need 1<=d<=%d, 1<=k<=64, 16<=n_enc<=2^20, "
                    "1<=max_batch<=65535",
                    enc::DIN);
    auto* s = new hpc_setenc_s();
    s->d = d;
    s->k = k;
    s->kd = k * d;
    s->n_enc = n_enc;
    s->max_batch = max_batch;
    s->chunks = (n_enc + enc::CH - 1) / enc::CH;
    s->L = enc::Layout::of(d, s->kd);
    s->wsplits = 64;
    auto bail = [&](int code) {
        if (s->mem) (void)hipFree(s->mem);
        if (s->staged) (void)hipEventDestroy(s->staged);
        delete s;
        return code;
    };
    if (hipGetDevice(&s->device) != hipSuccess)
        return bail(fail(HPC_ERR_HIP, "hpc_setenc_create: hipGetDevice failed"));
    if (hipEventCreateWithFlags(&s->staged, hipEventDisableTiming) != hipSuccess)
        return bail(fail(HPC_ERR_HIP, "hpc_setenc_create: event creation failed"));
    const int64_t P = (int64_t)max_batch * n_enc;
    const size_t np = (size_t)s->L.total;
    const size_t b_par = al(np * 4);
    const size_t b_w1s = al((size_t)enc::NMB * 64 * 16), b_w2 = al((size_t)enc::NMB * enc::NKB * 64 * 16);
    const size_t b_whr = al((size_t)enc::H * s->kd * 4);
    const size_t b_g2 = al((size_t)max_batch * enc::H * 4), b_dout = al((size_t)max_batch * s->kd * 4);
    const size_t b_lp = al((size_t)max_batch * 8);
    const size_t b_sx = al((size_t)P * enc::DIN * 4), b_sh = al((size_t)P * enc::H * 4);
    const size_t b_wp = al((size_t)s->wsplits * enc::H * std::max(enc::H, s->kd) * 4);
    const size_t total = 4 * b_par + b_w1s + 2 * b_w2 + b_whr + b_g2 + b_dout + b_lp + b_sx +
                         3 * b_sh + b_wp;
    hipError_t e = hipMalloc(&s->mem, total);
    if (e != hipSuccess) {
        s->mem = nullptr;
        return bail(fail(HPC_ERR_NO_MEMORY, "hpc_setenc_create: %zu bytes: %s", total,
                         hipGetErrorString(e)));
    }
    char* p = s->mem;
    auto take = [&](size_t b) {
        char* q = p;
        p += b;
        return q;
    };
    s->theta = reinterpret_cast<float*>(take(b_par));
    s->grad = reinterpret_cast<float*>(take(b_par));
    s->m1 = reinterpret_cast<float*>(take(b_par));
    s->m2 = reinterpret_cast<float*>(take(b_par));
    s->W1s = reinterpret_cast<bf16x8*>(take(b_w1s));
    s->W2Ts = reinterpret_cast<bf16x8*>(take(b_w2));
    s->W2s = reinterpret_cast<bf16x8*>(take(b_w2));
    s->Whr = reinterpret_cast<float*>(take(b_whr));
    s->g2 = reinterpret_cast<float*>(take(b_g2));
    s->dout = reinterpret_cast<float*>(take(b_dout));
    s->loss_part = reinterpret_cast<double*>(take(b_lp));
    s->sX = reinterpret_cast<float*>(take(b_sx));
    s->sH1 = reinterpret_cast<float*>(take(b_sh));
    s->sG2 = reinterpret_cast<float*>(take(b_sh));
    s->sG1 = reinterpret_cast<float*>(take(b_sh));
    s->wpart = reinterpret_cast<float*>(take(b_wp));
    hipLaunchKernelGGL(enc::k_enc_init, dim3(256), dim3(256), 0, nullptr, s->theta, d, s->kd, seed);
    hipLaunchKernelGGL(k_fill_f32, dim3(256), dim3(256), 0, nullptr, s->m1, (int64_t)np, 0.f);
    hipLaunchKernelGGL(k_fill_f32, dim3(256), dim3(256), 0, nullptr, s->m2, (int64_t)np, 0.f);
    hipLaunchKernelGGL(k_fill_f32, dim3(256), dim3(256), 0, nullptr, s->grad, (int64_t)np, 0.f);
    int rc = swizzle(s, nullptr);
    if (rc) return bail(rc);
    if (hipDeviceSynchronize() != hipSuccess)
        return bail(fail(HPC_ERR_HIP, "hpc_setenc_create: initialisation failed"));
    *out = s;
    return HPC_OK;
}

int hpc_setenc_destroy(hpc_setenc model) {
    if (!model) return HPC_OK;
    int prev = 0;
    HPC_HIP(hipGetDevice(&prev));
    HPC_HIP(hipSetDevice(model->device));
    HPC_HIP(hipDeviceSynchronize());
    if (model->mem) HPC_HIP(hipFree(model->mem));
    if (model->imem) HPC_HIP(hipFree(model->imem));
    if (model->pinned) HPC_HIP(hipHostFree(model->pinned));
    if (model->staged) HPC_HIP(hipEventDestroy(model->staged));
    delete model;
    HPC_HIP(hipSetDevice(prev));
    return HPC_OK;
}

int hpc_setenc_param_count(hpc_setenc model, int64_t* n_params) {
    if (!model || !n_params) return fail(HPC_ERR_INVALID_ARG, "hpc_setenc_param_count: NULL");
    *n_params = model->L.total;
    return HPC_OK;
}

int hpc_setenc_get_params(hpc_setenc model, int32_t rounded, float* host) {
    int rc = check_model(model, "hpc_setenc_get_params");
    if (rc) return rc;
    if (!host) return fail(HPC_ERR_INVALID_ARG, "hpc_setenc_get_params: NULL host");
    HPC_HIP(hipDeviceSynchronize());
    HPC_HIP(hipMemcpy(host, model->theta, (size_t)model->L.total * 4, hipMemcpyDeviceToHost));
    if (rounded) {
        // the values the kernels use: weights rounded to BF16 (nearest even)
        auto rnd = [](float v) { return (float)(__bf16)v; };
        const enc::Layout& L = model->L;
        for (int64_t e = L.W1; e < L.b1; ++e) host[e] = rnd(host[e]);
        for (int64_t e = L.W2; e < L.b2; ++e) host[e] = rnd(host[e]);
        for (int64_t e = L.Wh; e < L.bh; ++e) host[e] = rnd(host[e]);
    }
    return HPC_OK;
}

int hpc_setenc_set_params(hpc_setenc model, const float* host) {
    int rc = check_model(model, "hpc_setenc_set_params");
    if (rc) return rc;
    if (!host) return fail(HPC_ERR_INVALID_ARG, "hpc_setenc_set_params: NULL host");
    HPC_HIP(hipDeviceSynchronize());
    HPC_HIP(hipMemcpy(model->theta, host, (size_t)model->L.total * 4, hipMemcpyHostToDevice));
    rc = swizzle(model, nullptr);
    if (rc) return rc;
    HPC_HIP(hipDeviceSynchronize());
    return HPC_OK;
}

int hpc_setenc_get_grads(hpc_setenc model, float* host) {
    int rc = check_model(model, "hpc_setenc_get_grads");
    if (rc) return rc;
    if (!host) return fail(HPC_ERR_INVALID_ARG, "hpc_setenc_get_grads: NULL host");
    HPC_HIP(hipDeviceSynchronize());
    HPC_HIP(hipMemcpy(host, model->grad, (size_t)model->L.total * 4, hipMemcpyDeviceToHost));
    return HPC_OK;
}

int hpc_setenc_propose(hpc_setenc model, const float* X, int64_t m, const int64_t* idx,
                       int64_t idx_len, const hpc_sample_desc* desc, int32_t n_samples, float* C,
                       int64_t c_len, void* hip_stream) {
    int rc = check_model(model, "hpc_setenc_propose");
    if (rc) return rc;
    if (!X || !C || m < 1) return fail(HPC_ERR_INVALID_ARG, "hpc_setenc_propose: need X, C, m>=1");
    rc = check_batch(model, "hpc_setenc_propose", idx, idx_len, desc, n_samples, c_len);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    rc = reserve_infer(model, n_samples);
    if (rc) return rc;
    rc = upload_desc(model, desc, n_samples, st);
    if (rc) return rc;
    return forward(model, X, m, idx, n_samples, C, st);
}

int hpc_setenc_grad(hpc_setenc model, const float* X, int64_t m, const int64_t* idx,
                    int64_t idx_len, const hpc_sample_desc* desc, int32_t n_samples,
                    const float* T, int64_t c_len, double* loss, void* hip_stream) {
    int rc = check_model(model, "hpc_setenc_grad");
    if (rc) return rc;
    if (!X || !T || m < 1) return fail(HPC_ERR_INVALID_ARG, "hpc_setenc_grad: need X, T, m>=1");
    if (n_samples > model->max_batch)
        return fail(HPC_ERR_INVALID_ARG, "hpc_setenc_grad: %d samples > max_batch %d", n_samples,
                    model->max_batch);
    rc = check_batch(model, "hpc_setenc_grad", idx, idx_len, desc, n_samples, c_len);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    rc = reserve_infer(model, n_samples);
    if (rc) return rc;
    rc = upload_desc(model, desc, n_samples, st);
    if (rc) return rc;
    rc = forward(model, X, m, idx, n_samples, nullptr, st);
    if (rc) return rc;
    const int32_t B = n_samples, kd = model->kd;
    const enc::Layout& L = model->L;
    hipLaunchKernelGGL(enc::k_enc_loss, dim3(B), dim3(256), 0, st, (const float*)model->obuf, T,
                       (const float*)model->stats, (const hpc_sample_desc*)model->desc_dev,
                       model->k, model->d, B, model->dout, model->loss_part);
    hipLaunchKernelGGL(enc::k_enc_head_wgrad, dim3((kd + 255) / 256, enc::H + 1), dim3(256), 0, st,
                       (const float*)model->pooled, (const float*)model->dout, B, kd,
                       model->grad + L.Wh, model->grad + L.bh);
    hipLaunchKernelGGL(enc::k_enc_head_dp, dim3(B), dim3(enc::H), 0, st, (const float*)model->Whr,
                       (const float*)model->dout, kd, (const hpc_sample_desc*)model->desc_dev,
                       model->n_enc, model->g2);
    const enc::RowArgs a = row_args(model, X, m, idx);
    hipLaunchKernelGGL(enc::k_enc_rows<true>, dim3(model->chunks, B), dim3(enc::NT), 0, st, a);
    const int64_t P = (int64_t)B * model->n_enc;
    rc = wgrad(model, model->sH1, enc::H, enc::H, model->sG2, enc::H, enc::H, P,
               model->grad + L.W2, st);
    if (rc) return rc;
    rc = wgrad(model, model->sX, enc::DIN, model->d, model->sG1, enc::H, enc::H, P,
               model->grad + L.W1, st);
    if (rc) return rc;
    rc = colsum(model, model->sG2, enc::H, enc::H, P, model->grad + L.b2, st);
    if (rc) return rc;
    rc = colsum(model, model->sG1, enc::H, enc::H, P, model->grad + L.b1, st);
    if (rc) return rc;
    if (loss)
        hipLaunchKernelGGL(k_sum_loss, dim3(1), dim3(64), 0, st, (const double*)model->loss_part,
                           B, loss);
    HPC_HIP(hipGetLastError());
    return HPC_OK;
}

int hpc_setenc_adam(hpc_setenc model, float lr, void* hip_stream) {
    int rc = check_model(model, "hpc_setenc_adam");
    if (rc) return rc;
    if (!(lr > 0.f) || std::isinf(lr)) return fail(HPC_ERR_INVALID_ARG, "hpc_setenc_adam: lr");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    model->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = (float)(1.0 - std::pow(0.9, (double)model->step));
    const float c2 = (float)(1.0 - std::pow(0.999, (double)model->step));
    hipLaunchKernelGGL(enc::k_adam, dim3(512), dim3(256), 0, st, model->theta,
                       (const float*)model->grad, model->m1, model->m2, (int64_t)model->L.total,
                       lr, b1, b2, 1e-8f, c1, c2);
    HPC_HIP(hipGetLastError());
    return swizzle(model, st);
}

int hpc_learned_seed(hpc_setenc model, const float* X, int64_t m, const int64_t* idx,
                     int64_t idx_len, const hpc_sample_desc* desc, int32_t n_samples, float* C,
                     float* C_kpp, int64_t c_len, int32_t precision, double* f_prop,
                     double* f_kpp, int32_t* accepted, void* hip_stream) {
    int rc = check_model(model, "hpc_learned_seed");
    if (rc) return rc;
    if (!C_kpp || !f_prop || !f_kpp)
        return fail(HPC_ERR_INVALID_ARG, "hpc_learned_seed: NULL C_kpp / f_prop / f_kpp");
    rc = hpc_setenc_propose(model, X, m, idx, idx_len, desc, n_samples, C, c_len, hip_stream);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    hipLaunchKernelGGL(k_fill_f32, dim3(256), dim3(256), 0, st, C_kpp, c_len, __builtin_nanf(""));
    HPC_HIP(hipGetLastError());
    // one pass from all-degenerate rows = the K-means++ seeding of a cold
    // start (re-seeding stream, pass 0) and the objective of that seeding
    rc = hpc_lloyd_batch(X, m, model->d, idx, idx_len, desc, n_samples, C_kpp, c_len, 1, 0.0,
                         precision, f_kpp, model->its, nullptr, hip_stream);
    if (rc) return rc;
    // one pass from the proposal = its objective (centroids unchanged)
    rc = hpc_lloyd_batch(X, m, model->d, idx, idx_len, desc, n_samples, C, c_len, 1, 0.0,
                         precision, f_prop, model->its, nullptr, hip_stream);
    if (rc) return rc;
    hipLaunchKernelGGL(k_select_init, dim3(n_samples), dim3(256), 0, st,
                       (const hpc_sample_desc*)model->desc_dev, model->kd, (const double*)f_prop,
                       (const double*)f_kpp, (const float*)C_kpp, C, accepted);
    HPC_HIP(hipGetLastError());
    return HPC_OK;
}

}  // extern "C"

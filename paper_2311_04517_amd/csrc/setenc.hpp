// Learned initializer: a set encoder that proposes the k starting centroids
// of a sample from the sample itself (the alternative to the K-means++
// seeding of Section 3; it is used only where its sample objective is no
// larger than the seeding's).
//
//   x~ = (x - mu) / sigma                    (per-sample normalisation)
//   h1 = relu(x~ W1 + b1)   d -> 256         (per point)
//   h2 = relu(h1 W2 + b2)   256 -> 256       (per point)
//   p  = mean over points of h2
//   o  = p Wh + bh          256 -> k*d       (head)
//   P  = mu + sigma * reshape(o, k, d)
//
// Per-point layers run on the matrix cores (MFMA 16x16x32 BF16, FP32
// accumulate) in transposed form: a wave computes Z^T = W^T X^T for 16
// points, so the feature index runs down the MFMA rows and the point index
// across the columns.  The D layout of a 16x16 output block gives lane l
// features 4(l/16)+r, r < 4, of point l%16 -- exactly the values that lane
// must supply as the B operand of the next layer if that layer's K order is
// permuted accordingly (kperm below).  The weight tables are stored
// pre-permuted, so activations never leave the registers between layers.
//
// Weights are BF16 for the matrix cores (the head uses the BF16-rounded
// values in FP32 arithmetic); biases, accumulators, pooled features,
// gradients and the Adam state are FP32.
#pragma once

#include "common.hpp"
#include "mfma_screen.hpp"

namespace hpc {
namespace enc {

constexpr int H = 256;       // hidden width
constexpr int NMB = H / 16;  // 16-row output blocks of a hidden layer
constexpr int NKB = H / 32;  // 32-wide K blocks of a hidden layer
constexpr int DIN = 32;      // padded input width (one K block)
constexpr int NT = 256;      // threads per workgroup of the row kernels
constexpr int TPW = 4;       // 16-point tiles per wave
constexpr int CH = NT / kWave * TPW * 16;  // points per workgroup (256)

// Input feature of K position (g, v) of a 32-wide K block: the first four
// come from the lower 16-feature output block, the last four from the upper.
__host__ __device__ inline int kperm(int g, int v) {
    return v < 4 ? 4 * g + v : 16 + 4 * g + (v - 4);
}

// Offsets of the parameters in the flat FP32 vector (order W1, b1, W2, b2,
// Wh, bh; matrices row-major, W1 is d x H, W2 H x H, Wh H x kd).
struct Layout {
    int64_t W1, b1, W2, b2, Wh, bh, total;
    __host__ __device__ static Layout of(int d, int kd) {
        Layout L{};
        L.W1 = 0;
        L.b1 = L.W1 + (int64_t)d * H;
        L.W2 = L.b1 + H;
        L.b2 = L.W2 + (int64_t)H * H;
        L.Wh = L.b2 + H;
        L.bh = L.Wh + (int64_t)H * kd;
        L.total = L.bh + kd;
        return L;
    }
};

struct RowArgs {
    const float* X;
    int64_t m;
    int32_t d;
    const int64_t* idx;
    const hpc_sample_desc* desc;
    int32_t n_enc;
    const float* stats;  // [b][DIN + 2]: mu, sigma, 1/sigma
    const bf16x8* W1s;   // [NMB][64]
    const bf16x8* W2Ts;  // [NMB][NKB][64]
    const bf16x8* W2s;   // [NMB][NKB][64]
    const float* b1;
    const float* b2;
    float* pooled_part;  // forward: [b][chunk][H]
    int32_t chunks;
    const float* g2;     // backward: [b][H], dL/dp / n_b
    float* sX;           // backward scratch, row b * n_enc + i: [.][DIN]
    float* sH1;          // [.][H]
    float* sG2;          // [.][H]
    float* sG1;          // [.][H]
};

__device__ __forceinline__ int n_points(const hpc_sample_desc& ds, int n_enc) {
    return ds.s < n_enc ? ds.s : n_enc;
}

// ---------------------------------------------------------------------------
// Per-sample normalisation: mu = mean of the encoder's points (the first
// n_b = min(s, n_enc) points of the sample), sigma = sqrt(mean |x - mu|^2)
// (1 if zero).  FP64 sums.  One workgroup per sample.
// ---------------------------------------------------------------------------
// An index outside [0, m) reads as a row of zeros (as in the Lloyd gather).
__device__ __forceinline__ float enc_coord(const float* __restrict__ X, int64_t m, int32_t d,
                                          int64_t row, int q) {
    return (row >= 0 && row < m) ? X[row * d + q] : 0.f;
}

__global__ __launch_bounds__(NT) void k_enc_stats(const float* __restrict__ X, int64_t m,
                                                  int32_t d, const int64_t* __restrict__ idx,
                                                  const hpc_sample_desc* __restrict__ desc,
                                                  int32_t n_enc, float* __restrict__ stats) {
    __shared__ double red[NT / kWave];
    __shared__ double mu[DIN];
    const hpc_sample_desc ds = desc[blockIdx.x];
    const int n = n_points(ds, n_enc);
    for (int q = 0; q < d; ++q) {
        double a = 0.0;
        for (int i = threadIdx.x; i < n; i += NT)
            a += (double)enc_coord(X, m, d, idx[ds.idx_offset + i], q);
        a = block_sum<NT>(a, red);
        if (threadIdx.x == 0) mu[q] = a / n;
    }
    __syncthreads();
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += NT) {
        const int64_t row = idx[ds.idx_offset + i];
        for (int q = 0; q < d; ++q) {
            const double e = (double)enc_coord(X, m, d, row, q) - mu[q];
            v = __fma_rn(e, e, v);
        }
    }
    v = block_sum<NT>(v, red);
    if (threadIdx.x == 0) {
        double sg = sqrt(v / n);
        if (!(sg > 0.0)) sg = 1.0;
        float* st = stats + (size_t)blockIdx.x * (DIN + 2);
        for (int q = 0; q < DIN; ++q) st[q] = q < d ? (float)mu[q] : 0.f;
        st[DIN] = (float)sg;
        st[DIN + 1] = (float)(1.0 / sg);
    }
}

// ---------------------------------------------------------------------------
// Operand tables from the FP32 master weights (BF16, pre-permuted) and the
// BF16-rounded head weights used by the FP32 head.
// ---------------------------------------------------------------------------
__global__ void k_enc_swizzle(const float* __restrict__ theta, int32_t d, int32_t kd,
                              bf16x8* __restrict__ W1s, bf16x8* __restrict__ W2Ts,
                              bf16x8* __restrict__ W2s, float* __restrict__ Whr) {
    const Layout L = Layout::of(d, kd);
    const int64_t n1 = (int64_t)NMB * 64, n2 = (int64_t)NMB * NKB * 64, nh = (int64_t)H * kd;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n1 + 2 * n2 + nh;
         e += (int64_t)gridDim.x * blockDim.x) {
        if (e < n1) {
            const int mb = (int)(e / 64), lane = (int)(e % 64), g = lane >> 4;
            const int col = 16 * mb + (lane & 15);
            bf16x8 v;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int row = 8 * g + t;
                v[t] = (__bf16)(row < d ? theta[L.W1 + (int64_t)row * H + col] : 0.f);
            }
            W1s[e] = v;
        } else if (e < n1 + 2 * n2) {
            const bool tr = e < n1 + n2;
            const int64_t f = tr ? e - n1 : e - n1 - n2;
            const int mb = (int)(f / (NKB * 64)), kb = (int)((f / 64) % NKB), lane = (int)(f % 64);
            const int g = lane >> 4, mrow = 16 * mb + (lane & 15);
            bf16x8 v;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int kk = 32 * kb + kperm(g, t);
                // W2T operand: element (mrow = output feature, kk = input feature)
                // W2  operand: element (mrow = input feature,  kk = output feature)
                const float w = tr ? theta[L.W2 + (int64_t)kk * H + mrow]
                                   : theta[L.W2 + (int64_t)mrow * H + kk];
                v[t] = (__bf16)w;
            }
            (tr ? W2Ts : W2s)[f] = v;
        } else {
            const int64_t f = e - n1 - 2 * n2;
            Whr[f] = (float)(__bf16)theta[L.Wh + f];
        }
    }
}

// ---------------------------------------------------------------------------
// The per-point layers over one chunk of CH points of one sample
// (grid: x = chunk, y = sample).  Forward: partial sums of h2 per chunk.
// Backward (BWD): recompute the forward, then dz2 = g2 * [z2 > 0],
// dh1^T = W2 dz2^T, dz1 = dh1 * [z1 > 0]; the rows x~, h1, dz2, dz1 go to
// scratch for the weight-gradient products (zero rows past the sample).
// ---------------------------------------------------------------------------
template <bool BWD>
__global__ __launch_bounds__(NT) void k_enc_rows(RowArgs a) {
    __shared__ float wsum[NT / kWave][H];
    const int b = blockIdx.y, c = blockIdx.x;
    const hpc_sample_desc ds = a.desc[b];
    const int n = n_points(ds, a.n_enc);
    const int lane = threadIdx.x & 63, wid = threadIdx.x / kWave, g = lane >> 4, pl = lane & 15;
    const float* st = a.stats + (size_t)b * (DIN + 2);
    const float inv_sigma = st[DIN + 1];
    float pool[NMB][4];
#pragma unroll
    for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
        for (int r = 0; r < 4; ++r) pool[mb][r] = 0.f;

    for (int t = 0; t < TPW; ++t) {
        const int p = c * CH + (wid * TPW + t) * 16 + pl;
        if (c * CH + (wid * TPW + t) * 16 >= a.n_enc) break;  // wave-uniform
        const bool valid = p < n;
        // B operand of layer 1: dims 8g..8g+7 of this lane's point
        bf16x8 xop;
        {
            const int64_t xr = valid ? a.idx[ds.idx_offset + p] : -1;
#pragma unroll
            for (int v = 0; v < 8; ++v) {
                const int q = 8 * g + v;
                const float xv =
                    (valid && q < a.d) ? (enc_coord(a.X, a.m, a.d, xr, q) - st[q]) * inv_sigma : 0.f;
                xop[v] = (__bf16)xv;
            }
        }
        const int64_t row = (int64_t)b * a.n_enc + p;
        if constexpr (BWD) {
            float4 lo, hi;
            lo.x = (float)xop[0]; lo.y = (float)xop[1]; lo.z = (float)xop[2]; lo.w = (float)xop[3];
            hi.x = (float)xop[4]; hi.y = (float)xop[5]; hi.z = (float)xop[6]; hi.w = (float)xop[7];
            if (p < a.n_enc) {
                *reinterpret_cast<float4*>(a.sX + row * DIN + 8 * g) = lo;
                *reinterpret_cast<float4*>(a.sX + row * DIN + 8 * g + 4) = hi;
            }
        }
        // layer 1: h1 as layer-2 B operands, and the signs of z1
        bf16x8 hop[NKB];
        uint64_t m1 = 0;
#pragma unroll
        for (int mb = 0; mb < NMB; ++mb) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.W1s[mb * 64 + lane], xop, acc, 0, 0, 0);
            float hv[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float z = acc[r] + a.b1[16 * mb + 4 * g + r];
                m1 |= (uint64_t)(z > 0.f) << (mb * 4 + r);
                const __bf16 hb = (__bf16)(valid && z > 0.f ? z : 0.f);
                hop[mb >> 1][(mb & 1) * 4 + r] = hb;
                hv[r] = (float)hb;
            }
            if constexpr (BWD) {
                if (p < a.n_enc)
                    *reinterpret_cast<float4*>(a.sH1 + row * H + 16 * mb + 4 * g) =
                        make_float4(hv[0], hv[1], hv[2], hv[3]);
            }
        }
        // layer 2
        bf16x8 dzop[NKB];
#pragma unroll
        for (int mb = 0; mb < NMB; ++mb) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < NKB; ++kb)
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.W2Ts[(mb * NKB + kb) * 64 + lane],
                                                              hop[kb], acc, 0, 0, 0);
            float dv[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int f = 16 * mb + 4 * g + r;
                const float z = acc[r] + a.b2[f];
                if constexpr (BWD) {
                    const __bf16 db = (__bf16)(valid && z > 0.f ? a.g2[(size_t)b * H + f] : 0.f);
                    dzop[mb >> 1][(mb & 1) * 4 + r] = db;
                    dv[r] = (float)db;
                } else {
                    pool[mb][r] += valid && z > 0.f ? z : 0.f;
                }
            }
            if constexpr (BWD) {
                if (p < a.n_enc)
                    *reinterpret_cast<float4*>(a.sG2 + row * H + 16 * mb + 4 * g) =
                        make_float4(dv[0], dv[1], dv[2], dv[3]);
            }
        }
        if constexpr (BWD) {
            // dh1^T = W2 dz2^T, masked by the signs of z1
#pragma unroll
            for (int ma = 0; ma < NMB; ++ma) {
                f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kb = 0; kb < NKB; ++kb)
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        a.W2s[(ma * NKB + kb) * 64 + lane], dzop[kb], acc, 0, 0, 0);
                float gv[4];
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    gv[r] = (valid && ((m1 >> (ma * 4 + r)) & 1)) ? acc[r] : 0.f;
                if (p < a.n_enc)
                    *reinterpret_cast<float4*>(a.sG1 + row * H + 16 * ma + 4 * g) =
                        make_float4(gv[0], gv[1], gv[2], gv[3]);
            }
        }
    }
    if constexpr (!BWD) {
        // sum over the 16 points of each lane group, then over the waves
#pragma unroll
        for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float v = pool[mb][r];
#pragma unroll
                for (int o = 1; o < 16; o <<= 1) v += __shfl_xor(v, o, 16);
                if (pl == 0) wsum[wid][16 * mb + 4 * g + r] = v;
            }
        __syncthreads();
        for (int f = threadIdx.x; f < H; f += NT) {
            float v = 0.f;
#pragma unroll
            for (int w = 0; w < NT / kWave; ++w) v += wsum[w][f];
            a.pooled_part[((size_t)b * a.chunks + c) * H + f] = v;
        }
    }
}

// pooled[b][f] = (sum over chunks) / n_b.  grid = samples.
__global__ void k_enc_pool(const float* __restrict__ part, int32_t chunks,
                           const hpc_sample_desc* __restrict__ desc, int32_t n_enc,
                           float* __restrict__ pooled) {
    const int b = blockIdx.x;
    const int n = n_points(desc[b], n_enc);
    for (int f = threadIdx.x; f < H; f += blockDim.x) {
        float v = 0.f;
        for (int c = 0; c < chunks; ++c) v += part[((size_t)b * chunks + c) * H + f];
        pooled[(size_t)b * H + f] = v / (float)n;
    }
}

// Head: o[b][j] = pooled[b] . Whr[:, j] + bh[j]; proposal row j / d, column
// j % d = mu + sigma * o, written at C + desc[b].c_offset (nullable C).
// grid: x = blocks of 256 outputs, y = sample.
__global__ void k_enc_head(const float* __restrict__ pooled, const float* __restrict__ Whr,
                           const float* __restrict__ bh, int32_t kd, int32_t d,
                           const float* __restrict__ stats, const hpc_sample_desc* __restrict__ desc,
                           float* __restrict__ obuf, float* __restrict__ C) {
    const int b = blockIdx.y;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= kd) return;
    const float* p = pooled + (size_t)b * H;
    float o = bh[j];
    for (int f = 0; f < H; ++f) o = __fmaf_rn(p[f], Whr[(size_t)f * kd + j], o);
    obuf[(size_t)b * kd + j] = o;
    if (C) {
        const float* st = stats + (size_t)b * (DIN + 2);
        C[desc[b].c_offset + j] = st[j % d] + st[DIN] * o;
    }
}

// Matching loss of a sample in normalised coordinates and its gradient
// dL/do / B.  The pairing is greedy and one-to-one: k times, the closest
// (proposal j, target l) pair among the rows not yet paired is taken (FP64
// squared distances; ties to the lowest j, then the lowest l).  Loss
// (1/k) sum_j |o_j - T~_pi(j)|^2.  One workgroup of 256 per sample; k <= 64.
// loss_part[b] = the sample's loss / B.
__global__ __launch_bounds__(256) void k_enc_loss(const float* __restrict__ obuf,
                                                  const float* __restrict__ T,
                                                  const float* __restrict__ stats,
                                                  const hpc_sample_desc* __restrict__ desc,
                                                  int32_t k, int32_t d, int32_t B,
                                                  float* __restrict__ dout,
                                                  double* __restrict__ loss_part) {
    __shared__ double Dm[64 * 64];
    __shared__ int pi[64];
    __shared__ unsigned char free_j[64], free_l[64];
    __shared__ double wv[4];
    __shared__ int wi[4];
    const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const hpc_sample_desc ds = desc[b];
    const float* st = stats + (size_t)b * (DIN + 2);
    const float* o = obuf + (size_t)b * k * d;
    const float* t = T + ds.c_offset;
    const double inv = 1.0 / (double)st[DIN];
    for (int e = tid; e < k * k; e += blockDim.x) {
        const int j = e / k, l = e % k;
        double s = 0.0;
        for (int q = 0; q < d; ++q) {
            const double tn = ((double)t[l * d + q] - (double)st[q]) * inv;
            const double df = (double)o[j * d + q] - tn;
            s = __fma_rn(df, df, s);
        }
        Dm[e] = s;
    }
    if (tid < 64) {
        free_j[tid] = 1;
        free_l[tid] = 1;
    }
    __syncthreads();
    for (int step = 0; step < k; ++step) {
        double v = __builtin_huge_val();
        int ix = 0x7fffffff;
        for (int e = tid; e < k * k; e += blockDim.x)
            if (free_j[e / k] && free_l[e % k] && (Dm[e] < v || (Dm[e] == v && e < ix))) {
                v = Dm[e];
                ix = e;
            }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double ov = __shfl_xor(v, off, 64);
            const int oi = __shfl_xor(ix, off, 64);
            if (ov < v || (ov == v && oi < ix)) {
                v = ov;
                ix = oi;
            }
        }
        if (lane == 0) {
            wv[w] = v;
            wi[w] = ix;
        }
        __syncthreads();
        if (tid == 0) {
            double bv = wv[0];
            int bi = wi[0];
            for (int q = 1; q < 4; ++q)
                if (wv[q] < bv || (wv[q] == bv && wi[q] < bi)) {
                    bv = wv[q];
                    bi = wi[q];
                }
            pi[bi / k] = bi % k;
            free_j[bi / k] = 0;
            free_l[bi % k] = 0;
        }
        __syncthreads();
    }
    double acc = tid < k ? Dm[tid * k + pi[tid]] : 0.0;
    acc = block_sum<256>(acc, wv);
    if (tid == 0) loss_part[b] = acc / k / B;
    for (int e = tid; e < k * d; e += blockDim.x) {
        const int j = e / d, q = e % d;
        const double tn = ((double)t[pi[j] * d + q] - (double)st[q]) * inv;
        dout[(size_t)b * k * d + e] = (float)(2.0 * ((double)o[e] - tn) / k / B);
    }
}

// Head backward.  dWh[f][j] = sum_b pooled[b][f] dout[b][j]; dbh[j] =
// sum_b dout[b][j] (row f == H).  grid: x = blocks of j, y = f in [0, H].
__global__ void k_enc_head_wgrad(const float* __restrict__ pooled, const float* __restrict__ dout,
                                 int32_t B, int32_t kd, float* __restrict__ gWh,
                                 float* __restrict__ gbh) {
    const int f = blockIdx.y;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= kd) return;
    float s = 0.f;
    for (int b = 0; b < B; ++b)
        s = __fmaf_rn(f < H ? pooled[(size_t)b * H + f] : 1.f, dout[(size_t)b * kd + j], s);
    if (f < H)
        gWh[(size_t)f * kd + j] = s;
    else
        gbh[j] = s;
}

// g2[b][f] = (sum_j Whr[f][j] dout[b][j]) / n_b: the gradient reaching
// each point's h2 through the mean.  grid = samples, H threads.
__global__ __launch_bounds__(H) void k_enc_head_dp(const float* __restrict__ Whr,
                                                   const float* __restrict__ dout, int32_t kd,
                                                   const hpc_sample_desc* __restrict__ desc,
                                                   int32_t n_enc, float* __restrict__ g2) {
    __shared__ float dj[256];
    const int b = blockIdx.x, f = threadIdx.x;
    float s = 0.f;
    for (int j0 = 0; j0 < kd; j0 += 256) {
        __syncthreads();
        if (j0 + f < kd) dj[f] = dout[(size_t)b * kd + j0 + f];
        __syncthreads();
        const int nj = kd - j0 < 256 ? kd - j0 : 256;
        for (int jj = 0; jj < nj; ++jj) s = __fmaf_rn(Whr[(size_t)f * kd + j0 + jj], dj[jj], s);
    }
    g2[(size_t)b * H + f] = s / (float)n_points(desc[b], n_enc);
}

// ---------------------------------------------------------------------------
// Weight gradient C = A^T B over P rows (A: P x lda, its first M columns;
// B: P x N, row stride ldb) on the matrix cores: the operands are rounded
// to BF16 (as the forward's are), products accumulate in FP32.  One
// workgroup of four waves per 64 x 64 output tile, each wave a 32 x 32
// quarter (2 x 2 blocks of v_mfma_f32_16x16x32_bf16).  The contraction runs
// over the rows p: per stage 128 rows of A's and B's 64 columns go to LDS
// transposed (column-major, p contiguous), so that a lane's eight K values
// of the MFMA operand (rows 8g .. 8g+7 of its column, g = lane / 16) are one
// 16-byte read.  Split over P (grid.z), each split writing its own partial
// [z][M][N].
// ---------------------------------------------------------------------------
constexpr int WG_ROWS = 128;              // rows of p per LDS stage
constexpr int WG_PAD = WG_ROWS + 8;       // LDS column stride (BF16): 272 B

__global__ __launch_bounds__(256) void k_wgrad(const float* __restrict__ A, int32_t lda, int32_t M,
                                               const float* __restrict__ Bm, int32_t ldb, int32_t N,
                                               int64_t P, int64_t per_split,
                                               float* __restrict__ part) {
    __shared__ __align__(16) __bf16 As[64 * WG_PAD];
    __shared__ __align__(16) __bf16 Bs[64 * WG_PAD];
    const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
    const int64_t p0 = blockIdx.z * per_split;
    const int64_t p1 = p0 + per_split < P ? p0 + per_split : P;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;  // this wave's quarter
    const int col = lane & 15, g = lane >> 4;
    // staging: thread (c, q) moves column c of rows 2i, 2i + 1 for i in
    // [16q, 16q + 16), two BF16 per 32-bit LDS store
    const int c = tid & 63, q = tid >> 6;
    const bool a_ok = m0 + c < M, b_ok = n0 + c < N;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int64_t pb = p0; pb < p1; pb += WG_ROWS) {
        float av[32], bv[32];
#pragma unroll
        for (int u = 0; u < 32; ++u) {
            const int64_t p = pb + 32 * q + u;
            av[u] = (p < p1 && a_ok) ? A[p * lda + m0 + c] : 0.f;
            bv[u] = (p < p1 && b_ok) ? Bm[p * ldb + n0 + c] : 0.f;
        }
        __syncthreads();  // the previous stage's operand reads are done
#pragma unroll
        for (int u = 0; u < 32; u += 2) {
            const int r = 32 * q + u;
            __bf16 pa[2] = {(__bf16)av[u], (__bf16)av[u + 1]};
            __bf16 pbv[2] = {(__bf16)bv[u], (__bf16)bv[u + 1]};
            *reinterpret_cast<uint32_t*>(&As[c * WG_PAD + r]) = *reinterpret_cast<uint32_t*>(pa);
            *reinterpret_cast<uint32_t*>(&Bs[c * WG_PAD + r]) = *reinterpret_cast<uint32_t*>(pbv);
        }
        __syncthreads();
#pragma unroll
        for (int kb = 0; kb < WG_ROWS; kb += 32) {
            bf16x8 ao[2], bo[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                ao[i] = *reinterpret_cast<const bf16x8*>(&As[(wm + 16 * i + col) * WG_PAD + kb + 8 * g]);
                bo[i] = *reinterpret_cast<const bf16x8*>(&Bs[(wn + 16 * i + col) * WG_PAD + kb + 8 * g]);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ao[i], bo[j], acc[i][j], 0, 0, 0);
        }
    }
    // lane (col, g) holds rows 4g .. 4g + 3 of column col of each block
    float* out = part + (size_t)blockIdx.z * M * N;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int mm = m0 + wm + 16 * i + 4 * g + r, nn = n0 + wn + 16 * j + col;
                if (mm < M && nn < N) out[(size_t)mm * N + nn] = acc[i][j][r];
            }
}

// Column sums of B (P x N, stride ldb), split over P: part[z][N].  Four
// rows per step with independent partial sums, so four loads are in flight
// per thread.
__global__ void k_colsum(const float* __restrict__ Bm, int32_t ldb, int32_t N, int64_t P,
                         int64_t per_split, float* __restrict__ part) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int64_t p0 = blockIdx.y * per_split;
    const int64_t p1 = p0 + per_split < P ? p0 + per_split : P;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    int64_t p = p0;
    for (; p + 4 <= p1; p += 4) {
        s0 += Bm[p * ldb + n];
        s1 += Bm[(p + 1) * ldb + n];
        s2 += Bm[(p + 2) * ldb + n];
        s3 += Bm[(p + 3) * ldb + n];
    }
    for (; p < p1; ++p) s0 += Bm[p * ldb + n];
    part[(size_t)blockIdx.y * N + n] = (s0 + s1) + (s2 + s3);
}

// out[e] = sum over splits of part[z][e] (fixed order).
__global__ void k_sum_splits(const float* __restrict__ part, int32_t splits, int64_t n,
                             float* __restrict__ out) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int z = 0; z < splits; ++z) s += part[(size_t)z * n + e];
        out[e] = s;
    }
}

// Adam (Kingma & Ba, ICLR 2015) on the FP32 master parameters.
__global__ void k_adam(float* __restrict__ theta, const float* __restrict__ grad,
                       float* __restrict__ m1, float* __restrict__ m2, int64_t n, float lr,
                       float beta1, float beta2, float eps, float c1, float c2) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x) {
        const float gr = grad[e];
        const float a = beta1 * m1[e] + (1.f - beta1) * gr;
        const float v = beta2 * m2[e] + (1.f - beta2) * gr * gr;
        m1[e] = a;
        m2[e] = v;
        theta[e] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
    }
}

// He-uniform initial weights from Philox (tag 4, counter (e/4, 0, 0, 0)):
// W ~ U(-a, a), a = sqrt(6 / fan_in) for W1, W2; a = sqrt(3 / H) / 4 for
// the head; biases 0.01 (hidden) and 0 (head).
__global__ void k_enc_init(float* __restrict__ theta, int32_t d, int32_t kd, uint64_t seed) {
    const Layout L = Layout::of(d, kd);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < L.total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const Words4 w = philox_block(seed, 4, (uint64_t)(e / 4), 0, 0);
        const double u = 2.0 * unit_double(w.w[e % 4]) - 1.0;
        float v;
        if (e < L.b1)
            v = (float)(u * sqrt(6.0 / d));
        else if (e < L.W2)
            v = 0.01f;
        else if (e < L.b2)
            v = (float)(u * sqrt(6.0 / H));
        else if (e < L.Wh)
            v = 0.01f;
        else if (e < L.bh)
            v = (float)(u * sqrt(3.0 / H) * 0.25);
        else
            v = 0.f;
        theta[e] = v;
    }
}

}  // namespace enc
}  // namespace hpc

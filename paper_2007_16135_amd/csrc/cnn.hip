// cnn.hip -- the k-NN embedding network on gfx950.
//
// Every convolution is an implicit GEMM on the BF16 matrix cores (FP32
// accumulation): the A operand is read straight from the packed activations
// with the tap shift applied per element and zeroed outside the row's own
// series, so no im2col buffer is ever written.  Series are packed back to
// back (row r = sample t of series s); a per-row word holds (t, L).
//
//   forward  y_l   = conv(h_l; W_l) + b_l      A = h_l (kAConv),  B = W_l^T
//   weights  dW_l  = sum_r h_l[r+tap-2] dy_l[r] A = h_l (kAConvT), B = dy_l, split-K
//   data     dh_l  = conv(dy_l; flip(W_l)^T) * [h_l > 0]
//
// Masters are FP32; the operand copies of the weights are rebuilt in BF16
// at the start of every call.
#include "cnn_kernels.h"

#include <stdint.h>

namespace twed {
namespace cnn {

typedef __attribute__((ext_vector_type(4))) short bf16x4;
typedef __attribute__((ext_vector_type(4))) float f32x4;

__device__ __forceinline__ uint16_t to_bf16(float f)
{
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest, ties to even
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float from_bf16(uint16_t h) { return __builtin_bit_cast(float, (uint32_t)h << 16); }

__device__ __forceinline__ int row_t(uint32_t info) { return (int)(info & 0xffffu); }
__device__ __forceinline__ int row_L(uint32_t info) { return (int)(info >> 16); }

// ---- GEMM ------------------------------------------------------------------------
//
// One wave computes a 64x64 tile of C as 4x4 blocks of v_mfma_f32_16x16x16_bf16.
// Fragment layout of that instruction on a 64-wide wave: A[i][k] sits in
// lane i + 16*(k/4), element k%4; B[k][j] in lane j + 16*(k/4), element k%4;
// the result C[i][j] in lane j + 16*(i/4), element i%4.  Each lane therefore
// loads four consecutive k of one A row and of one B column per step.

// Four consecutive k of A row m, k >= kk, zero at or beyond kend.
template <int AM>
__device__ __forceinline__ bf16x4 load_a(const GemmArgs &g, int m, int kk, int kend)
{
    bf16x4 v = bf16x4{0, 0, 0, 0};
    if (m >= g.M) return v;
    if constexpr (AM == kAPlain) {
        const uint16_t *p = g.A + (int64_t)m * g.lda_m;
        if (g.lda_k == 1 && (g.lda_m & 3) == 0 && kk + 3 < kend) {
            v = __builtin_bit_cast(bf16x4, *reinterpret_cast<const uint2 *>(p + kk));
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (kk + e < kend) v[e] = (short)p[(int64_t)(kk + e) * g.lda_k];
        }
    } else if constexpr (AM == kAConv) {
        const int C = g.conv_C;
        const uint32_t info = g.row_info[m];
        const int t = row_t(info), L = row_L(info);
        if ((C & 3) == 0 && kk + 3 < kend) {
            const int tap = kk / C, c = kk - tap * C;
            const int ts = t + tap - kKsize / 2;
            const int src = m + tap - kKsize / 2;
            if (ts >= 0 && ts < L && src >= 0 && src < g.M)
                v = __builtin_bit_cast(bf16x4, *reinterpret_cast<const uint2 *>(g.A + (int64_t)src * C + c));
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int k = kk + e;
                if (k >= kend) continue;
                const int tap = k / C, c = k - tap * C;
                const int ts = t + tap - kKsize / 2;
                const int src = m + tap - kKsize / 2;
                if (ts >= 0 && ts < L && src >= 0 && src < g.M) v[e] = (short)g.A[(int64_t)src * C + c];
            }
        }
    } else {  // kAConvT: row m = (tap, c), k = packed row
        const int C = g.conv_C;
        const int tap = m / C, c = m - (m / C) * C;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int r = kk + e;
            if (r >= kend) continue;
            const uint32_t info = g.row_info[r];
            const int ts = row_t(info) + tap - kKsize / 2;
            const int src = r + tap - kKsize / 2;
            if (ts >= 0 && ts < row_L(info) && src >= 0 && src < g.K)
                v[e] = (short)g.A[(int64_t)src * C + c];
        }
    }
    return v;
}

// Four consecutive k of B column n.
__device__ __forceinline__ bf16x4 load_b(const GemmArgs &g, int n, int kk, int kend)
{
    bf16x4 v = bf16x4{0, 0, 0, 0};
    if (n >= g.N) return v;
    const uint16_t *p = g.B + (int64_t)n * g.ldb_n;
    if (g.ldb_k == 1 && (g.ldb_n & 3) == 0 && kk + 3 < kend) {
        v = __builtin_bit_cast(bf16x4, *reinterpret_cast<const uint2 *>(p + kk));
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (kk + e < kend) v[e] = (short)p[(int64_t)(kk + e) * g.ldb_k];
    }
    return v;
}

template <int AM, int OM>
__global__ __launch_bounds__(64) void gemm_kernel(GemmArgs g, int kchunk)
{
    const int lane = threadIdx.x;
    const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
    const int kbeg = blockIdx.z * kchunk;
    const int kend = kbeg + kchunk < g.K ? kbeg + kchunk : g.K;
    const int li = lane & 15, lk = (lane >> 4) * 4;

    f32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = kbeg; k0 < kend; k0 += 16) {
        const int kk = k0 + lk;
        bf16x4 a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = load_a<AM>(g, m0 + 16 * i + li, kk, kend);
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = load_b(g, n0 + 16 * j + li, kk, kend);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
    }

#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int m = m0 + 16 * i + (lane >> 4) * 4 + e;
            if (m >= g.M) continue;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int n = n0 + 16 * j + li;
                if (n >= g.N) continue;
                float v = acc[i][j][e];
                const int64_t at = (int64_t)m * g.ldc + n;
                if constexpr (OM == kOutAtomic) {
                    atomicAdd((float *)g.C + at, v);
                } else if constexpr (OM == kOutDist) {
                    ((float *)g.C)[at] = g.row_norm[m] + g.col_norm[n] - 2.0f * v;
                } else {
                    if (g.bias) v += g.bias[n];
                    if (g.relu) v = v > 0.f ? v : 0.f;
                    if constexpr (OM == kOutF32) {
                        ((float *)g.C)[at] = v;
                    } else {
                        if (g.mask && !(from_bf16(g.mask[at]) > 0.f)) v = 0.f;
                        ((uint16_t *)g.C)[at] = to_bf16(v);
                    }
                }
            }
        }
    }
}

template <int AM>
static hipError_t gemm_by_out(int out_mode, const GemmArgs &g, dim3 grid, int kchunk, hipStream_t st)
{
    switch (out_mode) {
    case kOutF32: hipLaunchKernelGGL((gemm_kernel<AM, kOutF32>), grid, dim3(64), 0, st, g, kchunk); break;
    case kOutBF16: hipLaunchKernelGGL((gemm_kernel<AM, kOutBF16>), grid, dim3(64), 0, st, g, kchunk); break;
    case kOutAtomic: hipLaunchKernelGGL((gemm_kernel<AM, kOutAtomic>), grid, dim3(64), 0, st, g, kchunk); break;
    case kOutDist: hipLaunchKernelGGL((gemm_kernel<AM, kOutDist>), grid, dim3(64), 0, st, g, kchunk); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_gemm(int out_mode, const GemmArgs &g, int splitk, hipStream_t st)
{
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    if (splitk < 1) splitk = 1;
    int kchunk = (g.K + splitk - 1) / splitk;
    kchunk = (kchunk + 15) / 16 * 16;  // whole MFMA steps per chunk
    if (kchunk < 16) kchunk = 16;
    const int zs = (g.K + kchunk - 1) / kchunk;
    dim3 grid((g.M + 63) / 64, (g.N + 63) / 64, zs < 1 ? 1 : zs);
    switch (g.a_mode) {
    case kAPlain: return gemm_by_out<kAPlain>(out_mode, g, grid, kchunk, st);
    case kAConv: return gemm_by_out<kAConv>(out_mode, g, grid, kchunk, st);
    case kAConvT: return gemm_by_out<kAConvT>(out_mode, g, grid, kchunk, st);
    default: return hipErrorInvalidValue;
    }
}

// ---- network pieces ------------------------------------------------------------------

// Row words (t, L), owning series and layer-1 features (x/8, L/256).
// Sample t of series s is X[off[s] + t] and packed row off[s] - row_base + t.
__global__ void features_kernel(const float *__restrict__ X, const int64_t *__restrict__ off, int nSeries,
                                int64_t row_base, int64_t R, uint32_t *__restrict__ row_info,
                                int32_t *__restrict__ row_series, uint16_t *__restrict__ feat)
{
    for (int s = blockIdx.y; s < nSeries; s += gridDim.y) {
        const int64_t b = off[s];
        const int L = (int)(off[s + 1] - b);
        for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < L; t += gridDim.x * blockDim.x) {
            const int64_t r = b - row_base + t;
            if (r < 0 || r >= R) break;  // offsets inconsistent with the chunk: write nothing
            row_info[r] = (uint32_t)t | ((uint32_t)L << 16);
            if (row_series) row_series[r] = s;
            feat[2 * r + 0] = to_bf16(X[b + t] * kXScale);
            feat[2 * r + 1] = to_bf16((float)L * kLScale);
        }
    }
}

// Segment means of layer 4 -> embedding (f32 and/or bf16) and the squared
// norm of the bf16 embedding.  One 128-thread block per series.
__global__ __launch_bounds__(128) void pool_kernel(const float *__restrict__ y4, const int64_t *__restrict__ off,
                                                   int nSeries, int64_t row_base, int64_t R,
                                                   float *__restrict__ emb, uint16_t *__restrict__ emb16,
                                                   float *__restrict__ sqnorm)
{
    __shared__ float part[2];
    const int s = blockIdx.x;
    const int q = threadIdx.x;  // embedding component
    const int64_t b = off[s] - row_base;
    int L = (int)(off[s + 1] - off[s]);
    if (b < 0 || b + L > R) L = 0;  // offsets inconsistent with the chunk: read nothing
    const int seg = q / kC4, c = q - (q / kC4) * kC4;
    const int lo = (seg * L) / kSegments, hi = ((seg + 1) * L) / kSegments;
    float acc = 0.f;
    for (int t = lo; t < hi; ++t) acc += y4[(b + t) * kC4 + c];
    const float v = hi > lo ? acc / (float)(hi - lo) : 0.f;
    if (emb) emb[(int64_t)s * kEmb + q] = v;
    const uint16_t h = to_bf16(v);
    if (emb16) emb16[(int64_t)s * kEmb + q] = h;
    if (sqnorm) {
        const float f = from_bf16(h);
        float sq = f * f;
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) sq += __shfl_xor(sq, m, 64);
        if ((q & 63) == 0) part[q >> 6] = sq;
        __syncthreads();
        if (q == 0) sqnorm[s] = part[0] + part[1];
    }
}

// Gradient of the pooling: dy4[r][c] = demb[s][seg*32 + c] / |segment|.
__global__ void pool_bwd_kernel(const float *__restrict__ demb, const uint32_t *__restrict__ row_info,
                                const int32_t *__restrict__ row_series, int64_t R, uint16_t *__restrict__ dy4)
{
    const int64_t total = R * kC4;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / kC4;
        const int c = (int)(i - r * kC4);
        const uint32_t info = row_info[r];
        const int t = row_t(info), L = row_L(info);
        // the segment holding t: the last one starting at or before t
        int seg = 0;
#pragma unroll
        for (int q = 1; q < kSegments; ++q)
            if (t >= (q * L) / kSegments) seg = q;
        const int lo = (seg * L) / kSegments, hi = ((seg + 1) * L) / kSegments;
        dy4[i] = to_bf16(demb[(int64_t)row_series[r] * kEmb + seg * kC4 + c] / (float)(hi - lo));
    }
}

// Column sums of a bf16 [R][C] matrix added to out[C] (C divides 256).
__global__ __launch_bounds__(256) void colsum_kernel(const uint16_t *__restrict__ g, int64_t R, int C,
                                                     float *__restrict__ out)
{
    __shared__ float red[256];
    const int c = threadIdx.x % C;
    const int lanes = 256 / C;
    const int64_t r0 = (int64_t)blockIdx.x * lanes + threadIdx.x / C;
    const int64_t stride = (int64_t)gridDim.x * lanes;
    float acc = 0.f;
    for (int64_t r = r0; r < R; r += stride) acc += from_bf16(g[r * C + c]);
    red[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < C) {
        float s = 0.f;
        for (int j = 0; j < lanes; ++j) s += red[j * C + threadIdx.x];
        atomicAdd(out + threadIdx.x, s);
    }
}

// Mean pair loss (log(1+p) - log(1+d))^2 with p = sqrt(|e_a - e_b|^2 + eps):
// one wave per pair, two embedding components per lane.
__global__ __launch_bounds__(64) void pair_loss_kernel(const float *__restrict__ emb, const int32_t *__restrict__ pairs,
                                                       const float *__restrict__ target, int P, int nSeries,
                                                       float inv_P, float *__restrict__ demb,
                                                       float *__restrict__ loss_sum)
{
    const int lane = threadIdx.x;
    for (int p = blockIdx.x; p < P; p += gridDim.x) {
        const int64_t ia = pairs[2 * p], ib = pairs[2 * p + 1];
        if (ia < 0 || ia >= nSeries || ib < 0 || ib >= nSeries) continue;  // uniform: one pair per wave
        const float d0 = emb[ia * kEmb + lane] - emb[ib * kEmb + lane];
        const float d1 = emb[ia * kEmb + 64 + lane] - emb[ib * kEmb + 64 + lane];
        float ss = d0 * d0 + d1 * d1;
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) ss += __shfl_xor(ss, m, 64);
        const float pd = sqrtf(ss + kEps);
        const float r = log1pf(pd) - log1pf(target[p]);
        const float coef = 2.f * r / ((1.f + pd) * pd) * inv_P;
        atomicAdd(demb + ia * kEmb + lane, coef * d0);
        atomicAdd(demb + ia * kEmb + 64 + lane, coef * d1);
        atomicAdd(demb + ib * kEmb + lane, -coef * d0);
        atomicAdd(demb + ib * kEmb + 64 + lane, -coef * d1);
        if (lane == 0) atomicAdd(loss_sum, r * r * inv_P);
    }
}

// AdamW (decoupled weight decay) on the flat FP32 parameters.
__global__ void adamw_kernel(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                             const float *__restrict__ g, int64_t n, float lr, float wd, float b1, float b2,
                             float eps, float c1, float c2)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float wi = w[i];
        w[i] = wi - lr * ((mi / c1) / (sqrtf(vi / c2) + eps) + wd * wi);
    }
}

__global__ void weight_copies_kernel(const float *__restrict__ w, int cin, int cout, uint16_t *__restrict__ wt,
                                     uint16_t *__restrict__ wb)
{
    const int total = kKsize * cin * cout;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        // i = (tap*cin + c)*cout + n
        const int n = i % cout, k = i / cout;
        const int tap = k / cin, c = k - (k / cin) * cin;
        const uint16_t h = to_bf16(w[i]);
        wt[(int64_t)n * (kKsize * cin) + k] = h;
        wb[(int64_t)c * (kKsize * cout) + (kKsize - 1 - tap) * cout + n] = h;
    }
}

__global__ void fill_kernel(float *__restrict__ p, int64_t n, float v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

static int grid_for(int64_t n, int per_block = 256, int cap = 8192)
{
    int64_t g = (n + per_block - 1) / per_block;
    if (g > cap) g = cap;
    return g < 1 ? 1 : (int)g;
}

hipError_t launch_features(const float *X, const int64_t *off, int nSeries, int64_t row_base, int64_t R,
                           int maxlen, uint32_t *row_info, int32_t *row_series, uint16_t *feat, hipStream_t st)
{
    if (nSeries <= 0) return hipSuccess;
    const int gx = (maxlen + 255) / 256, gy = nSeries < 65535 ? nSeries : 65535;
    hipLaunchKernelGGL(features_kernel, dim3(gx < 1 ? 1 : gx, gy), dim3(256), 0, st, X, off, nSeries, row_base, R,
                       row_info, row_series, feat);
    return hipGetLastError();
}

hipError_t launch_pool(const float *y4, const int64_t *off, int nSeries, int64_t row_base, int64_t R, float *emb,
                       uint16_t *emb16, float *sqnorm, hipStream_t st)
{
    if (nSeries <= 0) return hipSuccess;
    hipLaunchKernelGGL(pool_kernel, dim3(nSeries), dim3(kEmb), 0, st, y4, off, nSeries, row_base, R, emb, emb16,
                       sqnorm);
    return hipGetLastError();
}

hipError_t launch_pool_bwd(const float *demb, const uint32_t *row_info, const int32_t *row_series, int64_t R,
                           uint16_t *dy4, hipStream_t st)
{
    if (R <= 0) return hipSuccess;
    hipLaunchKernelGGL(pool_bwd_kernel, dim3(grid_for(R * kC4)), dim3(256), 0, st, demb, row_info, row_series, R,
                       dy4);
    return hipGetLastError();
}

hipError_t launch_colsum(const uint16_t *g, int64_t R, int C, float *out, hipStream_t st)
{
    if (R <= 0) return hipSuccess;
    if (C <= 0 || 256 % C != 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(colsum_kernel, dim3(grid_for(R, (256 / C) * 16, 1024)), dim3(256), 0, st, g, R, C, out);
    return hipGetLastError();
}

hipError_t launch_pair_loss(const float *emb, const int32_t *pairs, const float *target, int P, int nSeries,
                            float *demb, float *loss_sum, hipStream_t st)
{
    if (P <= 0) return hipSuccess;
    const int grid = P < 16384 ? P : 16384;
    hipLaunchKernelGGL(pair_loss_kernel, dim3(grid), dim3(64), 0, st, emb, pairs, target, P, nSeries,
                       1.0f / (float)P, demb, loss_sum);
    return hipGetLastError();
}

hipError_t launch_adamw(float *w, float *m, float *v, const float *g, int64_t n, float lr, float wd, int64_t step,
                        hipStream_t st)
{
    const double b1 = 0.9, b2 = 0.999;
    const double c1 = 1.0 - __builtin_pow(b1, (double)step), c2 = 1.0 - __builtin_pow(b2, (double)step);
    hipLaunchKernelGGL(adamw_kernel, dim3(grid_for(n)), dim3(256), 0, st, w, m, v, g, n, lr, wd, (float)b1, (float)b2,
                       1e-8f, (float)c1, (float)c2);
    return hipGetLastError();
}

hipError_t launch_weight_copies(const float *w, int cin, int cout, uint16_t *wt, uint16_t *wb, hipStream_t st)
{
    hipLaunchKernelGGL(weight_copies_kernel, dim3(grid_for((int64_t)kKsize * cin * cout)), dim3(256), 0, st, w, cin,
                       cout, wt, wb);
    return hipGetLastError();
}

hipError_t launch_fill(float *p, int64_t n, float v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

}  // namespace cnn
}  // namespace twed

// cnn_kernels.h -- host-side launch interface of the embedding network and
// k-NN selection kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace twed {
namespace cnn {

// Network shape: features (x/8, L/256) -> 64 -> 64 -> 64 -> 4 channels,
// kernel 5 with same padding inside each series, ReLU after layers 1-3,
// 32 length-relative segment means of layer 4 -> 128-d embedding.
constexpr int kLayers = 4;
constexpr int kKsize = 5;
constexpr int kChan[kLayers + 1] = {2, 64, 64, 64, 4};
constexpr int kC4 = 4;
constexpr int kSegments = 32;
constexpr int kEmb = kSegments * kC4;
constexpr float kXScale = 1.0f / 8.0f;
constexpr float kLScale = 1.0f / 256.0f;
constexpr float kEps = 1e-6f;
// Longest series the network accepts (row words hold t and L in 16 bits).
constexpr int64_t kMaxSeriesLen = 65535;

// Flat FP32 parameter vector: per layer W (kKsize, C_in, C_out) row-major,
// then b (C_out).
constexpr int64_t layer_w_count(int l) { return (int64_t)kKsize * kChan[l] * kChan[l + 1]; }
constexpr int64_t layer_offset(int l)
{
    int64_t o = 0;
    for (int i = 0; i < l; ++i) o += layer_w_count(i) + kChan[i + 1];
    return o;
}
constexpr int64_t kParamCount = layer_offset(kLayers);

// A operand forms of the GEMM.
enum AMode : int {
    kAPlain = 0,  // A[m][k] = A[m*lda_m + k*lda_k]
    kAConv = 1,   // A[m][k] = h[(m + tap - 2)*C + c], k = tap*C + c; zero outside row m's series
    kAConvT = 2,  // A[m][k] = h[(k + tap - 2)*C + c], m = tap*C + c; zero outside row k's series
};
// Epilogues.
enum OutMode : int {
    kOutF32 = 0,     // C = acc (+ bias) (ReLU), f32
    kOutBF16 = 1,    // C = acc (+ bias) (ReLU) (* [mask > 0]), bf16
    kOutAtomic = 2,  // C += acc (f32 atomics; split-K)
    kOutDist = 3,    // C = row_norm[m] + col_norm[n] - 2 acc, f32
};

struct GemmArgs {
    int M = 0, N = 0, K = 0;
    int a_mode = kAPlain;
    const uint16_t *A = nullptr;  // bf16
    int64_t lda_m = 0, lda_k = 0;
    int conv_C = 0;                     // channels of h for the conv forms
    const uint32_t *row_info = nullptr;  // (t | L << 16) per packed row, conv forms
    const uint16_t *B = nullptr;        // bf16, B[k][n] = B[k*ldb_k + n*ldb_n]
    int64_t ldb_k = 0, ldb_n = 0;
    void *C = nullptr;
    int64_t ldc = 0;
    const float *bias = nullptr;
    int relu = 0;
    const uint16_t *mask = nullptr;  // bf16 [M][ldc]
    const float *row_norm = nullptr, *col_norm = nullptr;
};
// A kAConv GEMM with 2, 4 or 64 channels, 5 taps and a dense [M][N] output (N = 64
// bf16, or N <= 16 f32) runs on an LDS-staged kernel; any other on the
// per-wave tile kernel.  Both give the same bits for the staged shapes.
hipError_t launch_gemm(int out_mode, const GemmArgs &g, int splitk, hipStream_t st);
// False when the environment sets TWED_CNN_GEMM=generic: then every GEMM and
// weight gradient takes the per-wave tile kernel (a cross-check of the staged ones).
bool conv_staged_enabled();

// Weight and bias gradient of one convolution layer in one pass, written (not
// added) to gWb[0 .. 5 cin cout + cout): dW (kKsize, cin, cout) then db (cout).
// h [R][cin] and dy [R][cout] bf16 packed rows, row words as in GemmArgs.
// (cin, cout) in {(64, 64), (64, 4), (2, 64)}; partial: device scratch of
// conv_wgrad_partial_bytes(R), 16-byte aligned.  Deterministic.
bool conv_wgrad_fits(int cin, int cout);
size_t conv_wgrad_partial_bytes(int64_t R);
hipError_t launch_conv_wgrad(int cin, int cout, const uint16_t *h, const uint32_t *row_info, const uint16_t *dy,
                             int64_t R, float *partial, float *gWb, hipStream_t st);

// Row words, owning series (optional) and layer-1 features of nSeries packed
// series.  off: device offsets of those series into X; packed row of sample
// t of series s is off[s] - row_base + t; rows outside [0, R) are skipped.
hipError_t launch_features(const float *X, const int64_t *off, int nSeries, int64_t row_base, int64_t R,
                           int maxlen, uint32_t *row_info, int32_t *row_series, uint16_t *feat, hipStream_t st);
// Segment means -> f32 and/or bf16 embeddings (and the bf16 squared norms).
hipError_t launch_pool(const float *y4, const int64_t *off, int nSeries, int64_t row_base, int64_t R, float *emb,
                       uint16_t *emb16, float *sqnorm, hipStream_t st);
hipError_t launch_pool_bwd(const float *demb, const uint32_t *row_info, const int32_t *row_series, int64_t R,
                           uint16_t *dy4, hipStream_t st);
hipError_t launch_colsum(const uint16_t *g, int64_t R, int C, float *out, hipStream_t st);
// Pairs with an index outside [0, nSeries) are skipped.
hipError_t launch_pair_loss(const float *emb, const int32_t *pairs, const float *target, int P, int nSeries,
                            float *demb, float *loss_sum, hipStream_t st);
hipError_t launch_adamw(float *w, float *m, float *v, const float *g, int64_t n, float lr, float wd, int64_t step,
                        hipStream_t st);
// bf16 operand copies of layer l's weights: wt [C_out][5 C_in] (forward),
// wb [C_in][5 C_out] with wb[c][u C_out + n] = W[4-u][c][n] (backward data).
hipError_t launch_weight_copies(const float *w, int cin, int cout, uint16_t *wt, uint16_t *wb, hipStream_t st);
hipError_t launch_fill(float *p, int64_t n, float v, hipStream_t st);

// k-NN selection.
// For each of nQ rows of `scores` (row stride ld, nDB columns), the n_cand
// smallest (ties: lowest column) -> cand[q*n_cand ..] (any order).
hipError_t launch_topk_select(const float *scores, int64_t ld, int nQ, int nDB, int n_cand, int32_t *cand,
                              hipStream_t st);
// pairs[2(q n_cand + c)] = (q0 + q, cand[q n_cand + c]) as int64, q < nQ;
// (-1, -1) for a candidate id outside [0, nDB).
hipError_t launch_make_pairs(const int32_t *cand, int nQ, int n_cand, int nDB, int64_t q0, int64_t *pairs,
                             hipStream_t st);
// For each query, the k smallest (dist, id) among its n_cand re-ranked
// candidates, ascending.
hipError_t launch_final_topk(const float *dist, const int32_t *cand, int nQ, int n_cand, int k, int64_t *ids,
                             float *out_dist, hipStream_t st);

}  // namespace cnn
}  // namespace twed

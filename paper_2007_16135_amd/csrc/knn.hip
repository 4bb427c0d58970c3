// knn.hip -- candidate selection for the learned k-NN query.
//
// Scores (squared embedding distances) of one query against the whole
// database are reduced to the n_cand smallest by an exact radix select on
// order-preserving 32-bit keys (three digit passes, histograms in LDS), then
// one ordered gather pass; ties at the threshold go to the lowest database
// ids, so the candidate set is a function of the scores alone.  After the
// exact TWED re-rank the k best candidates are picked by (distance, id).
#include "cnn_kernels.h"

#include <stdint.h>

namespace twed {
namespace cnn {

constexpr int kSelThreads = 256;
constexpr int kSelWaves = kSelThreads / 64;

__device__ __forceinline__ uint32_t order_key(float f)
{
    const uint32_t u = __builtin_bit_cast(uint32_t, f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Exclusive prefix of `flag` over the block in thread order; returns the
// prefix and writes the block total to *total.  Uses tmp[kSelWaves].
__device__ __forceinline__ uint32_t block_prefix(bool flag, uint32_t *tmp, uint32_t *total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t bal = __ballot(flag);
    const uint32_t in_wave = (uint32_t)__builtin_popcountll(bal & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
    if (lane == 0) tmp[wave] = (uint32_t)__builtin_popcountll(bal);
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kSelWaves; ++w) {
        const uint32_t c = tmp[w];
        before += w < wave ? c : 0u;
        all += c;
    }
    __syncthreads();
    *total = all;
    return before + in_wave;
}

__global__ __launch_bounds__(kSelThreads) void topk_select_kernel(const float *__restrict__ scores, int64_t ld,
                                                                  int nDB, int n_cand, int32_t *__restrict__ cand)
{
    constexpr int kBins = 2048;
    __shared__ uint32_t hist[kBins];
    __shared__ uint32_t tmp[kSelWaves];
    __shared__ uint32_t wsum[kSelWaves];
    __shared__ uint32_t sel_bin, sel_before;

    const int q = blockIdx.x;
    const float *row = scores + (int64_t)q * ld;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    uint32_t prefix = 0, pmask = 0, want = (uint32_t)n_cand;
    const int shifts[3] = {21, 10, 0};
    const int widths[3] = {11, 11, 10};
    for (int pass = 0; pass < 3; ++pass) {
        const int sh = shifts[pass];
        const uint32_t dmask = (1u << widths[pass]) - 1u;
        for (int i = tid; i < kBins; i += kSelThreads) hist[i] = 0;
        __syncthreads();
        for (int i = tid; i < nDB; i += kSelThreads) {
            const uint32_t key = order_key(row[i]);
            if ((key & pmask) == prefix) atomicAdd(&hist[(key >> sh) & dmask], 1u);
        }
        __syncthreads();
        // the bin where the running count reaches `want`
        constexpr int kPer = kBins / kSelThreads;
        uint32_t loc[kPer], sum = 0;
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            loc[j] = hist[tid * kPer + j];
            sum += loc[j];
        }
        uint32_t inc = sum;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t o = (uint32_t)__shfl_up((int)inc, d, 64);
            if (lane >= d) inc += o;
        }
        if (lane == 63) wsum[wave] = inc;
        __syncthreads();
        uint32_t base = 0;
#pragma unroll
        for (int w = 0; w < kSelWaves; ++w) base += w < wave ? wsum[w] : 0u;
        const uint32_t excl = base + inc - sum;
        if (excl < want && want <= excl + sum) {
            uint32_t run = excl;
#pragma unroll
            for (int j = 0; j < kPer; ++j) {
                if (run + loc[j] >= want) {
                    sel_bin = (uint32_t)(tid * kPer + j);
                    sel_before = run;
                    break;
                }
                run += loc[j];
            }
        }
        __syncthreads();
        prefix |= sel_bin << sh;
        pmask |= dmask << sh;
        want -= sel_before;
        __syncthreads();
    }
    // prefix is now the key of the n_cand-th smallest score; `want` of the
    // entries equal to it are taken (lowest ids first)
    const uint32_t thr = prefix;
    const uint32_t n_less = (uint32_t)n_cand - want;
    uint32_t base_less = 0, base_eq = 0;
    int32_t *out = cand + (int64_t)q * n_cand;
    for (int i0 = 0; i0 < nDB; i0 += kSelThreads) {
        const int i = i0 + tid;
        const uint32_t key = i < nDB ? order_key(row[i]) : 0xffffffffu;
        const bool less = i < nDB && key < thr;
        const bool eq = i < nDB && key == thr;
        uint32_t tot_less, tot_eq;
        const uint32_t pl = block_prefix(less, tmp, &tot_less);
        const uint32_t pe = block_prefix(eq, tmp, &tot_eq);
        if (less) out[base_less + pl] = i;
        if (eq && base_eq + pe < want) out[n_less + base_eq + pe] = i;
        base_less += tot_less;
        base_eq += tot_eq;
        if (base_less >= n_less && base_eq >= want) break;  // uniform across the block
    }
}

hipError_t launch_topk_select(const float *scores, int64_t ld, int nQ, int nDB, int n_cand, int32_t *cand,
                              hipStream_t st)
{
    if (nQ <= 0) return hipSuccess;
    if (n_cand < 1 || n_cand > nDB) return hipErrorInvalidValue;
    hipLaunchKernelGGL(topk_select_kernel, dim3(nQ), dim3(kSelThreads), 0, st, scores, ld, nDB, n_cand, cand);
    return hipGetLastError();
}

// A candidate id outside [0, nDB) becomes the pair (-1, -1), which the
// batched sweep turns into NaN without touching memory.
__global__ void make_pairs_kernel(const int32_t *__restrict__ cand, int64_t total, int n_cand, int nDB, int64_t q0,
                                  int64_t *__restrict__ pairs)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t c = cand[i];
        const bool ok = c >= 0 && c < nDB;
        pairs[2 * i] = ok ? q0 + i / n_cand : -1;
        pairs[2 * i + 1] = ok ? c : -1;
    }
}

hipError_t launch_make_pairs(const int32_t *cand, int nQ, int n_cand, int nDB, int64_t q0, int64_t *pairs,
                             hipStream_t st)
{
    const int64_t total = (int64_t)nQ * n_cand;
    if (total <= 0) return hipSuccess;
    int64_t g = (total + 255) / 256;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(make_pairs_kernel, dim3((int)g), dim3(256), 0, st, cand, total, n_cand, nDB, q0, pairs);
    return hipGetLastError();
}

// One wave per query: k rounds, each taking the smallest (distance, id) key
// above the previous round's.
__global__ __launch_bounds__(64) void final_topk_kernel(const float *__restrict__ dist, const int32_t *__restrict__ cand,
                                                        int n_cand, int k, int64_t *__restrict__ ids,
                                                        float *__restrict__ out_dist)
{
    const int q = blockIdx.x;
    const int lane = threadIdx.x;
    const float *d = dist + (int64_t)q * n_cand;
    const int32_t *c = cand + (int64_t)q * n_cand;
    uint64_t last = 0;
    bool first = true;
    for (int r = 0; r < k; ++r) {
        uint64_t best = ~0ull;
        for (int i = lane; i < n_cand; i += 64) {
            const uint64_t key = ((uint64_t)order_key(d[i]) << 32) | (uint32_t)c[i];
            if ((first || key > last) && key < best) best = key;
        }
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) {
            const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)best, m, 64);
            const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(best >> 32), m, 64);
            const uint64_t o = ((uint64_t)hi << 32) | lo;
            best = o < best ? o : best;
        }
        last = best;
        first = false;
        if (lane == 0) {
            const uint32_t kd = (uint32_t)(best >> 32);
            const uint32_t u = (kd & 0x80000000u) ? (kd & 0x7fffffffu) : ~kd;
            ids[(int64_t)q * k + r] = (int64_t)(uint32_t)best;
            out_dist[(int64_t)q * k + r] = __builtin_bit_cast(float, u);
        }
    }
}

hipError_t launch_final_topk(const float *dist, const int32_t *cand, int nQ, int n_cand, int k, int64_t *ids,
                             float *out_dist, hipStream_t st)
{
    if (nQ <= 0) return hipSuccess;
    hipLaunchKernelGGL(final_topk_kernel, dim3(nQ), dim3(64), 0, st, dist, cand, n_cand, k, ids, out_dist);
    return hipGetLastError();
}

}  // namespace cnn
}  // namespace twed

// cnn.hip -- the k-NN embedding network on gfx950.
//
// Every convolution is an implicit GEMM on the BF16 matrix cores (FP32
// accumulation): the A operand is read straight from the packed activations
// with the tap shift applied per element and zeroed outside the row's own
// series, so no im2col buffer is ever written.  Series are packed back to
// back (row r = sample t of series s); a per-row word holds (t, L).
//
//   forward  y_l   = conv(h_l; W_l) + b_l      A = h_l (kAConv),  B = W_l^T
//   weights  dW_l  = sum_r h_l[r+tap-2] dy_l[r] A = h_l (kAConvT), B = dy_l
//   data     dh_l  = conv(dy_l; flip(W_l)^T) * [h_l > 0]
//
// Two kernel families: gemm_kernel, one wave per 64x64 output tile reading
// its operands from the caches (any shape; the k-NN score GEMM), and the
// LDS-staged convolution kernels that serve every layer of the network
// (conv_kernel: forward and data gradient; conv_wgrad_kernel: weight and
// bias gradient), where four waves share each staged block of rows.
//
// Masters are FP32; the operand copies of the weights are rebuilt in BF16
// at the start of every call.
#include "cnn_kernels.h"

#include <stdint.h>
#include <algorithm>
#include <cstdlib>
#include <cstring>

namespace twed {
namespace cnn {

typedef __attribute__((ext_vector_type(4))) short bf16x4;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
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
// Every product below runs on v_mfma_f32_16x16x32_bf16 (FP32 accumulation).
// On a 64-wide wave lane l holds row l % 16 of the A block and column l % 16
// of the B block, eight k each; the k of lane group g = l / 16, element e is
// taken as 8 g + e for both operands (the instruction pairs A and B elements
// of the same lane group and slot, so any such assignment that both operands
// share gives the same sum).  The result C[i][j] sits in lane j + 16 (i / 4),
// element i % 4.
__device__ __forceinline__ bf16x8 frag8(uint32_t a, uint32_t b, uint32_t c, uint32_t d)
{
    return __builtin_bit_cast(bf16x8, uint4{a, b, c, d});
}
__device__ __forceinline__ bf16x8 frag8(bf16x4 lo, bf16x4 hi)
{
    const uint2 l = __builtin_bit_cast(uint2, lo), h = __builtin_bit_cast(uint2, hi);
    return frag8(l.x, l.y, h.x, h.y);
}
__device__ __forceinline__ f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

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
    const int li = lane & 15, lk = (lane >> 4) * 8;

    f32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = kbeg; k0 < kend; k0 += 32) {
        const int kk = k0 + lk;
        bf16x8 a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            a[i] = frag8(load_a<AM>(g, m0 + 16 * i + li, kk, kend), load_a<AM>(g, m0 + 16 * i + li, kk + 4, kend));
#pragma unroll
        for (int j = 0; j < 4; ++j)
            b[j] = frag8(load_b(g, n0 + 16 * j + li, kk, kend), load_b(g, n0 + 16 * j + li, kk + 4, kend));
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = mfma32(a[i], b[j], acc[i][j]);
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

// ---- LDS-staged convolutions over 64 channels ---------------------------------------
//
// The GEMM above re-reads every operand from the caches per wave: each h row
// five times (once per tap) and the whole weight operand once per 64-row
// tile.  The two kernels below stage a block of rows in LDS once and let four
// waves share it.

// Staging geometry.  Strides are in bf16 elements; rows are 16-byte aligned
// and 4 (mod 32) dwords apart, so each 8 lanes of a 16-byte fragment read
// cover the 32 banks once.
constexpr int kConvRows = 256;     // rows per workgroup (64 per wave)
constexpr int kHStride = 72;       // staged h row: 64 channels + 8
constexpr int kWgRows = 256;       // source rows per weight-gradient chunk
constexpr int kHtStride = 264;     // staged h^T row: 256 rows + 8
constexpr int kDtStride = 280;     // staged dy^T row: rows s0-8 .. s0+263, + 8
constexpr int kWgMaxGroups = 512;  // weight-gradient workgroups (two per CU)

__device__ __forceinline__ uint4 lds4(const uint16_t *p) { return *reinterpret_cast<const uint4 *>(p); }
__device__ __forceinline__ uint2 lds2(const uint16_t *p) { return *reinterpret_cast<const uint2 *>(p); }
__device__ __forceinline__ uint32_t lds1(const uint16_t *p) { return *reinterpret_cast<const uint32_t *>(p); }

// LDS slot of weight row (output column) n: slot 16 nb + i holds column
// 32 (nb / 2) + 8 (i / 4) + 4 (nb % 2) + i % 4, so that the MFMA results of
// slot blocks 2p and 2p+1 give each lane 8 consecutive output columns.
__device__ __forceinline__ int w_slot(int n)
{
    return 16 * (2 * (n >> 5) + ((n >> 2) & 1)) + 4 * ((n >> 3) & 3) + (n & 3);
}

// out[r][n] = sum_{tap, c} h[r + tap - 2][c] W'[n][C tap + c] with h rows
// outside row r's series read as zero: the kAConv form with C channels
// (C = 2, 4 or 64; K = 5 C), W'[n][k] = B[n*K + k].  A persistent workgroup
// stages W' once, then takes row blocks of 256 (blockIdx.x, + gridDim.x, ..):
// wave w computes rows 64w .. 64w+63 of the block against all N <= 16 NB
// columns, while the h rows of the workgroup's next block are already on
// their way into registers.  The k steps of 32 run in the same order as in
// gemm_kernel, with the same zero padding past K, on the same instruction, so
// both kernels produce the same bits.
template <int C, int NB, int OM, bool MASK>
__global__ __launch_bounds__(256, 2) void conv_kernel(GemmArgs g, int nBlocks)
{
    constexpr int K = kKsize * C;
    constexpr int KP = (K + 31) / 32 * 32;  // K padded to whole MFMA steps
    constexpr int HS = C == 64 ? kHStride : C;  // staged h row (bf16); 1 or 2 dwords for C = 2, 4
    constexpr int WS = KP + 8;                  // staged W' row
    constexpr int kHRows = kConvRows + 4;
    __shared__ __align__(16) uint16_t hS[kHRows * HS];
    __shared__ __align__(16) uint16_t wS[NB * 16 * WS];
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int li = lane & 15, kq = lane >> 4;
    const int R = g.M, N = g.N;

    // W', once per workgroup (rows N .. 16 NB - 1 only feed columns that are never stored).
    {
        constexpr int kWUnits = C == 64 ? NB * 16 * 40 : NB * 16 * (KP / 2);  // 16-byte units, or dwords
        constexpr int kWLoads = (kWUnits + 255) / 256;
        uint4 wv[kWLoads];
#pragma unroll
        for (int q = 0; q < kWLoads; ++q) {
            const int idx = tid + 256 * q;
            wv[q] = uint4{0u, 0u, 0u, 0u};
            if constexpr (C == 64) {
                if (idx < kWUnits && idx / 40 < N) wv[q] = *reinterpret_cast<const uint4 *>(g.B + (int64_t)idx * 8);
            } else {
                const int n = idx / (KP / 2), d = idx - n * (KP / 2);
                if (idx < kWUnits && n < N && d < K / 2)
                    wv[q].x = *reinterpret_cast<const uint32_t *>(g.B + (int64_t)n * K + 2 * d);
            }
        }
#pragma unroll
        for (int q = 0; q < kWLoads; ++q) {
            const int idx = tid + 256 * q;
            if (idx >= kWUnits) continue;
            if constexpr (C == 64) {
                const int n = idx / 40;
                *reinterpret_cast<uint4 *>(wS + (NB == 4 ? w_slot(n) : n) * WS + (idx - n * 40) * 8) = wv[q];
            } else {
                const int n = idx / (KP / 2), d = idx - n * (KP / 2);
                *reinterpret_cast<uint32_t *>(wS + (NB == 4 ? w_slot(n) : n) * WS + 2 * d) = wv[q].x;  // zero past K
            }
        }
    }

    // h rows r0-2 .. r0+257 of a block (zero outside [0, R)) and the row words
    // of this lane's four rows: registers, then LDS.
    constexpr int kHUnits = C == 64 ? kHRows * 8 : kHRows;  // 16-byte units for C = 64, rows otherwise
    constexpr int kHLoads = (kHUnits + 255) / 256;
    uint4 hv[kHLoads];
    uint32_t info[4];
    auto load_block = [&](int64_t r0) {
#pragma unroll
        for (int q = 0; q < kHLoads; ++q) {
            const int idx = tid + 256 * q;
            hv[q] = uint4{0u, 0u, 0u, 0u};
            const int row = C == 64 ? idx >> 3 : idx;
            const int64_t gr = r0 - 2 + row;
            if (idx < kHUnits && gr >= 0 && gr < R) {
                if constexpr (C == 64) {
                    hv[q] = *reinterpret_cast<const uint4 *>(g.A + gr * 64 + (idx & 7) * 8);
                } else if constexpr (C == 4) {
                    const uint2 v = *reinterpret_cast<const uint2 *>(g.A + gr * 4);
                    hv[q].x = v.x;
                    hv[q].y = v.y;
                } else {
                    hv[q].x = *reinterpret_cast<const uint32_t *>(g.A + gr * 2);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t m = r0 + 64 * w + 16 * i + li;
            info[i] = m < R ? g.row_info[m] : 0u;  // L = 0: no tap valid
        }
    };
    auto store_block = [&]() {
#pragma unroll
        for (int q = 0; q < kHLoads; ++q) {
            const int idx = tid + 256 * q;
            if (idx >= kHUnits) continue;
            if constexpr (C == 64) {
                *reinterpret_cast<uint4 *>(hS + (idx >> 3) * kHStride + (idx & 7) * 8) = hv[q];
            } else if constexpr (C == 4) {
                *reinterpret_cast<uint2 *>(hS + idx * 4) = uint2{hv[q].x, hv[q].y};
            } else {
                *reinterpret_cast<uint32_t *>(hS + idx * 2) = hv[q].x;
            }
        }
    };

    if ((int)blockIdx.x < nBlocks) load_block((int64_t)blockIdx.x * kConvRows);
    for (int blk = blockIdx.x; blk < nBlocks; blk += gridDim.x) {
        const int64_t r0 = (int64_t)blk * kConvRows;
        store_block();
        // Bit tap of valid[i]: row (i-block i, lane li) reads a sample of its own series at that tap.
        uint32_t valid[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int t = row_t(info[i]), L = row_L(info[i]);
            uint32_t bits = 0;
#pragma unroll
            for (int tap = 0; tap < kKsize; ++tap) {
                const int ts = t + tap - kKsize / 2;
                if (ts >= 0 && ts < L) bits |= 1u << tap;
            }
            valid[i] = bits;
        }
        __syncthreads();
        if (blk + (int)gridDim.x < nBlocks) load_block((int64_t)(blk + gridDim.x) * kConvRows);

        // Mask words of this block's outputs (data gradients), needed at the end.
        constexpr int kMaskUnits = NB == 4 ? 8 : 1;
        uint4 mv[kMaskUnits];
        if constexpr (MASK) {
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                const int64_t m = r0 + 64 * w + 16 * rb + li;
#pragma unroll
                for (int h2 = 0; h2 < 2; ++h2) {
                    mv[2 * rb + h2] = uint4{0u, 0u, 0u, 0u};
                    if (m < R) mv[2 * rb + h2] = *reinterpret_cast<const uint4 *>(g.mask + m * 64 + 32 * h2 + 8 * kq);
                }
            }
        }

        // acc[rb][nb]: rows 16 rb .. of this wave (MFMA columns) x W' slots 16 nb .. (MFMA rows).
        f32x4 acc[4][NB];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
        for (int ks = 0; ks < KP / 32; ++ks) {
            bf16x8 hf[4], wf[NB];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = 64 * w + 16 * i + li;  // staged row of tap 0 is row + 0
                uint32_t d[4] = {0u, 0u, 0u, 0u};
                if constexpr (C == 64) {
                    // 32 channels of one tap: k = 64 tap + 32 half + 8 kq + e
                    const int tap = ks / 2, half = ks % 2;
                    const uint4 v = lds4(hS + (row + tap) * kHStride + 32 * half + 8 * kq);
                    const bool ok = (valid[i] >> tap) & 1u;
                    d[0] = ok ? v.x : 0u;
                    d[1] = ok ? v.y : 0u;
                    d[2] = ok ? v.z : 0u;
                    d[3] = ok ? v.w : 0u;
                } else if constexpr (C == 4) {
                    // k = 8 kq + e: taps 2 kq and 2 kq + 1, four channels each
#pragma unroll
                    for (int hh = 0; hh < 2; ++hh) {
                        const int tap = 2 * kq + hh;
                        if (tap < kKsize && ((valid[i] >> tap) & 1u)) {
                            const uint2 v = lds2(hS + (row + tap) * 4);
                            d[2 * hh] = v.x;
                            d[2 * hh + 1] = v.y;
                        }
                    }
                } else {
                    // k = 8 kq + e: taps 4 kq .. 4 kq + 3, two channels each
#pragma unroll
                    for (int hh = 0; hh < 4; ++hh) {
                        const int tap = 4 * kq + hh;
                        if (tap < kKsize && ((valid[i] >> tap) & 1u)) d[hh] = lds1(hS + (row + tap) * 2);
                    }
                }
                hf[i] = frag8(d[0], d[1], d[2], d[3]);
            }
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const uint4 v = lds4(wS + (16 * j + li) * WS + 32 * ks + 8 * kq);
                wf[j] = frag8(v.x, v.y, v.z, v.w);
            }
            // out^T = W' h^T: the products and their k order are those of gemm_kernel.
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j) acc[i][j] = mfma32(wf[j], hf[i], acc[i][j]);
        }

        // Lane (li, kq) holds, for row 16 rb + li, the columns of slots 16 nb + 4 kq + e:
        // with the slot order of w_slot, columns 8 kq .. 8 kq + 7 and 32 + 8 kq .. (NB = 4),
        // or 4 kq .. 4 kq + 3 (NB = 1).
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
            const int64_t m = r0 + 64 * w + 16 * rb + li;
            if (m >= R) continue;
            if constexpr (OM == kOutF32) {
                const int n0 = 4 * kq;
                float v[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    v[e] = acc[rb][0][e] + (g.bias && n0 + e < N ? g.bias[n0 + e] : 0.f);
                    if (g.relu) v[e] = v[e] > 0.f ? v[e] : 0.f;
                }
                if (N == 4) {
                    if (kq == 0) *reinterpret_cast<float4 *>((float *)g.C + m * 4) = float4{v[0], v[1], v[2], v[3]};
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (n0 + e < N) ((float *)g.C)[m * N + n0 + e] = v[e];
                }
            } else {
#pragma unroll
                for (int h2 = 0; h2 < 2; ++h2) {
                    const int n0 = 32 * h2 + 8 * kq;
                    uint32_t o[4];
#pragma unroll
                    for (int pr = 0; pr < 4; ++pr) {
                        // columns n0 + 2 pr, n0 + 2 pr + 1: slot block 2 h2 + pr / 2, element 2 (pr % 2) ..
                        const f32x4 &A = acc[rb][2 * h2 + pr / 2];
                        const int e = 2 * (pr % 2);
                        float v0 = A[e] + (g.bias ? g.bias[n0 + 2 * pr] : 0.f);
                        float v1 = A[e + 1] + (g.bias ? g.bias[n0 + 2 * pr + 1] : 0.f);
                        if (g.relu) {
                            v0 = v0 > 0.f ? v0 : 0.f;
                            v1 = v1 > 0.f ? v1 : 0.f;
                        }
                        o[pr] = (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)v0) |
                                ((uint32_t)__builtin_bit_cast(uint16_t, (__bf16)v1) << 16);
                    }
                    if constexpr (MASK) {
                        const uint4 mq = mv[2 * rb + h2];
                        const uint32_t mw[4] = {mq.x, mq.y, mq.z, mq.w};
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            if (!(from_bf16((uint16_t)(mw[c] & 0xffffu)) > 0.f)) o[c] &= 0xffff0000u;
                            if (!(from_bf16((uint16_t)(mw[c] >> 16)) > 0.f)) o[c] &= 0x0000ffffu;
                        }
                    }
                    *reinterpret_cast<uint4 *>((uint16_t *)g.C + m * 64 + n0) = uint4{o[0], o[1], o[2], o[3]};
                }
            }
        }
        __syncthreads();  // hS is free for the next block
    }
}

// The staged kernel serves A = kAConv with 2, 4 or 64 channels and 5 taps,
// B = W' rows of K = 5 C, a dense [M][N] output: N = 64 in bf16 (forward
// layers 1-3 and the data gradients) or N <= 16 in f32 (forward layer 4).
static bool conv_fits(int out_mode, const GemmArgs &g)
{
    const int C = g.conv_C;
    if (g.a_mode != kAConv || !(C == 2 || C == 4 || C == 64) || g.K != kKsize * C) return false;
    if (g.ldb_k != 1 || g.ldb_n != g.K || g.ldc != g.N) return false;
    const uintptr_t in_align = C == 64 ? 15u : (uintptr_t)(2 * C - 1);
    if (((uintptr_t)g.A & in_align) || ((uintptr_t)g.B & (C == 64 ? 15u : 3u))) return false;
    if (((uintptr_t)g.C | (uintptr_t)g.mask) & 15u) return false;
    if (out_mode == kOutBF16) return g.N == 64;
    if (out_mode == kOutF32) return C == 64 && g.N <= 16 && !g.mask;
    return false;
}

static int device_cus()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return cus;
}

// Persistent grid: as many workgroups as fit on the device at once.
template <int C, int NB, int OM, bool MASK>
static hipError_t launch_conv(const GemmArgs &g, int nBlocks, hipStream_t st)
{
    static const int per_cu = [] {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, conv_kernel<C, NB, OM, MASK>, 256, 0) != hipSuccess)
            n = 0;
        return n;
    }();
    const int slots = std::max(1, per_cu) * std::max(1, device_cus());
    const int grid = std::min(nBlocks, slots);
    hipLaunchKernelGGL((conv_kernel<C, NB, OM, MASK>), dim3(grid), dim3(256), 0, st, g, nBlocks);
    return hipGetLastError();
}

bool conv_staged_enabled()
{
    const char *env = std::getenv("TWED_CNN_GEMM");
    return !(env && std::strcmp(env, "generic") == 0);
}

// ---- weight gradient ------------------------------------------------------------------
//
// dW[u][c][n] = sum_r [row r reads its own series at tap u] h[r + u - 2][c] dy[r][n].
// Taking the sum over source rows s = r + u - 2 instead, the h operand is the
// same for all five taps and only dy shifts:
//   dW[u][c][n] = sum_s h[s][c] dy[s + 2 - u][n] [0 <= t_s + 2 - u < L_s],
// where the condition (s and s + 2 - u in one series) depends on row s alone.
// A workgroup owns 256-row chunks of s; per chunk it stages h^T, dy^T (two
// rows of halo each side) and the four condition masks (u = 2 always holds),
// and the waves accumulate MFMA blocks with A = h^T (16 channels x 32 rows)
// and B = the shifted, masked dy^T.  A shift by one row is a 16-bit funnel
// shift of the aligned 16-byte fragment and its neighbours.  An extra A row of
// ones yields the bias gradient sum_s dy[s][n] in the same pass.  Each
// workgroup writes its partial [5 CIN COUT + COUT] once; a second kernel
// sums the partials in a fixed order, so the result is deterministic.
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void conv_wgrad_kernel(const uint16_t *__restrict__ h,
                                                         const uint32_t *__restrict__ row_info,
                                                         const uint16_t *__restrict__ dy, int R, int chunks,
                                                         float *__restrict__ partial, int row_len)
{
    constexpr int kHRows = CIN < 16 ? 16 : CIN;
    constexpr int kDRows = COUT < 16 ? 16 : COUT;
    constexpr bool kWide = COUT >= 64;              // waves split the output columns
    constexpr int kCB = (CIN >= 64 && kWide) ? 4 : 1;  // channel blocks per wave
    constexpr bool kOnesRow = CIN < 16;             // the ones row sits in channel block 0
    __shared__ __align__(16) uint16_t hT[kHRows * kHtStride];
    __shared__ __align__(16) uint16_t dT[kDRows * kDtStride];
    __shared__ __align__(16) uint16_t mk[4 * kWgRows];
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int li = lane & 15, kq = lane >> 4;
    const int jb = kWide ? w : 0;   // output column block
    const int cb0 = kWide ? 0 : w;  // first channel block
    constexpr uint32_t kOne2 = 0x3f803f80u;  // two bf16 ones

    // Rows that no chunk overwrites: the ones row and zero padding of h^T,
    // zero padding of dy^T.
    for (int idx = tid; idx < (kHRows - CIN) * kHtStride; idx += 256) {
        const int row = CIN + idx / kHtStride;
        hT[row * kHtStride + idx % kHtStride] = row == CIN && kOnesRow ? (uint16_t)0x3f80 : (uint16_t)0;
    }
    for (int idx = tid; idx < (kDRows - COUT) * kDtStride; idx += 256) dT[COUT * kDtStride + idx] = 0;

    f32x4 acc[kKsize][kCB], accb = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int u = 0; u < kKsize; ++u)
#pragma unroll
        for (int cb = 0; cb < kCB; ++cb) acc[u][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
    // The separate ones block (64 channels): row 0 of the block is ones.
    const bf16x8 ones = li == 0 ? frag8(kOne2, kOne2, kOne2, kOne2) : frag8(0u, 0u, 0u, 0u);
    const bool bias_wave = !kOnesRow && cb0 == 0;

    for (int ch = blockIdx.x; ch < chunks; ch += gridDim.x) {
        const int64_t s0 = (int64_t)ch * kWgRows;
        __syncthreads();  // the previous chunk's reads are done
        // Loads first (one wait for memory per chunk), then the transposing stores.
        // h^T[c][s - s0], s in [s0, s0 + 256), zero at or beyond R; dy^T[n][s - s0 + 8],
        // s in [s0 - 8, s0 + 264), zero outside [0, R).  A 16-byte unit holds 8
        // channels of one row; a thread takes four consecutive rows of one unit column.
        constexpr int kHUnits = CIN == 64 ? 8 * (kWgRows / 4) : kWgRows / 4;        // (unit column, row group)
        constexpr int kDUnits = COUT == 64 ? 8 * (kWgRows / 4 + 4) : kWgRows / 4 + 4;
        constexpr int kHLoads = (kHUnits + 255) / 256, kDLoads = (kDUnits + 255) / 256;
        uint4 hv[kHLoads][4], dv[kDLoads][4];
#pragma unroll
        for (int q = 0; q < kHLoads; ++q) {
            const int idx = tid + 256 * q;
            const int grp = CIN == 64 ? idx >> 3 : idx, col = CIN == 64 ? idx & 7 : 0;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t sr = s0 + 4 * grp + e;
                hv[q][e] = uint4{0u, 0u, 0u, 0u};
                if (idx < kHUnits && sr < R) {
                    if constexpr (CIN == 64) hv[q][e] = *reinterpret_cast<const uint4 *>(h + sr * 64 + 8 * col);
                    else hv[q][e].x = *reinterpret_cast<const uint32_t *>(h + sr * 2);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < kDLoads; ++q) {
            const int idx = tid + 256 * q;
            const int grp = COUT == 64 ? idx >> 3 : idx, col = COUT == 64 ? idx & 7 : 0;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t sr = s0 - 8 + 4 * grp + e;
                dv[q][e] = uint4{0u, 0u, 0u, 0u};
                if (idx < kDUnits && sr >= 0 && sr < R) {
                    if constexpr (COUT == 64) {
                        dv[q][e] = *reinterpret_cast<const uint4 *>(dy + sr * 64 + 8 * col);
                    } else {
                        const uint2 v = *reinterpret_cast<const uint2 *>(dy + sr * 4);
                        dv[q][e].x = v.x;
                        dv[q][e].y = v.y;
                    }
                }
            }
        }
        int mt = 0, mL = 0;
        if (s0 + tid < R) {
            const uint32_t info = row_info[s0 + tid];
            mt = row_t(info);
            mL = row_L(info);
        }
        // Four rows of channel pair (2k, 2k+1) -> two transposed 8-byte stores.
        auto put = [](uint16_t *base, int stride, int ch, int col4, uint32_t x0, uint32_t x1, uint32_t x2,
                      uint32_t x3) {
            *reinterpret_cast<uint2 *>(base + ch * stride + col4) =
                uint2{(x0 & 0xffffu) | (x1 << 16), (x2 & 0xffffu) | (x3 << 16)};
            *reinterpret_cast<uint2 *>(base + (ch + 1) * stride + col4) =
                uint2{(x0 >> 16) | (x1 & 0xffff0000u), (x2 >> 16) | (x3 & 0xffff0000u)};
        };
#pragma unroll
        for (int q = 0; q < kHLoads; ++q) {
            const int idx = tid + 256 * q;
            if (idx >= kHUnits) continue;
            const int grp = CIN == 64 ? idx >> 3 : idx, col = CIN == 64 ? idx & 7 : 0;
            const uint4 *v = hv[q];
            put(hT, kHtStride, 8 * col, 4 * grp, v[0].x, v[1].x, v[2].x, v[3].x);
            if constexpr (CIN == 64) {
                put(hT, kHtStride, 8 * col + 2, 4 * grp, v[0].y, v[1].y, v[2].y, v[3].y);
                put(hT, kHtStride, 8 * col + 4, 4 * grp, v[0].z, v[1].z, v[2].z, v[3].z);
                put(hT, kHtStride, 8 * col + 6, 4 * grp, v[0].w, v[1].w, v[2].w, v[3].w);
            }
        }
#pragma unroll
        for (int q = 0; q < kDLoads; ++q) {
            const int idx = tid + 256 * q;
            if (idx >= kDUnits) continue;
            const int grp = COUT == 64 ? idx >> 3 : idx, col = COUT == 64 ? idx & 7 : 0;
            const uint4 *v = dv[q];
            put(dT, kDtStride, 8 * col, 4 * grp, v[0].x, v[1].x, v[2].x, v[3].x);
            put(dT, kDtStride, 8 * col + 2, 4 * grp, v[0].y, v[1].y, v[2].y, v[3].y);
            if constexpr (COUT == 64) {
                put(dT, kDtStride, 8 * col + 4, 4 * grp, v[0].z, v[1].z, v[2].z, v[3].z);
                put(dT, kDtStride, 8 * col + 6, 4 * grp, v[0].w, v[1].w, v[2].w, v[3].w);
            }
        }
        // Condition masks for u = 0, 1, 3, 4 (0xffff where s and s + 2 - u share a series).
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int u = q < 2 ? q : q + 1;
            const int tr = mt + kKsize / 2 - u;
            mk[q * kWgRows + tid] = (tr >= 0 && tr < mL) ? (uint16_t)0xffff : (uint16_t)0;
        }
        __syncthreads();

#pragma unroll 2
        for (int ks = 0; ks < kWgRows / 32; ++ks) {
            const int kl = 32 * ks + 8 * kq;  // this lane's eight source rows: kl .. kl+7
            bf16x8 a[kCB];
#pragma unroll
            for (int cb = 0; cb < kCB; ++cb) {
                const uint4 v = lds4(hT + (16 * (cb0 + cb) + li) * kHtStride + kl);
                a[cb] = frag8(v.x, v.y, v.z, v.w);
            }
            const uint16_t *drow = dT + (16 * jb + li) * kDtStride + kl + 8;
            const uint32_t p1 = lds1(drow - 2);  // rows kl-2, kl-1
            const uint4 q = lds4(drow);          // rows kl .. kl+7
            const uint32_t w0 = lds1(drow + 8);  // rows kl+8, kl+9
            // Pairs of rows shifted by one: (kl+1, kl+2), (kl+3, kl+4), (kl+5, kl+6).
            const uint32_t m1 = __builtin_amdgcn_alignbit(q.y, q.x, 16);
            const uint32_t m3 = __builtin_amdgcn_alignbit(q.z, q.y, 16);
            const uint32_t m5 = __builtin_amdgcn_alignbit(q.w, q.z, 16);
            // B for tap u holds rows kl + e + 2 - u.
            uint4 bu[kKsize];
            bu[0] = uint4{q.y, q.z, q.w, w0};
            bu[1] = uint4{m1, m3, m5, __builtin_amdgcn_alignbit(w0, q.w, 16)};
            bu[2] = q;
            bu[3] = uint4{__builtin_amdgcn_alignbit(q.x, p1, 16), m1, m3, m5};
            bu[4] = uint4{p1, q.x, q.y, q.z};
#pragma unroll
            for (int qm = 0; qm < 4; ++qm) {
                const int u = qm < 2 ? qm : qm + 1;
                const uint4 m = lds4(mk + qm * kWgRows + kl);
                bu[u].x &= m.x;
                bu[u].y &= m.y;
                bu[u].z &= m.z;
                bu[u].w &= m.w;
            }
#pragma unroll
            for (int u = 0; u < kKsize; ++u) {
                const bf16x8 b = frag8(bu[u].x, bu[u].y, bu[u].z, bu[u].w);
#pragma unroll
                for (int cb = 0; cb < kCB; ++cb) acc[u][cb] = mfma32(a[cb], b, acc[u][cb]);
            }
            if (bias_wave) accb = mfma32(ones, frag8(q.x, q.y, q.z, q.w), accb);
        }
    }

    // Partial of this workgroup: C[i][j] of a block sits in lane j + 16 (i / 4), element i % 4.
    float *P = partial + (int64_t)blockIdx.x * row_len;
    const int n = 16 * jb + li;
    if (n < COUT) {
#pragma unroll
        for (int u = 0; u < kKsize; ++u)
#pragma unroll
            for (int cb = 0; cb < kCB; ++cb)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int c = 16 * (cb0 + cb) + 4 * kq + e;
                    if (c < CIN) P[(u * CIN + c) * COUT + n] = acc[u][cb][e];
                    if (kOnesRow && u == kKsize / 2 && cb == 0 && c == CIN) P[kKsize * CIN * COUT + n] = acc[u][cb][e];
                }
        if (bias_wave && kq == 0) P[kKsize * CIN * COUT + n] = accb[0];
    }
}

// out[e] = sum_g partial[g][e], g in order, e < row_len (a multiple of 4).
// Block: 16 float4 columns x 16 slices of g; slice sums combine in order.
__global__ __launch_bounds__(256) void partial_sum_kernel(const float *__restrict__ partial, int G, int row_len,
                                                          float *__restrict__ out)
{
    __shared__ float4 red[16][16];
    const int col = threadIdx.x & 15, sl = threadIdx.x >> 4;
    const int e4 = (blockIdx.x * 16 + col) * 4;
    float4 s = float4{0.f, 0.f, 0.f, 0.f};
    if (e4 < row_len) {
#pragma unroll 4
        for (int gi = sl; gi < G; gi += 16) {
            const float4 v = *reinterpret_cast<const float4 *>(partial + (int64_t)gi * row_len + e4);
            s.x += v.x;
            s.y += v.y;
            s.z += v.z;
            s.w += v.w;
        }
    }
    red[sl][col] = s;
    __syncthreads();
    if (sl == 0 && e4 < row_len) {
        float4 t = red[0][col];
        for (int k = 1; k < 16; ++k) {
            t.x += red[k][col].x;
            t.y += red[k][col].y;
            t.z += red[k][col].z;
            t.w += red[k][col].w;
        }
        out[e4] = t.x;
        out[e4 + 1] = t.y;
        out[e4 + 2] = t.z;
        out[e4 + 3] = t.w;
    }
}

static int wgrad_groups(int64_t R)
{
    const int64_t chunks = (R + kWgRows - 1) / kWgRows;
    if (chunks <= 0) return 0;
    const int64_t per = (chunks + kWgMaxGroups - 1) / kWgMaxGroups;
    return (int)((chunks + per - 1) / per);
}

static int wgrad_row_len(int cin, int cout) { return kKsize * cin * cout + cout; }

size_t conv_wgrad_partial_bytes(int64_t R)
{
    return (size_t)wgrad_groups(R) * (size_t)wgrad_row_len(64, 64) * sizeof(float);
}

bool conv_wgrad_fits(int cin, int cout)
{
    return (cin == 64 && cout == 64) || (cin == 64 && cout == 4) || (cin == 2 && cout == 64);
}

hipError_t launch_conv_wgrad(int cin, int cout, const uint16_t *h, const uint32_t *row_info, const uint16_t *dy,
                             int64_t R, float *partial, float *gWb, hipStream_t st)
{
    if (!conv_wgrad_fits(cin, cout) || R > 0x7fffffffLL) return hipErrorInvalidValue;
    if (((uintptr_t)h | (uintptr_t)dy) & 7u || (uintptr_t)partial & 15u) return hipErrorInvalidValue;
    const int G = wgrad_groups(R);
    if (G == 0) return hipSuccess;
    const int chunks = (int)((R + kWgRows - 1) / kWgRows);
    const int row_len = wgrad_row_len(cin, cout);
    if (cin == 64 && cout == 64)
        hipLaunchKernelGGL((conv_wgrad_kernel<64, 64>), dim3(G), dim3(256), 0, st, h, row_info, dy, (int)R, chunks,
                           partial, row_len);
    else if (cin == 64)
        hipLaunchKernelGGL((conv_wgrad_kernel<64, 4>), dim3(G), dim3(256), 0, st, h, row_info, dy, (int)R, chunks,
                           partial, row_len);
    else
        hipLaunchKernelGGL((conv_wgrad_kernel<2, 64>), dim3(G), dim3(256), 0, st, h, row_info, dy, (int)R, chunks,
                           partial, row_len);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(partial_sum_kernel, dim3((row_len / 4 + 15) / 16), dim3(256), 0, st, partial, G, row_len,
                       gWb);
    return hipGetLastError();
}

hipError_t launch_gemm(int out_mode, const GemmArgs &g, int splitk, hipStream_t st)
{
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    if (conv_fits(out_mode, g) && conv_staged_enabled()) {
        const int nBlocks = (g.M + kConvRows - 1) / kConvRows;
        const bool mask = g.mask != nullptr;
        if (out_mode == kOutF32) return launch_conv<64, 1, kOutF32, false>(g, nBlocks, st);
        if (g.conv_C == 64)
            return mask ? launch_conv<64, 4, kOutBF16, true>(g, nBlocks, st)
                        : launch_conv<64, 4, kOutBF16, false>(g, nBlocks, st);
        if (g.conv_C == 4)
            return mask ? launch_conv<4, 4, kOutBF16, true>(g, nBlocks, st)
                        : launch_conv<4, 4, kOutBF16, false>(g, nBlocks, st);
        return mask ? launch_conv<2, 4, kOutBF16, true>(g, nBlocks, st)
                    : launch_conv<2, 4, kOutBF16, false>(g, nBlocks, st);
    }
    if (splitk < 1) splitk = 1;
    int kchunk = (g.K + splitk - 1) / splitk;
    kchunk = (kchunk + 31) / 32 * 32;  // whole MFMA steps per chunk
    if (kchunk < 32) kchunk = 32;
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

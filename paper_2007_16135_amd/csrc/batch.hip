// batch.hip -- many TWED pairs in one persistent launch.
//
// The paper's batch mode (section "cuTWED Implementation Remarks") maps
// (series pair, diagonal entry) onto a 2-D grid and fills the whole distance
// matrix; its section "Validation using Real Datasets" notes that the
// symmetric case needs only the upper triangle.  Here each pair is swept by
// one wave with the whole band in registers: the shorter series is spread
// over the 64 lanes (K = ceil(n/64) columns per lane, K <= KMAX), the longer
// one streams through them, and the three live diagonals never leave the
// register file.  Waves pull pairs from an atomic ticket; in the symmetric
// mode the series are visited longest-first so the expensive pairs start
// first and the cheap ones fill the tail.  Results are bitwise equal to the
// single-pair sweep: both evaluate every cell with the same lane code, and
// the cell arithmetic is symmetric under transposition.
#include "twed_dispatch.h"

#include <math.h>

namespace twed {

int batch_kmax(int dimt)
{
    if (dimt <= 1) return 16;
    if (dimt <= 4) return 8;
    if (dimt <= 8) return 4;
    if (dimt <= 16) return 2;
    return 1;
}

template <int DIMT>
__host__ __device__ constexpr int kmax_of()
{
    return DIMT <= 1 ? 16 : (DIMT <= 4 ? 8 : (DIMT <= 8 ? 4 : (DIMT <= 16 ? 2 : 1)));
}

// Sweeps one pair with one wave; returns DP(nA, nB) in every lane.  Pairs
// here are short enough that the FP32 offset is zero (the single-pair sweep
// applies one only beyond kOffsetMinLength samples), so the two paths stay
// bitwise equal.
template <typename CT, typename AT, int DIMT, int PM, int K>
__device__ __forceinline__ AT sweep_pair(const CT *__restrict__ rowsA, int nA, const CT *__restrict__ rowsB,
                                         int nB, const CostArgs<CT> &ca)
{
    const int lane = threadIdx.x & (kWave - 1);
    const AT INF = pinf<AT>();
    const int c0 = 1 + lane * K;
    Lane<CT, AT, DIMT, K> L;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        Row<CT, DIMT> b;
        load_row<CT, DIMT>(rowsB, c0 + j <= nB ? c0 + j : nB, b);
#pragma unroll
        for (int k = 0; k < DIMT; ++k) L.bx[j][k] = b.x[k];
        L.bt[j] = b.t;
        L.bdel[j] = (AT)b.del;
        L.up[j] = INF;
        L.xp[j] = INF;
    }
    const int q = nB - 1;
    const int lstar = q / K, jstar = q - (q / K) * K;

    AT sh_l = INF;
    AT sh_x = lane == 0 ? -AT(0) : INF;  // X(0,0) = -beta with beta = 0
    AT sh_xo = INF;
    // Lane l reads row t - l at step t with no clamping: before row 0 and
    // past row nA it reads a neighbouring series or the 64 zero rows that pad
    // every packed buffer (rows -63 .. nA + 64 are touched).  Those rows only
    // meet +inf operands (before row 0) or feed no result (past row nA).
    // For wide samples, lanes whose columns all lie past nB (they feed no
    // result: values only flow to higher lanes) read lane 0's row, which the
    // wave's load then serves once instead of fetching rows nobody needs.
    const int row_lane = (DIMT < 8 || c0 <= nB) ? lane : 0;
    const CT *pa = rowsA - (ptrdiff_t)row_lane * Row<CT, DIMT>::kStride;
    Row<CT, DIMT> ra, rb;
    load_row<CT, DIMT>(pa, 0, ra);
    auto step = [&](const Row<CT, DIMT> &row) {
        AT left = sh_l, xl;
        lane_row<CT, AT, DIMT, PM, K>(L, row, left, sh_xo, xl, ca.nu, ca.p, ca.invp, CT(0));
        sh_xo = sh_x;
        sh_l = shift_in(left, INF);
        sh_x = shift_in(xl, INF);
    };
    const int T = nA + lstar + 1;  // last step: lane lstar finishes row nA
    int t = 0;
    // two steps per iteration: the band registers alternate without copies
    for (; t + 2 <= T; t += 2) {
        load_row<CT, DIMT>(pa, t + 1, rb);
        step(ra);
        load_row<CT, DIMT>(pa, t + 2, ra);
        step(rb);
    }
    if (t < T) step(ra);
    AT res = L.up[0];
#pragma unroll
    for (int j = 1; j < K; ++j)
        if (j == jstar) res = L.up[j];
    return lane_value(res, lstar);
}

template <typename CT, typename AT, int DIMT, int PM, int K, int KHI>
__device__ __forceinline__ AT sweep_dispatch(int k, const CT *rowsA, int nA, const CT *rowsB, int nB,
                                             const CostArgs<CT> &ca)
{
    if constexpr (K > kmax_of<DIMT>() || K > KHI) {
        return AT(0);
    } else {
        if (k == K) return sweep_pair<CT, AT, DIMT, PM, K>(rowsA, nA, rowsB, nB, ca);
        return sweep_dispatch<CT, AT, DIMT, PM, K + 1, KHI>(k, rowsA, nA, rowsB, nB, ca);
    }
}

// Items item0 .. nItems-1; pairs of KLO..KHI columns per lane (clipped to
// what the sample width allows) are swept, the others left to other launches.
template <typename CT, typename AT, int DIMT, int PM, int KLO, int KHI>
__global__ __launch_bounds__(64) void batch_kernel(const CT *__restrict__ rowsX, const CT *__restrict__ rowsY,
                                                   const int64_t *__restrict__ offX,
                                                   const int64_t *__restrict__ offY,
                                                   const int32_t *__restrict__ order,
                                                   const int64_t *__restrict__ pairs, int64_t nX, int64_t nY,
                                                   int64_t item0, int64_t nItems, int mode, CostArgs<CT> ca, AT *D,
                                                   uint32_t *ticket, int chunk)
{
    constexpr int S = Row<CT, DIMT>::kStride;
    constexpr int KMAX = kmax_of<DIMT>() < KHI ? kmax_of<DIMT>() : KHI;
    // A ticket is `chunk` consecutive items: for short pairs one atomic per
    // pair on a single counter would cost more than the pair itself.
    for (;;) {
        const int64_t first = item0 + (int64_t)next_ticket(ticket) * chunk;
        if (first >= nItems) break;
        const int64_t last = first + chunk < nItems ? first + chunk : nItems;
        for (int64_t item = first; item < last; ++item) {
            int64_t a, b;
            if (mode == kSymmetric) {
                // item -> (i < j) over the length-sorted order: j-th group holds
                // the pairs (0..j-1, j).
                int64_t j = (int64_t)((1.0 + sqrt(1.0 + 8.0 * (double)item)) * 0.5);
                while (j * (j - 1) / 2 > item) --j;
                while ((j + 1) * j / 2 <= item) ++j;
                const int64_t i = item - j * (j - 1) / 2;
                a = order[i];
                b = order[j];
            } else if (mode == kRect) {
                a = item / nY;
                b = item - a * nY;
            } else {
                a = pairs[2 * item];
                b = pairs[2 * item + 1];
            }
            // a pair-list entry outside the collections yields NaN
            const bool ok = a >= 0 && a < nX && b >= 0 && b < nY;
            if (!ok) {  // uniform: one item per wave
                D[item] = (AT)__builtin_nan("");
                continue;
            }
            const int64_t xa = offX[a], la = offX[a + 1] - xa;
            const int64_t yb = offY[b], lb = offY[b + 1] - yb;
            const CT *ra = rowsX + (xa + a) * S;
            const CT *rb = rowsY + (yb + b) * S;
            // shorter operand across the lanes
            const bool swap = lb > la;
            const CT *rowsA = swap ? rb : ra;
            const CT *rowsB = swap ? ra : rb;
            const int nA = (int)(swap ? lb : la);
            const int nB = (int)(swap ? la : lb);
            const int k = (nB + kWave - 1) / kWave;
            // Pairs wider than one wave are swept by the single-pair path instead.
            if (k >= KLO && k <= KMAX) {
                // d is the same in every lane; every lane stores it (one
                // transaction), so the loop body holds no lane-conditional branch.
                const AT d = sweep_dispatch<CT, AT, DIMT, PM, KLO, KMAX>(k, rowsA, nA, rowsB, nB, ca);
                if (mode == kSymmetric) {
                    D[a * nX + b] = d;
                    D[b * nX + a] = d;
                } else {
                    D[item] = d;
                }
            }
        }
    }
}

// One short query against many series: one lane per pair.  The query (at
// most kLaneMaxQuery samples) sits in LDS and every lane reads the same row
// at the same time (a broadcast); each lane sweeps its own series column by
// column with the query's DP column in registers.  Every cell is evaluated
// with the arithmetic of lane_row (transposed, which changes nothing: the
// point and time terms are symmetric and the minimum is exact), so results
// are bitwise those of the wave-per-pair sweep and of twed_pair.  It
// replaces that sweep for this shape because a wave per pair would spend
// most of its lanes and steps filling and draining a 64-lane pipeline for a
// few hundred cells.
//
// RAW: the series are read as the caller holds them (Y: dim components per
// sample, TY: timestamps) instead of as staged rows, and each sample's
// deletion cost is computed from the sample before it with the staging
// kernel's arithmetic, so a collection queried once needs no staging pass
// (a staged collection, reused by many queries, reads its rows instead).
template <typename CT, typename AT, int DIMT, int PM, bool RAW>
__global__ __launch_bounds__(kWave) void batch_lane_kernel(const CT *__restrict__ rowsQ, int nQ,
                                                           const CT *__restrict__ rowsY,
                                                           const CT *__restrict__ Yraw,
                                                           const CT *__restrict__ TYraw, int dim,
                                                           const int64_t *__restrict__ offY, int64_t nY,
                                                           CostArgs<CT> ca, AT *D, uint32_t *ticket)
{
    constexpr int S = Row<CT, DIMT>::kStride;
    constexpr int QM = kLaneMaxQuery;
    __shared__ CT q[(QM + 1) * S];
    const int lane = threadIdx.x;
    for (int k = lane; k < (nQ + 1) * S; k += kWave) q[k] = rowsQ[k];
    __syncthreads();
    const AT INF = pinf<AT>();
    for (;;) {
        const int64_t first = (int64_t)next_ticket(ticket) * kWave;
        if (first >= nY) break;
        const int64_t item = first + lane;
        const bool ok = item < nY;
        const int64_t b = ok ? item : first;  // idle lanes repeat a pair and store nothing
        const int64_t yb = offY[b];
        const int lb = (int)(offY[b + 1] - yb);
        const CT *rb = rowsY + (yb + b) * S;
        int maxL = lb;
#pragma unroll
        for (int m = kWave / 2; m >= 1; m >>= 1) {
            const int o = __shfl_xor(maxL, m, kWave);
            maxL = o > maxL ? o : maxL;
        }
        // DP(i, j-1) and X(i, j-1) of the query rows i = 0..nQ
        AT up[QM + 1], xq[QM + 1];
        up[0] = AT(0);
        xq[0] = AT(0);
#pragma unroll
        for (int i = 1; i <= QM; ++i) {
            up[i] = INF;
            xq[i] = INF;
        }
        AT res = INF;
        CT px[DIMT], pt = CT(0);  // RAW: the sample before (the zero pad at j = 1)
#pragma unroll
        for (int k = 0; k < DIMT; ++k) px[k] = CT(0);
        for (int j = 1; j <= maxL; ++j) {
            Row<CT, DIMT> bj;
            if constexpr (RAW) {
                // columns past lb repeat sample lb (nothing reads them)
                const int64_t r = yb + (j <= lb ? j : lb) - 1;
#pragma unroll
                for (int k = 0; k < DIMT; ++k) bj.x[k] = k < dim ? Yraw[r * dim + k] : CT(0);
                bj.t = TYraw[r];
                const CT d = point_dist<DIMT, PM, CT>(bj.x, px, ca.p, ca.invp);
                bj.del = fma_(ca.nu, fabs_(bj.t - pt), d) + ca.lambda;
#pragma unroll
                for (int k = 0; k < DIMT; ++k) px[k] = bj.x[k];
                pt = bj.t;
            } else {
                load_row<CT, DIMT>(rb, j <= lb ? j : lb, bj);
            }
            const AT bdel = (AT)bj.del;
            AT above = INF;       // DP(i-1, j), starting at the pad row
            AT diag = xq[0];      // X(i-1, j-1)
            // an offset the compiler cannot see through: the query rows are
            // read from LDS in every column instead of being hoisted out of
            // the column loop (all of them would not fit in registers)
            uint32_t qo = 0;
            asm volatile("" : "+v"(qo));
#pragma unroll
            for (int i = 1; i <= QM; ++i) {
                if (i <= nQ) {
                    Row<CT, DIMT> a;
#pragma unroll
                    for (int k = 0; k < DIMT; ++k) a.x[k] = q[qo + i * S + k];
                    a.t = q[qo + i * S + DIMT];
                    a.del = q[qo + i * S + DIMT + 1];
                    const CT dist = point_dist<DIMT, PM, CT>(a.x, bj.x, ca.p, ca.invp);
                    const AT e = (AT)fma_(ca.nu, fabs_(a.t - bj.t), dist);
                    const AT v = dmin(dmin(diag + e, above + (AT)a.del), up[i] + bdel);
                    diag = xq[i];
                    xq[i] = v + e;
                    up[i] = v;
                    above = v;
                }
            }
            up[0] = INF;
            xq[0] = INF;
            AT last = up[1];
#pragma unroll
            for (int i = 2; i <= QM; ++i)
                if (i == nQ) last = up[i];
            res = j == lb ? last : res;
        }
        if (ok) D[item] = res;
    }
}

// Calls f<KLO, KHI>() with the batch_kernel range of a width class.  Samples
// of more than one component have KMAX <= 8, so their three classes share
// one kernel.
template <typename CT, typename AT, int DIMT, int PM, typename F>
static auto by_class(int cls, F &&f)
{
    if constexpr (kmax_of<DIMT>() > kBatchNarrowMax) {
        if (cls == kBatchNarrow) return f.template operator()<1, kBatchNarrowMax>();
        if (cls == kBatchWide) return f.template operator()<kBatchNarrowMax + 1, kmax_of<DIMT>()>();
    }
    return f.template operator()<1, kmax_of<DIMT>()>();
}

template <typename CT, typename AT, int DIMT, int PM>
static int batch_occupancy(int cls)
{
    return by_class<CT, AT, DIMT, PM>(cls, [&]<int KLO, int KHI>() -> int {
        int blocks = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batch_kernel<CT, AT, DIMT, PM, KLO, KHI>, kWave,
                                                         0) != hipSuccess)
            return 0;
        return blocks;
    });
}

hipError_t launch_batch(Prec prec, const CostParams &cp, const BatchArgs &a, hipStream_t st)
{
    return by_prec(prec, cp.dimt, cp.pm, [&]<typename CT, typename AT, int DIMT, int PM>() -> hipError_t {
        return by_class<CT, AT, DIMT, PM>(a.kclass, [&]<int KLO, int KHI>() -> hipError_t {
            hipLaunchKernelGGL((batch_kernel<CT, AT, DIMT, PM, KLO, KHI>), dim3(a.grid), dim3(kWave), 0, st,
                               (const CT *)a.rowsX, (const CT *)a.rowsY, a.offX, a.offY, a.order, a.pairs, a.nX,
                               a.nY, a.item0, a.nItems, a.mode, CostArgs<CT>::make(cp), (AT *)a.D, a.ticket,
                               a.chunk > 1 ? a.chunk : 1);
            return hipGetLastError();
        });
    });
}

hipError_t launch_batch_lane(Prec prec, const CostParams &cp, const void *rowsQ, int nQ, const void *rowsY,
                            const void *Yraw, const void *TYraw, const int64_t *offY, int64_t nY, void *D,
                            uint32_t *ticket, int grid, hipStream_t st)
{
    if (nQ < 1 || nQ > kLaneMaxQuery) return hipErrorInvalidValue;
    return by_prec(prec, cp.dimt, cp.pm, [&]<typename CT, typename AT, int DIMT, int PM>() -> hipError_t {
        if (Yraw)
            hipLaunchKernelGGL((batch_lane_kernel<CT, AT, DIMT, PM, true>), dim3(grid), dim3(kWave), 0, st,
                               (const CT *)rowsQ, nQ, nullptr, (const CT *)Yraw, (const CT *)TYraw, cp.dim, offY,
                               nY, CostArgs<CT>::make(cp), (AT *)D, ticket);
        else
            hipLaunchKernelGGL((batch_lane_kernel<CT, AT, DIMT, PM, false>), dim3(grid), dim3(kWave), 0, st,
                               (const CT *)rowsQ, nQ, (const CT *)rowsY, nullptr, nullptr, cp.dim, offY, nY,
                               CostArgs<CT>::make(cp), (AT *)D, ticket);
        return hipGetLastError();
    });
}

int batch_max_workers(Prec prec, const CostParams &cp, int kclass)
{
    int per_cu = 0;
    hipError_t e = by_prec(prec, cp.dimt, cp.pm, [&]<typename CT, typename AT, int DIMT, int PM>() -> hipError_t {
        per_cu = batch_occupancy<CT, AT, DIMT, PM>(kclass);
        return hipSuccess;
    });
    if (e != hipSuccess || per_cu <= 0) return 0;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return per_cu * cus;
}

template <typename AT>
__global__ void diag_zero_kernel(AT *D, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        D[i * n + i] = AT(0);
}

template <typename AT>
__global__ void copy_one_kernel(const AT *src, AT *dst)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) dst[0] = src[0];
}

hipError_t launch_batch_diag_zero(Prec prec, void *D, int64_t n, hipStream_t st)
{
    const int grid = (int)((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024);
    if (prec == kF32)
        hipLaunchKernelGGL(diag_zero_kernel<float>, dim3(grid), dim3(256), 0, st, (float *)D, n);
    else
        hipLaunchKernelGGL(diag_zero_kernel<double>, dim3(grid), dim3(256), 0, st, (double *)D, n);
    return hipGetLastError();
}

hipError_t launch_copy_one(Prec prec, const void *src, void *dst, hipStream_t st)
{
    if (prec == kF32)
        hipLaunchKernelGGL(copy_one_kernel<float>, dim3(1), dim3(64), 0, st, (const float *)src, (float *)dst);
    else
        hipLaunchKernelGGL(copy_one_kernel<double>, dim3(1), dim3(64), 0, st, (const double *)src, (double *)dst);
    return hipGetLastError();
}

}  // namespace twed

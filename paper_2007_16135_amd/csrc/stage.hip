// stage.hip -- input staging and deletion costs.
//
// Step 1 of the "Improved Time Warp Edit Distance" algorithm computes the
// consecutive-sample distances of A and B concurrently; here one launch does
// both series (or every series of a batch) and folds in the stiffness and
// deletion penalty:
//   del(i) = d(X'_i, X'_{i-1}) + nu*|T'_i - T'_{i-1}| + lambda,  X'_0 = 0, T'_0 = 0.
// The result is written as packed, 16-byte aligned rows (see Row in
// twed_device.h) so that the sweep fetches a sample, its timestamp and its
// deletion cost with whole 16-byte loads.
#include "twed_dispatch.h"

namespace twed {

int dimt_for(int dim)
{
    if (dim <= 4) return dim < 1 ? 1 : dim;
    if (dim <= 8) return 8;
    if (dim <= 16) return 16;
    if (dim <= 32) return 32;
    return -1;
}

int row_stride(Prec prec, int dimt)
{
    const int vec = prec == kF64 ? 2 : 4;
    return (dimt + 2 + vec - 1) / vec * vec;
}

template <typename CT, int DIMT, int PM>
__global__ __launch_bounds__(256) void stage_kernel(const CT *__restrict__ X, const CT *__restrict__ T,
                                                    const int64_t *__restrict__ off, int64_t nSeries,
                                                    int64_t n_single, int dim, CostArgs<CT> ca,
                                                    CT *__restrict__ rows, uint32_t *zero_ptr,
                                                    int64_t zero_words, int64_t total_rows, int first_prev)
{
    constexpr int S = Row<CT, DIMT>::kStride;
    const int64_t gtid = (int64_t)blockIdx.y * gridDim.x * blockDim.x + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t gsize = (int64_t)gridDim.x * gridDim.y * blockDim.x;
    for (int64_t w = gtid; w < zero_words; w += gsize) zero_ptr[w] = 0u;
    // kRowPad zero rows before and kRowPadTail after the packed rows (read,
    // never used, by sweep lanes that run ahead of or behind the series)
    for (int64_t w = gtid; w < (int64_t)kRowPadTail * S; w += gsize) {
        if (w < (int64_t)kRowPad * S) rows[w - (int64_t)kRowPad * S] = CT(0);
        rows[total_rows * S + w] = CT(0);
    }

    for (int64_t s = blockIdx.y; s < nSeries; s += gridDim.y) {
        const int64_t b = off ? off[s] : 0;
        const int64_t n = off ? off[s + 1] - b : n_single;
        CT *out = rows + (b + s) * S;
        for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r <= n;
             r += (int64_t)gridDim.x * blockDim.x) {
            CT cur[DIMT], prev[DIMT];
#pragma unroll
            for (int k = 0; k < DIMT; ++k) {
                cur[k] = (r >= 1 && k < dim) ? X[(b + r - 1) * dim + k] : CT(0);
                prev[k] = ((r >= 2 || (r == 1 && first_prev)) && k < dim) ? X[(b + r - 2) * dim + k] : CT(0);
            }
            const CT tc = (r >= 1 && T) ? T[b + r - 1] : CT(0);
            const CT tp = ((r >= 2 || (r == 1 && first_prev)) && T) ? T[b + r - 2] : CT(0);
            CT del = CT(0);
            if (r >= 1) {
                const CT d = point_dist<DIMT, PM, CT>(cur, prev, ca.p, ca.invp);
                del = fma_(ca.nu, fabs_(tc - tp), d) + ca.lambda;
            }
            CT v[S];
#pragma unroll
            for (int k = 0; k < S; ++k) v[k] = CT(0);
#pragma unroll
            for (int k = 0; k < DIMT; ++k) v[k] = cur[k];
            v[DIMT] = tc;
            v[DIMT + 1] = del;
            CT *o = out + r * S;
#pragma unroll
            for (int k = 0; k < S; ++k) o[k] = v[k];
        }
    }
}

hipError_t launch_stage(Prec prec, const CostParams &cp, const void *X, const void *T,
                        const int64_t *off, int64_t nSeries, int64_t n_single, int64_t max_len,
                        int64_t total_rows, void *rows, uint32_t *zero_ptr, int64_t zero_words, hipStream_t st,
                        bool first_prev)
{
    // Deletion costs are a cost term: computed in the cost precision.
    const Prec cprec = prec == kF64 ? kF64 : kF32;
    return by_prec(cprec, cp.dimt, cp.pm, [&]<typename CT, typename AT, int DIMT, int PM>() -> hipError_t {
        const int64_t rows_per = max_len + 1;
        int gx = (int)((rows_per + 255) / 256);
        if (gx > 2048) gx = 2048;
        if (gx < 1) gx = 1;
        int gy = (int)(nSeries < 4096 ? nSeries : 4096);
        if (gy < 1) gy = 1;
        hipLaunchKernelGGL((stage_kernel<CT, DIMT, PM>), dim3(gx, gy), dim3(256), 0, st,
                           (const CT *)X, (const CT *)T, off, nSeries, n_single, cp.dim,
                           CostArgs<CT>::make(cp), (CT *)rows, zero_ptr, zero_words, total_rows,
                           first_prev ? 1 : 0);
        return hipGetLastError();
    });
}

template <typename AT>
__global__ void dump_border_kernel(AT *dump, int64_t nA, int64_t nB)
{
    const int64_t W = nB + 1;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= nA + nB;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (i == 0) dump[0] = AT(0);
        else if (i <= nB) dump[i] = pinf<AT>();
        else dump[(i - nB) * W] = pinf<AT>();
    }
}

hipError_t launch_dump_border(Prec prec, void *dump, int64_t nA, int64_t nB, hipStream_t st)
{
    const int grid = (int)((nA + nB + 256) / 256 < 1024 ? (nA + nB + 256) / 256 : 1024);
    if (prec == kF32)
        hipLaunchKernelGGL(dump_border_kernel<float>, dim3(grid), dim3(256), 0, st, (float *)dump, nA, nB);
    else
        hipLaunchKernelGGL(dump_border_kernel<double>, dim3(grid), dim3(256), 0, st, (double *)dump, nA, nB);
    return hipGetLastError();
}

__global__ void widen_kernel(const float *src, double *dst, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (double)src[i];
}

hipError_t launch_widen(const float *src, double *dst, int64_t n, hipStream_t st)
{
    const int grid = (int)((n + 255) / 256 < 2048 ? (n + 255) / 256 : 2048);
    hipLaunchKernelGGL(widen_kernel, dim3(grid < 1 ? 1 : grid), dim3(256), 0, st, src, dst, n);
    return hipGetLastError();
}

}  // namespace twed

// probe.hip -- VALU throughput probe for roofline reporting.
//
// Not part of the distance computation: a loop of independent vector
// operations whose timed rate is the lane-operation ceiling that the sweeps
// are measured against.  Every lane runs eight independent chains, so the
// issue rate, not the latency of one operation, bounds the loop.  The kinds
// match what the sweeps issue: FP32 / FP64 fused multiply-adds, and an add
// followed by a minimum (the deletion and match updates of a cell).
#include "../../include/twed.h"
#include "capi_util.h"

#include <stdint.h>

namespace twed {
namespace {

constexpr int kChains = 8;
constexpr int kProbeThreads = 256;

// Operation of one probe chain step.
enum ProbeOp : int { kFma = 0, kAddMin = 1, kSqrt = 2, kAdd = 3, kMin3 = 4 };

template <typename T, int OP>
__global__ __launch_bounds__(kProbeThreads) void valu_probe_kernel(int64_t iters, T seed, T *__restrict__ sink)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    T a[kChains], c[kChains];
#pragma unroll
    for (int r = 0; r < kChains; ++r) {
        a[r] = seed + (T)(gid & 7) + (T)r;
        c[r] = seed * (T)(r + 2);
    }
    const T b = seed * (T)0.5;
    for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int r = 0; r < kChains; ++r) {
            if constexpr (OP == kFma && sizeof(T) == 4) {
                a[r] = __builtin_fmaf(a[r], b, c[r]);
            } else if constexpr (OP == kFma) {
                a[r] = __builtin_fma(a[r], b, c[r]);
            } else if constexpr (OP == kAddMin && sizeof(T) == 4) {
                a[r] = __builtin_fminf(a[r] + b, c[r]);
            } else if constexpr (OP == kAddMin) {
                a[r] = __builtin_fmin(a[r] + b, c[r]);
            } else if constexpr (OP == kSqrt) {
                static_assert(sizeof(T) == 4, "the square-root probe is FP32 (the sweep's cost type)");
                a[r] = __builtin_amdgcn_sqrtf(a[r]);
            } else if constexpr (OP == kAdd) {
                a[r] = a[r] + b;
            } else {
                static_assert(sizeof(T) == 4, "three-way minimum probe is FP32");
                a[r] = __builtin_fminf(__builtin_fminf(a[r], b), c[r]);
            }
        }
    }
    T s = a[0];
#pragma unroll
    for (int r = 1; r < kChains; ++r) s += a[r];
    sink[gid] = s;
}

}  // namespace
}  // namespace twed

using namespace twed;
using namespace twed::capi;

extern "C" twed_status twed_probe_valu(int32_t kind, int64_t waves, int64_t iters, void *sink, double *lane_ops,
                                       hipStream_t stream)
{
    last_error().clear();
    if (kind < 0 || kind > 7) return fail(TWED_ERR_INVALID, "kind must be 0..7");
    if (waves < 4 || waves % 4 != 0 || waves > (int64_t(1) << 24)) return fail(TWED_ERR_INVALID, "waves must be a multiple of 4 in [4, 2^24]");
    if (iters < 1) return fail(TWED_ERR_INVALID, "iters must be >= 1");
    if (!sink) return fail(TWED_ERR_INVALID, "sink is NULL");
    const int blocks = (int)(waves * 64 / kProbeThreads);
    const double per_iter = kind == 1 || kind == 3 ? 2.0 : 1.0;  // add + min count as two operations
    switch (kind) {
    case 0:
        hipLaunchKernelGGL((valu_probe_kernel<float, kFma>), dim3(blocks), dim3(kProbeThreads), 0, stream, iters,
                           0.999f, (float *)sink);
        break;
    case 1:
        hipLaunchKernelGGL((valu_probe_kernel<float, kAddMin>), dim3(blocks), dim3(kProbeThreads), 0, stream, iters,
                           0.999f, (float *)sink);
        break;
    case 2:
        hipLaunchKernelGGL((valu_probe_kernel<double, kFma>), dim3(blocks), dim3(kProbeThreads), 0, stream, iters,
                           0.999, (double *)sink);
        break;
    case 3:
        hipLaunchKernelGGL((valu_probe_kernel<double, kAddMin>), dim3(blocks), dim3(kProbeThreads), 0, stream, iters,
                           0.999, (double *)sink);
        break;
    case 4:
        hipLaunchKernelGGL((valu_probe_kernel<float, kSqrt>), dim3(blocks), dim3(kProbeThreads), 0, stream, iters,
                           0.999f, (float *)sink);
        break;
    case 5:
        hipLaunchKernelGGL((valu_probe_kernel<float, kAdd>), dim3(blocks), dim3(kProbeThreads), 0, stream, iters,
                           0.999f, (float *)sink);
        break;
    case 6:
        hipLaunchKernelGGL((valu_probe_kernel<double, kAdd>), dim3(blocks), dim3(kProbeThreads), 0, stream, iters,
                           0.999, (double *)sink);
        break;
    default:
        hipLaunchKernelGGL((valu_probe_kernel<float, kMin3>), dim3(blocks), dim3(kProbeThreads), 0, stream, iters,
                           0.999f, (float *)sink);
        break;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail_hip(e, "probe launch");
    if (lane_ops) *lane_ops = (double)waves * 64.0 * (double)iters * kChains * per_iter;
    return TWED_OK;
}

// diagonal.hip -- the band sweep with one kernel launch per anti-diagonal.
//
// This is the evaluation order of the "Improved Time Warp Edit Distance"
// algorithm as the paper's own implementation runs it (section "cuTWED
// Implementation Remarks"): a host loop over the nA + nB + 1 diagonals, one
// 1-D grid per diagonal over its indices, and three diagonal vectors in device
// memory rotated by pointer.  Index = column (Eq. (1)), so the three operands
// of a cell are z_{d-1}[c], z_{d-1}[c-1] and x_{d-2}[c-1]: unit stride across
// the threads of a diagonal.  The vectors hold nB + 1 entries (the column
// never exceeds nB).  Alongside each DP diagonal z the sweep keeps
// x = DP + e, so that a cell evaluates one point distance (the lagged half of
// the match cost was added when the up-left cell was computed).
//
// It is kept as an independent cross-check of the register-band pipeline and
// to measure what per-diagonal launches cost; it is not the fast path.
#include "twed_dispatch.h"

namespace twed {

template <typename CT, typename AT, int DIMT, int PM>
__global__ __launch_bounds__(256) void diagonal_kernel(const CT *__restrict__ rowsA, const CT *__restrict__ rowsB,
                                                       int nA, int nB, int d, CostArgs<CT> ca,
                                                       const AT *__restrict__ z1, const AT *__restrict__ x2,
                                                       AT *__restrict__ z0, AT *__restrict__ x0,
                                                       const CT *beta_ptr, AT *out, AT *dump)
{
    // all-FP32 sweeps lower every cost by beta (see pair_offset)
    const CT beta = kShifted<AT> ? beta_ptr[0] : CT(0);
    const int cmin = d - nA > 0 ? d - nA : 0;
    const int cmax = d < nB ? d : nB;
    const int c = cmin + (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (c > cmax) return;
    const int r = d - c;  // Eq. (2)
    AT v, xv;
    if (r == 0 && c == 0) {
        v = AT(0);
        xv = -(AT)beta;
    } else if (r == 0 || c == 0) {
        v = pinf<AT>();
        xv = pinf<AT>();
    } else {
        Row<CT, DIMT> a, b;
        load_row<CT, DIMT>(rowsA, r, a);
        load_row<CT, DIMT>(rowsB, c, b);
        const CT dist = point_dist<DIMT, PM, CT>(a.x, b.x, ca.p, ca.invp);
        const CT ec = fma_(ca.nu, fabs_(a.t - b.t), dist);
        const AT e = kShifted<AT> ? (AT)(ec - beta) : (AT)ec;
        const AT dela = kShifted<AT> ? (AT)(a.del - beta) : (AT)a.del;
        const AT delb = kShifted<AT> ? (AT)(b.del - beta) : (AT)b.del;
        v = dmin(dmin(x2[c - 1] + e, z1[c] + dela), z1[c - 1] + delb);
        xv = v + e;
    }
    z0[c] = v;
    x0[c] = xv;
    const AT vd = kShifted<AT> ? (AT)((double)v + (double)beta * (double)d) : v;
    if (dump) dump[(size_t)r * (size_t)(nB + 1) + (size_t)c] = vd;
    if (r == nA && c == nB) out[0] = vd;
}

hipError_t launch_diagonal(Prec prec, const CostParams &cp, const DiagonalArgs &a, hipStream_t st)
{
    return by_prec(prec, cp.dimt, cp.pm, [&]<typename CT, typename AT, int DIMT, int PM>() -> hipError_t {
        const int nA = (int)a.nA, nB = (int)a.nB;
        const CostArgs<CT> ca = CostArgs<CT>::make(cp);
        for (int d = 0; d <= nA + nB; ++d) {
            const int cmin = d - nA > 0 ? d - nA : 0;
            const int cmax = d < nB ? d : nB;
            const int len = cmax - cmin + 1;
            AT *z0 = (AT *)a.z[d % 3];
            AT *x0 = (AT *)a.x[d % 3];
            const AT *z1 = (const AT *)a.z[(d + 2) % 3];
            const AT *x2 = (const AT *)a.x[(d + 1) % 3];
            hipLaunchKernelGGL((diagonal_kernel<CT, AT, DIMT, PM>), dim3((len + 255) / 256), dim3(256), 0, st,
                               (const CT *)a.rowsA, (const CT *)a.rowsB, nA, nB, d, ca, z1, x2, z0, x0,
                               (const CT *)a.beta, (AT *)a.out, (AT *)a.dump);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    });
}

}  // namespace twed

// twed_device.h -- device-side building blocks shared by the TWED kernels
// (gfx950, wave64).
//
// Cost terms follow the section "Time Warp Edit Distance" with Marteau's
// stiffness and deletion penalty; the band geometry follows Eq. (1)/(2).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "twed_kernels.h"

namespace twed {

constexpr int kWave = 64;

// Lp flavour of the point distance.  One-component samples always use |x-y|.
enum PMode : int { kL1 = 0, kL2 = 1, kLp = 2 };

template <typename T> __device__ __forceinline__ T pinf();
template <> __device__ __forceinline__ float pinf<float>() { return __builtin_inff(); }
template <> __device__ __forceinline__ double pinf<double>() { return __builtin_inf(); }

__device__ __forceinline__ float dmin(float a, float b) { return __builtin_fminf(a, b); }
__device__ __forceinline__ double dmin(double a, double b) { return __builtin_fmin(a, b); }

__device__ __forceinline__ float fabs_(float a) { return __builtin_fabsf(a); }
__device__ __forceinline__ double fabs_(double a) { return __builtin_fabs(a); }

__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Square root: f32 uses the hardware instruction (1 ulp).  f64 takes the
// steps of the correctly rounded library routine -- the hardware reciprocal
// root refined by one coupled Newton step of the root and its half-inverse,
// then two corrections of the root -- without the routine's rescaling of
// arguments below 2^-767 and its special-value tests (13 instructions
// instead of 18): the same bits for a = 0 and for every a >= 2^-767, a root
// within a few ulps for 2^-1000 <= a < 2^-767, and 0 below 2^-1000 (squared
// distances under 1e-301).  Arguments are finite and non-negative here.
__device__ __forceinline__ float sqrt_(float a) { return __builtin_amdgcn_sqrtf(a); }
__device__ __forceinline__ double sqrt_(double a)
{
    const double y = __builtin_amdgcn_rsq(a);
    double g = a * y, h = 0.5 * y;
    const double r = __builtin_fma(-h, g, 0.5);
    g = __builtin_fma(g, r, g);
    h = __builtin_fma(h, r, h);
    double d = __builtin_fma(-g, g, a);
    g = __builtin_fma(d, h, g);
    d = __builtin_fma(-g, g, a);
    g = __builtin_fma(d, h, g);
    return a >= 0x1p-1000 ? g : 0.0;
}

__device__ __forceinline__ float pow_(float a, float b) { return powf(a, b); }
__device__ __forceinline__ double pow_(double a, double b) { return pow(a, b); }

// ---- packed sample rows ------------------------------------------------------
//
// The staging kernel writes every series as rows of STRIDE elements:
//   [x_0 .. x_{DIMT-1}, t, del, pad...]
// where row 0 is the zero pad (x = 0, t = 0) of the zero-padded series, the
// components beyond the real dimension are zero, and del is the deletion
// cost of that sample (unused in row 0).  Rows are 16-byte aligned so one
// sample is fetched with whole 16-byte loads.
template <typename CT, int DIMT>
struct Row {
    static constexpr int kVec = 16 / (int)sizeof(CT);
    static constexpr int kStride = (DIMT + 2 + kVec - 1) / kVec * kVec;
    CT x[DIMT];
    CT t;
    CT del;
};

template <typename CT, int DIMT>
__device__ __forceinline__ void load_row(const CT *__restrict__ base, int64_t r, Row<CT, DIMT> &row)
{
    constexpr int S = Row<CT, DIMT>::kStride;
    const CT *p = base + r * S;
    CT v[S];
    if constexpr (sizeof(CT) == 4) {
#pragma unroll
        for (int q = 0; q < S / 4; ++q) {
            float4 f = reinterpret_cast<const float4 *>(p)[q];
            v[4 * q + 0] = f.x; v[4 * q + 1] = f.y; v[4 * q + 2] = f.z; v[4 * q + 3] = f.w;
        }
    } else {
#pragma unroll
        for (int q = 0; q < S / 2; ++q) {
            double2 f = reinterpret_cast<const double2 *>(p)[q];
            v[2 * q + 0] = f.x; v[2 * q + 1] = f.y;
        }
    }
#pragma unroll
    for (int k = 0; k < DIMT; ++k) row.x[k] = v[k];
    row.t = v[DIMT];
    row.del = v[DIMT + 1];
}

// Lp distance between two samples (with the 1/p root).
template <int DIMT, int PM, typename CT>
__device__ __forceinline__ CT point_dist(const CT (&a)[DIMT], const CT (&b)[DIMT], CT p, CT invp)
{
    if constexpr (DIMT == 1) {
        return fabs_(a[0] - b[0]);
    } else if constexpr (PM == kL1) {
        CT s = fabs_(a[0] - b[0]);
#pragma unroll
        for (int k = 1; k < DIMT; ++k) s += fabs_(a[k] - b[k]);
        return s;
    } else if constexpr (PM == kL2) {
        CT d = a[0] - b[0];
        CT s = d * d;
#pragma unroll
        for (int k = 1; k < DIMT; ++k) {
            d = a[k] - b[k];
            s = fma_(d, d, s);
        }
        return sqrt_(s);
    } else {
        CT s = CT(0);
#pragma unroll
        for (int k = 0; k < DIMT; ++k) {
            CT d = fabs_(a[k] - b[k]);
            s += d > CT(0) ? pow_(d, p) : CT(0);
        }
        return s > CT(0) ? pow_(s, invp) : CT(0);
    }
}

// ---- cross-lane moves ----------------------------------------------------------

// DPP control "wave_shr:1": lane i receives lane i-1; lane 0 keeps `old`.
constexpr int kDppWaveShr1 = 0x138;

__device__ __forceinline__ float shift_in(float v, float lane0)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
        __builtin_bit_cast(int, lane0), __builtin_bit_cast(int, v), kDppWaveShr1, 0xf, 0xf, false));
}

__device__ __forceinline__ double shift_in(double v, double lane0)
{
    uint64_t u = __builtin_bit_cast(uint64_t, v);
    uint64_t o = __builtin_bit_cast(uint64_t, lane0);
    uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)o, (int)(uint32_t)u,
                                                        kDppWaveShr1, 0xf, 0xf, false);
    uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(o >> 32), (int)(uint32_t)(u >> 32),
                                                        kDppWaveShr1, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ float lane_value(float v, int lane)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}

__device__ __forceinline__ double lane_value(double v, int lane)
{
    uint64_t u = __builtin_bit_cast(uint64_t, v);
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ uint32_t wave_uniform(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

// Next value of a work counter, the same in every lane.  Every lane executes
// the atomic (lane 0 adds 1, the others 0) so no lane-conditional branch sits
// in the caller's loop: a branch on the lane id around an operation whose
// result drives a uniform loop lets the compiler thread that branch across
// the loop latch, which leaves the other lanes looping on a stale value.
__device__ __forceinline__ uint32_t next_ticket(uint32_t *counter)
{
    const uint32_t mine = atomicAdd(counter, __lane_id() == 0 ? 1u : 0u);
    return (uint32_t)__builtin_amdgcn_readlane((int)mine, 0);
}

// Device-scope load of a progress word, the same in every lane.
__device__ __forceinline__ uint32_t load_progress(const uint32_t *p)
{
    return wave_uniform(__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// ---- the band segment a lane carries ----------------------------------------------
//
// A wave sweeps a strip of 64*K consecutive columns; lane l owns columns
// c0 + l*K + j (j < K) and at step t works on row r = t - l, so the 64 lanes
// always sit on one anti-diagonal of the DP matrix (Eq. (1): diagonal
// r + c).  Per column the lane keeps
//   up[j] = DP(r-1, c)                  (previous diagonal, same column)
//   xp[j] = DP(r-1, c) + e(r-1, c)      (match operand one diagonal later)
// where e(r, c) = d(A'_r, B'_c) + nu*|TA'_r - TB'_c|.  The match cost of the
// next diagonal, mat(r+1, c+1) = e(r+1, c+1) + e(r, c), therefore needs only
// the new cell's own e: each cell evaluates one point distance.
template <typename CT, typename AT, int DIMT, int K>
struct Lane {
    CT bx[K][DIMT];
    CT bt[K];
    AT bdel[K];
    AT up[K];
    AT xp[K];
};

// All-FP32 sweeps shift every cost by a per-diagonal offset beta (see
// pair_offset); the other precisions keep beta = 0 and skip the subtraction.
template <typename AT>
constexpr bool kShifted = sizeof(AT) == 4;

// One row of the lane's K columns.  `left` = DP(r, c0-1), `diag` =
// X(r-1, c0-1).  Returns DP(r, last column) in `left` and X(r, last) in
// `xlast`.  With the offset, every cost (deletions and both halves e of a
// match) is lowered by beta, i.e. DP'(r, c) = DP(r, c) - beta*(r + c).
template <typename CT, typename AT, int DIMT, int PM, int K>
__device__ __forceinline__ void lane_row(Lane<CT, AT, DIMT, K> &L, const Row<CT, DIMT> &a, AT &left,
                                         AT diag, AT &xlast, CT nu, CT p, CT invp, CT beta)
{
    const AT dela = kShifted<AT> ? (AT)(a.del - beta) : (AT)a.del;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const CT dist = point_dist<DIMT, PM, CT>(a.x, L.bx[j], p, invp);
        const CT ec = fma_(nu, fabs_(a.t - L.bt[j]), dist);
        const AT e = kShifted<AT> ? (AT)(ec - beta) : (AT)ec;
        const AT v = dmin(dmin(diag + e, L.up[j] + dela), left + L.bdel[j]);
        diag = L.xp[j];
        L.xp[j] = v + e;
        L.up[j] = v;
        left = v;
    }
    xlast = L.xp[K - 1];
}

// lane_row for unshifted accumulators, also returning the move into each of
// the K cells as byte j of the result: 0 the match, 1 the deletion in A (from
// the cell above), 2 the deletion in B (from the cell on the left), ties
// resolved in that order.  The cell values are those of lane_row.
template <typename CT, typename AT, int DIMT, int PM, int K>
__device__ __forceinline__ uint64_t lane_row_dirs(Lane<CT, AT, DIMT, K> &L, const Row<CT, DIMT> &a, AT &left,
                                                  AT diag, AT &xlast, CT nu, CT p, CT invp)
{
    static_assert(!kShifted<AT> && K <= 8, "moves are recorded for FP64 accumulators, K <= 8");
    const AT dela = (AT)a.del;
    uint64_t code = 0;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const CT dist = point_dist<DIMT, PM, CT>(a.x, L.bx[j], p, invp);
        const AT e = (AT)fma_(nu, fabs_(a.t - L.bt[j]), dist);
        const AT m = diag + e, u = L.up[j] + dela, l = left + L.bdel[j];
        const AT v = dmin(dmin(m, u), l);
        const uint64_t mv = (m <= u && m <= l) ? 0u : (u <= l ? 1u : 2u);
        code |= mv << (8 * j);
        diag = L.xp[j];
        L.xp[j] = v + e;
        L.up[j] = v;
        left = v;
    }
    xlast = L.xp[K - 1];
    return code;
}

// ---- sibling recurrences ----------------------------------------------------------
//
// Section "Generalized Dynamic Programming Extensions" (its "Direct
// Extension: LCS") notes that any program whose cells need only the cells
// above, to the left and up-left can be swept the same way.  The strip sweep
// runs three more of them over the same staged rows (timestamps and deletion
// costs unused):
//   DTW    D(r, c) = d(A_r, B_c) + min(D(r-1, c), D(r, c-1), D(r-1, c-1))
//   edit   E(r, c) = min(E(r-1, c) + 1, E(r, c-1) + 1, E(r-1, c-1) + [A_r != B_c])
//   indel  I(r, c) = min(I(r-1, c) + 1, I(r, c-1) + 1, A_r == B_c ? I(r-1, c-1) : inf)
// The indel distance is nA + nB - 2 * LCS(A, B), so the LCS length follows
// from it.  For these the X value a cell hands on is its DP value itself.
// (The Rec enum is in twed_kernels.h.)

template <typename CT, typename AT, int DIMT, int PM, int K, int REC, bool DIRS>
__device__ __forceinline__ uint64_t lane_row_sibling(Lane<CT, AT, DIMT, K> &L, const Row<CT, DIMT> &a, AT &left,
                                                     AT diag, AT &xlast, CT p, CT invp)
{
    static_assert(REC != kRecTwed && K <= 8, "sibling recurrences only");
    uint64_t code = 0;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const AT up = L.up[j];
        AT v;
        uint64_t mv = 0;
        if constexpr (REC == kRecDtw) {
            const AT d = (AT)point_dist<DIMT, PM, CT>(a.x, L.bx[j], p, invp);
            v = d + dmin(dmin(diag, up), left);
            if constexpr (DIRS) mv = (diag <= up && diag <= left) ? 0u : (up <= left ? 1u : 2u);
        } else {
            const AT sub = a.x[0] == L.bx[j][0] ? AT(0) : (REC == kRecEdit ? AT(1) : pinf<AT>());
            const AT m = diag + sub, u = up + AT(1), l = left + AT(1);
            v = dmin(dmin(m, u), l);
            if constexpr (DIRS) mv = (m <= u && m <= l) ? 0u : (u <= l ? 1u : 2u);
        }
        if constexpr (DIRS) code |= mv << (8 * j);
        diag = up;
        L.up[j] = v;
        L.xp[j] = v;
        left = v;
    }
    xlast = L.xp[K - 1];
    return code;
}

// ---- FP32 drift control --------------------------------------------------------
//
// Every monotone path from (0,0) to (nA,nB) crosses each of the nA + nB
// diagonals once, a deletion advancing one diagonal and a match two.  So
// lowering every deletion cost and both halves of every match cost by the
// same beta lowers every path -- and the minimum -- by exactly
// beta*(nA + nB): DP = DP' + beta*(nA + nB).  With beta close to the optimal
// path's cost per diagonal the stored values DP' stay small, and so do the
// FP32 rounding errors that accumulate along the path.  beta is the cheaper
// of two admissible paths divided by nA + nB (an upper bound on the target):
//   match along the main diagonal, then delete the rest of the longer series;
//   match (1,1), then delete the rest of A and the rest of B.
// One wave computes it with FP64 partial sums in a fixed order (lane-strided,
// then a fixed butterfly), and the result is symmetric in (A, B).
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
    return v;
}

template <typename CT, int DIMT, int PM>
__device__ __forceinline__ CT pair_offset(const CT *__restrict__ rowsA, int nA, const CT *__restrict__ rowsB,
                                          int nB, CT nu, CT p, CT invp)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int m = nA < nB ? nA : nB;
    const int nL = nA < nB ? nB : nA;
    const CT *rowsL = nA < nB ? rowsB : rowsA;
    auto e_of = [&](const Row<CT, DIMT> &a, const Row<CT, DIMT> &b) -> double {
        return (double)fma_(nu, fabs_(a.t - b.t), point_dist<DIMT, PM, CT>(a.x, b.x, p, invp));
    };
    double diag = 0.0, sa = 0.0, sb = 0.0, rest = 0.0;
    for (int i = 1 + lane; i <= nL; i += kWave) {
        Row<CT, DIMT> ra, rb;
        if (i < m) {
            load_row<CT, DIMT>(rowsA, i, ra);
            load_row<CT, DIMT>(rowsB, i, rb);
            diag += e_of(ra, rb);
        }
        if (i >= 2 && i <= nA) {
            load_row<CT, DIMT>(rowsA, i, ra);
            sa += (double)ra.del;
        }
        if (i >= 2 && i <= nB) {
            load_row<CT, DIMT>(rowsB, i, rb);
            sb += (double)rb.del;
        }
        if (i > m) {
            load_row<CT, DIMT>(rowsL, i, ra);
            rest += (double)ra.del;
        }
    }
    diag = wave_sum(diag);
    sa = wave_sum(sa);
    sb = wave_sum(sb);
    rest = wave_sum(rest);
    Row<CT, DIMT> a1, b1, am, bm;
    load_row<CT, DIMT>(rowsA, 1, a1);
    load_row<CT, DIMT>(rowsB, 1, b1);
    load_row<CT, DIMT>(rowsA, m, am);
    load_row<CT, DIMT>(rowsB, m, bm);
    const double via_diag = (2.0 * diag + e_of(am, bm)) + rest;
    const double via_del = e_of(a1, b1) + (sa + sb);
    const double best = via_diag < via_del ? via_diag : via_del;
    return (CT)(best / (double)(nA + nB));
}

}  // namespace twed

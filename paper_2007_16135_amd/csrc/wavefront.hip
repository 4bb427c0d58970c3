// wavefront.hip -- single-pair TWED sweep as a persistent pipeline of waves.
//
// The paper's section "Improved Time Warp Edit Distance" shows that cell
// (row, col) needs only its up, left and up-left neighbours, so the cells of
// one anti-diagonal (Eq. (1): diagonal = row + col, index = col) are
// independent and only three diagonals are ever live.  Its implementation
// (section "cuTWED Implementation Remarks") launches one grid per diagonal.
// Here the band is carried in registers instead:
//
//  * The columns 1..nB are cut into strips of 64*K.  One wave owns a strip;
//    lane l owns K consecutive columns and at step t works on row t - l, so
//    the wave's 64 lanes always hold a 64-cell segment of one anti-diagonal,
//    and the three live diagonals of that segment are the lane registers
//    (up, left and the match operand, see Lane in twed_device.h).
//  * The left and up-left operands of a lane's first column come from lane
//    l-1 through one DPP wave shift per step.
//  * Lane 0 of strip s takes them from the right-boundary column of strip
//    s-1 (DP and DP+e per row), which that strip's lane 63 writes to one of
//    two global slots and publishes every 64 rows with a release flag; the
//    consumer polls the flag and acquires before loading 64 rows at once.
//    Two slots suffice: strip s+2 can only write row r after strip s+1 has
//    published row r, which it does after reading it.
//  * Waves take strips from an atomic ticket, so the wave that strip s waits
//    for has always started: no co-residency assumption, no deadlock.
//
// Memory stays O(nA + nB): packed inputs, two boundary columns, one flag per
// strip.  Every cell is evaluated once, in the operation order of the lane
// code, so the result does not depend on scheduling.
#include "twed_dispatch.h"

namespace twed {

// Polls of a predecessor's flag before a wave gives up (tens of seconds).
constexpr uint32_t kMaxPolls = 1u << 23;

template <typename AT>
struct alignas(2 * sizeof(AT)) Pair2 {
    AT dp;
    AT x;
};

template <typename CT, typename AT, int DIMT, int PM, int K>
__global__ __launch_bounds__(64) void wavefront_kernel(const CT *__restrict__ rowsA, const CT *__restrict__ rowsB,
                                                       int nA, int nB, CostArgs<CT> ca, Pair2<AT> *bnd,
                                                       uint32_t *flags, uint32_t *ticket, uint32_t *err,
                                                       int nStrips, const CT *beta_ptr, AT *out, AT *dump)
{
    const int lane = threadIdx.x;
    constexpr int W = kWave * K;
    const AT INF = pinf<AT>();
    const CT beta = kShifted<AT> ? beta_ptr[0] : CT(0);

    for (;;) {
        const int s = (int)next_ticket(ticket);
        if (s >= nStrips) break;

        // ---- columns of this lane
        const int c0 = 1 + s * W + lane * K;
        Lane<CT, AT, DIMT, K> L;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            Row<CT, DIMT> b;
            const int c = c0 + j <= nB ? c0 + j : nB;
            load_row<CT, DIMT>(rowsB, c, b);
#pragma unroll
            for (int k = 0; k < DIMT; ++k) L.bx[j][k] = b.x[k];
            L.bt[j] = b.t;
            L.bdel[j] = kShifted<AT> ? (AT)(b.del - beta) : (AT)b.del;
            L.up[j] = INF;   // DP(0, c)
            L.xp[j] = INF;   // DP(0, c) + e(0, c)
        }

        const bool has_in = s > 0;
        const bool has_out = s + 1 < nStrips;
        const Pair2<AT> *in_slot = bnd + (size_t)((s + 1) & 1) * (size_t)(nA + 1);
        Pair2<AT> *out_slot = bnd + (size_t)(s & 1) * (size_t)(nA + 1);
        const uint32_t *in_flag = flags + (s > 0 ? s - 1 : 0);
        uint32_t *out_flag = flags + s;

        const int last_strip = (nB - 1) / W;
        const int qs = (nB - 1) - last_strip * W;
        const int lstar = qs / K, jstar = qs - (qs / K) * K;
        const bool result_strip = s == last_strip;

        // Operands shifted in from lane l-1 after each step: sh_l is the left
        // operand DP(r, c0-1) of the next step, sh_xo its up-left operand
        // X(r-1, c0-1) = DP + e, and sh_x the X value that becomes sh_xo one
        // step later.  Lane 0 takes them from the strip's left boundary
        // instead: +inf on the pad row and column, except X(0, 0) = 0 (minus
        // the offset) for the first strip.
        AT sh_l = INF;
        AT sh_x = (lane == 0 && !has_in) ? -(AT)beta : INF;
        AT sh_xo = INF;

        const int T = nA + kWave;  // lane 63 reaches row nA at step nA + 63
        Row<CT, DIMT> cur;
        load_row<CT, DIMT>(rowsA, 0, cur);
        Pair2<AT> chunk{INF, INF};

        for (int t0 = 0; t0 < T; t0 += kWave) {
            if (has_in) {
                const uint32_t need = (uint32_t)(t0 + kWave < nA ? t0 + kWave : nA);
                // Bounded wait, uniform across the wave: a wave that gives up
                // marks the error word (the result strip then reports NaN) and
                // carries on, so every wave still reaches the end of the grid.
                uint32_t polls = 0;
                while (load_progress(in_flag) < need) {
                    __builtin_amdgcn_s_sleep(2);
                    if (++polls > kMaxPolls) {
                        __hip_atomic_fetch_or(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        break;
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                const int rr = t0 + 1 + lane < nA ? t0 + 1 + lane : nA;
                chunk = in_slot[rr];
            }
            const int steps = T - t0 < kWave ? T - t0 : kWave;
            for (int i = 0; i < steps; ++i) {
                const int t = t0 + i;
                const int r = t - lane;
                int rn = r + 1;
                rn = rn < 0 ? 0 : (rn > nA ? nA : rn);
                Row<CT, DIMT> nxt;
                load_row<CT, DIMT>(rowsA, rn, nxt);

                AT left = sh_l, xl;
                lane_row<CT, AT, DIMT, PM, K>(L, cur, left, sh_xo, xl, ca.nu, ca.p, ca.invp, beta);

                if (dump != nullptr && r >= 1 && r <= nA) {
#pragma unroll
                    for (int j = 0; j < K; ++j)
                        if (c0 + j <= nB)
                            dump[(size_t)r * (size_t)(nB + 1) + (size_t)(c0 + j)] =
                                kShifted<AT> ? (AT)((double)L.up[j] + (double)beta * (double)(r + c0 + j)) : L.up[j];
                }
                // Stores of wave-uniform values are done by every lane (one
                // transaction): no lane-conditional branch in the step loop.
                if (result_strip && t == nA + lstar) {
                    AT res = L.up[0];
#pragma unroll
                    for (int j = 1; j < K; ++j)
                        if (j == jstar) res = L.up[j];
                    res = lane_value(res, lstar);
                    if (kShifted<AT>) res = (AT)((double)res + (double)beta * (double)(nA + nB));
                    if (load_progress(err) != 0u) res = __builtin_nan("");
                    out[0] = res;
                }
                if (has_out && t >= kWave && t <= nA + kWave - 1)
                    out_slot[t - (kWave - 1)] = Pair2<AT>{lane_value(left, kWave - 1), lane_value(xl, kWave - 1)};

                const AT bl = has_in ? lane_value(chunk.dp, i) : INF;
                const AT bx = has_in ? lane_value(chunk.x, i) : INF;
                sh_xo = sh_x;
                sh_l = shift_in(left, bl);
                sh_x = shift_in(xl, bx);
                cur = nxt;

                if (has_out) {
                    const int r63 = t - (kWave - 1);
                    if (r63 >= 1 && ((r63 & (kWave - 1)) == 0 || r63 == nA)) {
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                        __hip_atomic_store(out_flag, (uint32_t)r63, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
            }
        }
    }
}

template <typename CT, typename AT, int DIMT, int PM, int K>
static hipError_t launch_k(const WavefrontArgs &a, const CostParams &cp, hipStream_t st)
{
    hipLaunchKernelGGL((wavefront_kernel<CT, AT, DIMT, PM, K>), dim3(a.grid), dim3(kWave), 0, st,
                       (const CT *)a.rowsA, (const CT *)a.rowsB, (int)a.nA, (int)a.nB, CostArgs<CT>::make(cp),
                       (Pair2<AT> *)a.bnd, a.flags, a.ticket, a.ticket + 1, (int)a.nStrips, (const CT *)a.beta,
                       (AT *)a.out, (AT *)a.dump);
    return hipGetLastError();
}

template <typename CT, typename AT, int DIMT, int PM, int K>
static int occupancy_k()
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, wavefront_kernel<CT, AT, DIMT, PM, K>, kWave, 0) !=
        hipSuccess)
        return 0;
    return blocks;
}

template <typename CT, int DIMT, int PM>
__global__ __launch_bounds__(64) void offset_kernel(const CT *__restrict__ rowsA, int nA,
                                                    const CT *__restrict__ rowsB, int nB, CostArgs<CT> ca,
                                                    CT *beta)
{
    const CT b = pair_offset<CT, DIMT, PM>(rowsA, nA, rowsB, nB, ca.nu, ca.p, ca.invp);
    beta[0] = b;  // every lane stores the same value
}

hipError_t launch_offset(Prec prec, const CostParams &cp, const void *rowsA, int64_t nA, const void *rowsB,
                         int64_t nB, void *beta, hipStream_t st)
{
    return by_prec(prec, cp.dimt, cp.pm, [&]<typename CT, typename AT, int DIMT, int PM>() -> hipError_t {
        hipLaunchKernelGGL((offset_kernel<CT, DIMT, PM>), dim3(1), dim3(kWave), 0, st, (const CT *)rowsA, (int)nA,
                           (const CT *)rowsB, (int)nB, CostArgs<CT>::make(cp), (CT *)beta);
        return hipGetLastError();
    });
}

hipError_t launch_wavefront(Prec prec, const CostParams &cp, int K, const WavefrontArgs &a, hipStream_t st)
{
    return by_prec(prec, cp.dimt, cp.pm, [&]<typename CT, typename AT, int DIMT, int PM>() -> hipError_t {
        switch (K) {
        case 1: return launch_k<CT, AT, DIMT, PM, 1>(a, cp, st);
        case 2: return launch_k<CT, AT, DIMT, PM, 2>(a, cp, st);
        case 4: return launch_k<CT, AT, DIMT, PM, 4>(a, cp, st);
        case 8: return launch_k<CT, AT, DIMT, PM, 8>(a, cp, st);
        default: return hipErrorInvalidValue;
        }
    });
}

int wavefront_max_workers(Prec prec, const CostParams &cp, int K)
{
    int per_cu = 0;
    hipError_t e = by_prec(prec, cp.dimt, cp.pm, [&]<typename CT, typename AT, int DIMT, int PM>() -> hipError_t {
        switch (K) {
        case 1: per_cu = occupancy_k<CT, AT, DIMT, PM, 1>(); break;
        case 2: per_cu = occupancy_k<CT, AT, DIMT, PM, 2>(); break;
        case 4: per_cu = occupancy_k<CT, AT, DIMT, PM, 4>(); break;
        case 8: per_cu = occupancy_k<CT, AT, DIMT, PM, 8>(); break;
        default: break;
        }
        return hipSuccess;
    });
    if (e != hipSuccess || per_cu <= 0) return 0;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return per_cu * cus;
}

}  // namespace twed

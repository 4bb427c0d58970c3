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
//    s-1 (DP and DP+e per row).  That strip collects its lane 63 outputs in
//    a register (one DPP shift per step), writes them to one of two global
//    slots every kChunk rows and publishes them with a release flag; the
//    consumer polls the flag and acquires before loading kChunk rows at once.
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

// Rows of the strip boundary handed over per flag update (a kernel argument,
// 16, 32 or 64).

// How a consumer reads a published boundary chunk.
//   0 (default): agent-scope acquire fence, then ordinary loads -- the
//      release/acquire pairing of the memory model.  The fence invalidates the
//      local L2, which also drops cached rows of A for every wave on it.
//   1: device-coherent (agent-scope atomic) loads of the chunk, issued after
//      the flag load has returned, with only a workgroup-scope fence: the L2
//      keeps its contents.  This leans on the hardware (no load is issued
//      before the branch on the flag resolves) rather than on a formal
//      acquire; measured no faster on MI355X, it is kept for tuning runs.
enum SyncMode : int { kSyncAcquireFence = 0, kSyncCoherentLoads = 1 };

template <typename AT>
__device__ __forceinline__ Pair2<AT> load_coherent(const Pair2<AT> *p)
{
    if constexpr (sizeof(AT) == 8) {
        const uint64_t *q = reinterpret_cast<const uint64_t *>(p);
        const uint64_t a = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t b = __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return Pair2<AT>{__builtin_bit_cast(AT, a), __builtin_bit_cast(AT, b)};
    } else {
        const uint64_t *q = reinterpret_cast<const uint64_t *>(p);
        const uint64_t a = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return Pair2<AT>{__builtin_bit_cast(AT, (uint32_t)a), __builtin_bit_cast(AT, (uint32_t)(a >> 32))};
    }
}

template <typename AT>
__device__ __forceinline__ void store_coherent(Pair2<AT> *p, const Pair2<AT> &v)
{
    if constexpr (sizeof(AT) == 8) {
        uint64_t *q = reinterpret_cast<uint64_t *>(p);
        __hip_atomic_store(q, __builtin_bit_cast(uint64_t, v.dp), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(q + 1, __builtin_bit_cast(uint64_t, v.x), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        uint64_t *q = reinterpret_cast<uint64_t *>(p);
        const uint64_t w = (uint64_t)__builtin_bit_cast(uint32_t, v.dp) |
                           ((uint64_t)__builtin_bit_cast(uint32_t, v.x) << 32);
        __hip_atomic_store(q, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}
// DPP control "wave_shl:1": lane i receives lane i+1; lane 63 keeps `old`.
constexpr int kDppWaveShl1 = 0x130;

__device__ __forceinline__ float collect(float v_lane63, float col)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
        __builtin_bit_cast(int, v_lane63), __builtin_bit_cast(int, col), kDppWaveShl1, 0xf, 0xf, false));
}

__device__ __forceinline__ double collect(double v_lane63, double col)
{
    uint64_t u = __builtin_bit_cast(uint64_t, col);
    uint64_t o = __builtin_bit_cast(uint64_t, v_lane63);
    uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)o, (int)(uint32_t)u,
                                                        kDppWaveShl1, 0xf, 0xf, false);
    uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(o >> 32), (int)(uint32_t)(u >> 32),
                                                        kDppWaveShl1, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// rowsA points at row 0 of A and must stay readable from row -64 to row
// nA + 64 (the staging pads the buffer): lanes that have not started yet, or
// have finished, read rows outside 1..nA and compute values nobody uses, so
// the row address needs no clamp.
template <typename CT, typename AT, int DIMT, int PM, int K, bool DUMP>
__global__ __launch_bounds__(64) void wavefront_kernel(const CT *__restrict__ rowsA, const CT *__restrict__ rowsB,
                                                       int nA, int nB, CostArgs<CT> ca, Pair2<AT> *bnd,
                                                       uint32_t *flags, uint32_t *ticket, uint32_t *err,
                                                       int nStrips, const CT *beta_ptr, AT *out, AT *dump,
                                                       int chunk_rows, int sync_mode)
{
    constexpr int S = Row<CT, DIMT>::kStride;
    const int kChunk = chunk_rows;
    const int lane = threadIdx.x;
    constexpr int W = kWave * K;
    const AT INF = pinf<AT>();
    const CT beta = kShifted<AT> ? beta_ptr[0] : CT(0);
    const CT *rowsA_lane = rowsA - (ptrdiff_t)lane * S;  // row t of this pointer = row t - lane of A

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
        Row<CT, DIMT> cur, nxt;
        load_row<CT, DIMT>(rowsA_lane, 0, cur);
        Pair2<AT> chunk{INF, INF};
        // Right-boundary collector: lane 63's (DP, X) of each step enters at
        // lane 63 and moves down one lane per step.
        AT col_dp = INF, col_x = INF;

        for (int t0 = 0; t0 < T; t0 += kChunk) {
            if (has_in) {
                // rows t0+1 .. t0+kChunk of the left boundary
                const uint32_t need = (uint32_t)(t0 + kChunk < nA ? t0 + kChunk : nA);
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
                const int rr = t0 + 1 + lane < nA ? t0 + 1 + lane : nA;
                if (sync_mode == kSyncCoherentLoads) {
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                    chunk = load_coherent(in_slot + rr);
                } else {
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    chunk = in_slot[rr];
                }
            }
            const int steps = T - t0 < kChunk ? T - t0 : kChunk;
            // One step: sweep row t - lane with `use`, prefetch row t + 1 -
            // lane into `fill`.  Steps alternate the two row buffers, so the
            // prefetched row never has to be copied.
            auto step = [&](int i, Row<CT, DIMT> &use, Row<CT, DIMT> &fill) {
                const int t = t0 + i;
                load_row<CT, DIMT>(rowsA_lane, t + 1, fill);

                AT left = sh_l, xl;
                lane_row<CT, AT, DIMT, PM, K>(L, use, left, sh_xo, xl, ca.nu, ca.p, ca.invp, beta);

                if constexpr (DUMP) {
                    const int r = t - lane;
                    if (r >= 1 && r <= nA) {
#pragma unroll
                        for (int j = 0; j < K; ++j)
                            if (c0 + j <= nB)
                                dump[(size_t)r * (size_t)(nB + 1) + (size_t)(c0 + j)] =
                                    kShifted<AT> ? (AT)((double)L.up[j] + (double)beta * (double)(r + c0 + j))
                                                 : L.up[j];
                    }
                }
                // The result is wave-uniform; every lane stores it (one
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

                const AT bl = has_in ? lane_value(chunk.dp, i) : INF;
                const AT bx = has_in ? lane_value(chunk.x, i) : INF;
                sh_xo = sh_x;
                sh_l = shift_in(left, bl);
                sh_x = shift_in(xl, bx);
                if (has_out) {
                    col_dp = collect(left, col_dp);
                    col_x = collect(xl, col_x);
                }
            };
            int i = 0;
            for (; i + 1 < steps; i += 2) {
                step(i, cur, nxt);
                step(i + 1, nxt, cur);
            }
            if (i < steps) {
                step(i, cur, nxt);
                cur = nxt;
            }
            if (has_out) {
                // lane kWave - steps + i holds row t0 + i - 63 of the boundary
                // (lanes without a row of this chunk write slot row 0, which
                // no consumer reads: no lane-conditional branch)
                int r = t0 + lane - (kWave - steps) - (kWave - 1);
                r = (lane >= kWave - steps && r >= 1 && r <= nA) ? r : 0;
                if (sync_mode == kSyncCoherentLoads)
                    store_coherent(out_slot + r, Pair2<AT>{col_dp, col_x});
                else
                    out_slot[r] = Pair2<AT>{col_dp, col_x};
                const int last = t0 + steps - kWave;  // last boundary row of this chunk
                if (last >= 1) {
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                    __hip_atomic_store(out_flag, (uint32_t)(last < nA ? last : nA), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
    }
}

template <typename CT, typename AT, int DIMT, int PM, int K>
static hipError_t launch_k(const WavefrontArgs &a, const CostParams &cp, hipStream_t st)
{
    if (a.dump) {
        // cell dumps are a validation aid: narrow strips only
        if constexpr (K <= 2) {
            hipLaunchKernelGGL((wavefront_kernel<CT, AT, DIMT, PM, K, true>), dim3(a.grid), dim3(kWave), 0, st,
                               (const CT *)a.rowsA, (const CT *)a.rowsB, (int)a.nA, (int)a.nB,
                               CostArgs<CT>::make(cp), (Pair2<AT> *)a.bnd, a.flags, a.ticket, a.ticket + 1,
                               (int)a.nStrips, (const CT *)a.beta, (AT *)a.out, (AT *)a.dump, a.chunk_rows,
                               a.sync_mode);
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;
        }
    }
    hipLaunchKernelGGL((wavefront_kernel<CT, AT, DIMT, PM, K, false>), dim3(a.grid), dim3(kWave), 0, st,
                       (const CT *)a.rowsA, (const CT *)a.rowsB, (int)a.nA, (int)a.nB, CostArgs<CT>::make(cp),
                       (Pair2<AT> *)a.bnd, a.flags, a.ticket, a.ticket + 1, (int)a.nStrips, (const CT *)a.beta,
                       (AT *)a.out, nullptr, a.chunk_rows, a.sync_mode);
    return hipGetLastError();
}

template <typename CT, typename AT, int DIMT, int PM, int K>
static int occupancy_k()
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, wavefront_kernel<CT, AT, DIMT, PM, K, false>, kWave,
                                                     0) != hipSuccess)
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

// wavefront_impl.h -- the strip sweep shared by the pair sweep (wavefront.hip)
// and the tile sweep (tile.hip).  See wavefront.hip for the design.
#pragma once

#include "twed_dispatch.h"

namespace twed {


// Polls of a predecessor's progress word before a wave gives up (tens of
// seconds either way: an LDS poll takes about 0.1 us with its sleep, a
// global one a few us).
constexpr uint32_t kMaxPollsLds = 1u << 28;
constexpr uint32_t kMaxPollsGlobal = 1u << 24;
// The error word (a global load, a few us) is read once every kErrEvery
// polls, so a waiting wave notices its predecessor's progress within one
// poll.
constexpr uint32_t kErrEvery = 64;

template <typename AT>
struct alignas(2 * sizeof(AT)) Pair2 {
    AT dp;
    AT x;
};

// Rows per global handoff (one window of the 64-lane boundary register).
// Inside a workgroup the handoff comes every 1 << sub_shift steps (8, 16 or
// 32; a kernel argument).
constexpr int kWindow = 64;
// Rows of one in-group boundary kept in LDS (power of two), plus one slot
// that absorbs the writes of lanes without a row.
constexpr int kRing = 128;

template <typename AT, int G>
struct GroupShared {
    Pair2<AT> ring[G > 1 ? G - 1 : 1][kRing + 1];  // boundary of wave w, read by wave w+1
    Pair2<AT> in_stage[kWindow];                   // wave 0's left boundary, one global window
    Pair2<AT> out_stage[kRing + 1];                // wave G-1's right boundary before it goes out
    uint32_t prod[G];                              // rows of that boundary published
    uint32_t cons[G];                              // rows of wave w's left boundary consumed
    uint32_t ticket[G];                            // ticket value seen by each wave (wave 0's is the claim)
};

__device__ __forceinline__ uint32_t load_lds_progress(const uint32_t *p)
{
    return wave_uniform(__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
}

// Bounded wait until *p >= need (uniform across the wave).  A wave that gives
// up marks the error word (the result strip then reports NaN) and carries
// on, and once the word is set no wave waits any more (it is read every
// kErrEvery polls), so every wave still reaches the end of the grid after at
// most one time-out.
template <bool LDS>
__device__ __forceinline__ void wait_progress(const uint32_t *p, uint32_t need, uint32_t *err)
{
    uint32_t polls = 0;
    while ((LDS ? load_lds_progress(p) : load_progress(p)) < need) {
        if (polls % kErrEvery == kErrEvery - 1 && load_progress(err) != 0u) break;
        __builtin_amdgcn_s_sleep(1);
        if (++polls > (LDS ? kMaxPollsLds : kMaxPollsGlobal)) {
            __hip_atomic_fetch_or(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
    }
}

// Block boundaries and extra outputs of the tile sweep (TILE kernels only;
// pair sweeps pass an empty set).  Cells are (DP, X = DP + e) pairs.
//   top     row 0 of the block, columns 0..nB (null: the pad row of a pair)
//   left    column 0 of the block, rows 0..nA (null: the pad column)
//   bottom  receives row nA, columns 1..nB
//   right   receives column nB, rows 1..nA
//   ckrow   receives rows ck_rows, 2*ck_rows, ... below nA (nB + 1 cells
//           each; column 0 is left to the host)
//   ckcol   receives columns ck_cols, 2*ck_cols, ... left of nB (nA + 1
//           cells each; row 0 is left to the host); ck_cols is a multiple
//           of the strip width
//   dirs    (DIRS kernels) one byte per cell, the move into it (0 match,
//           1 deletion in A from the cell above, 2 deletion in B from the
//           cell on the left), in sweep order: strip s, step t, lane, column
//   dummy   64*K cells that lanes without a cell to store write instead
template <typename AT>
struct TileIO {
    const Pair2<AT> *top;
    const Pair2<AT> *left;
    Pair2<AT> *bottom;
    Pair2<AT> *right;
    Pair2<AT> *ckrow;
    Pair2<AT> *ckcol;
    Pair2<AT> *dummy;
    uint8_t *dirs;
    int ck_rows;
    int ck_cols;
};

template <int K>
__device__ __forceinline__ void store_dirs(uint8_t *p, uint64_t code)
{
    if constexpr (K == 8) *reinterpret_cast<uint64_t *>(p) = code;
    else if constexpr (K == 4) *reinterpret_cast<uint32_t *>(p) = (uint32_t)code;
    else if constexpr (K == 2) *reinterpret_cast<uint16_t *>(p) = (uint16_t)code;
    else *p = (uint8_t)code;
}

// Strip widths compiled for a sample dimension: beyond 16 components a lane
// holds at most two columns (wider strips would not fit the register file).
template <int DIMT, int K>
constexpr bool kStripCompiled = DIMT <= 16 || K <= 2;

// One strip of 64*K columns swept by one wave.  Its left boundary (DP and X =
// DP + e of column c0-1, per row) comes from the previous strip: through LDS
// when that strip belongs to the same workgroup (handoff every kSub rows,
// workgroup-scope release/acquire), through a global slot and flag
// otherwise (every kWindow rows, agent scope).  Its right boundary goes the
// same two ways to the next strip.
//
// rowsA points at row 0 of A and must stay readable from row -64 to row
// nA + 63 + the prefetch distance (the staging pads the buffer with kRowPad
// rows before and kRowPadTail after): lanes that have not started yet, or
// have finished, read rows outside 1..nA and compute values nobody uses, so
// the row address needs no clamp.
//
// A tile sweep (TILE) starts from a given top row and left column instead of
// the pad row and column.  A lane processes rows 0 and below before its
// first real row; in a pair sweep those rows keep the +inf state of the pad
// row, and in a tile the lane loads its top-row cells at the step where it
// sits on row 0, so that row 1 starts from them.
template <typename CT, typename AT, int DIMT, int PM, int K, int G, bool DUMP, bool TILE, int REC, bool DIRS>
__device__ __forceinline__ void sweep_strip(GroupShared<AT, G> &sh, int w, int g, int s, int cbase,
                                            const CT *__restrict__ rowsA,
                                            const CT *__restrict__ rowsB, int nA, int nB, const CostArgs<CT> &ca,
                                            Pair2<AT> *bnd, uint32_t *flags, uint32_t *err, int nStrips, CT beta,
                                            AT *out, AT *dump, int sub_shift, const TileIO<AT> &io)
{
    static_assert(REC == kRecTwed || TILE, "sibling recurrences run as tiles");
    static_assert(!DIRS || TILE, "moves are recorded by tile sweeps");
    const int kSub = 1 << sub_shift;
    constexpr int S = Row<CT, DIMT>::kStride;
    constexpr int W = kWave * K;
    const int lane = threadIdx.x & (kWave - 1);
    const AT INF = pinf<AT>();
    // Row t - lane of A, the row lane `lane` works on at step t: a pointer
    // that advances by one row per step (a 64-bit add, no multiply).
    const CT *row_ptr = rowsA - (ptrdiff_t)lane * S;
    // ---- columns of this lane (the strip's first column is 1 + cbase)
    const int c0 = 1 + cbase + lane * K;
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

    const bool in_global = w == 0 && (s > 0 || (TILE && io.left != nullptr));
    const bool in_lds = w > 0;
    const bool has_out = s + 1 < nStrips;
    const bool out_lds = has_out && w < G - 1;
    const bool out_global = has_out && w == G - 1;
    // global slots alternate between consecutive groups (see the header comment)
    const Pair2<AT> *in_slot = (TILE && s == 0) ? io.left : bnd + (size_t)((g + 1) & 1) * (size_t)(nA + 1);
    Pair2<AT> *out_slot = bnd + (size_t)(g & 1) * (size_t)(nA + 1);
    const uint32_t *in_flag = flags + (g > 0 ? g - 1 : 0);
    uint32_t *out_flag = flags + g;

    // column nB sits in the last strip, at lane lstar, column jstar
    const bool result_strip = s == nStrips - 1;
    const int qs = (nB - 1) - cbase;
    const int lstar = qs / K, jstar = qs - (qs / K) * K;

    // Operands shifted in from lane l-1 after each step: sh_l is the left
    // operand DP(r, c0-1) of the next step, sh_xo its up-left operand
    // X(r-1, c0-1) = DP + e, and sh_x the X value that becomes sh_xo one
    // step later.  Lane 0 takes them from the strip's left boundary
    // instead: +inf on the pad row and column, except X(0, 0) = 0 (minus
    // the offset) for the first strip.
    AT sh_l = INF;
    AT sh_x = (lane == 0 && s == 0) ? -(AT)beta : INF;
    AT sh_xo = INF;
    Pair2<AT> *ck_col = nullptr;
    if constexpr (TILE) {
        // X(0, c0 - 1) of this strip: from the top row, else the corner
        AT x0 = INF;
        if (io.top != nullptr) x0 = io.top[cbase].x;
        else if (s == 0) x0 = io.left != nullptr ? io.left[0].x : AT(0);
        sh_x = lane == 0 ? x0 : INF;
        if (io.ckcol != nullptr && has_out && (cbase + W) % io.ck_cols == 0)
            ck_col = io.ckcol + (size_t)((cbase + W) / io.ck_cols - 1) * (size_t)(nA + 1);
    }

    const int T = nA + kWave;  // lane 63 reaches row nA at step nA + 63
    // The last strip stops once lane lstar has swept row nA (its lanes past
    // lstar hold columns beyond nB): the result is then in that lane's
    // registers, and the step loop carries no test for it.
    const int T_run = result_strip ? nA + lstar + 1 : T;
    // Rows of A are loaded kAhead steps before their use, from a ring of
    // kAhead + 1 rows (kAhead + 1 divides every sub-chunk of 8, 16 or 32
    // steps).  Narrow strips of small samples load three rows ahead.  So do
    // pair sweeps of wide strips whose ring of rows stays small next to the
    // lane's columns (at most 96 registers for the K columns' rows), e.g. 8-D
    // FP32 rows: consecutive groups on one XCD read rows far apart, so a row
    // often comes from the Infinity Cache, and one step of even eight
    // columns does not hide that latency.  Tile sweeps of wide strips load
    // one row ahead (a deeper ring pushed the tile kernels of eight-wave
    // groups past 256 registers), and so do large samples.
    constexpr int kRowRegs = Row<CT, DIMT>::kStride * (int)sizeof(CT) / 4;
    constexpr int kAhead = (DIMT <= 8 && (K <= 2 || (!TILE && kRowRegs * K <= 64))) ? 3 : 1;
    // lane 0 prefetches up to row nA + 63 + kAhead: inside the zero rows
    // that end every packed buffer
    static_assert(kWave - 1 + kAhead <= kRowPadTail, "row prefetch runs past the buffer padding");
    Row<CT, DIMT> cur, nxt;
    Row<CT, DIMT> ring[kAhead + 1];
    if constexpr (kAhead == 1) {
        load_row<CT, DIMT>(row_ptr, 0, cur);
    } else {
#pragma unroll
        for (int k = 0; k < kAhead; ++k) load_row<CT, DIMT>(row_ptr, k, ring[k]);
    }
    row_ptr += kAhead * S;  // row kAhead - lane: the first prefetch
    // Lane 0's left operands of the next step come from one LDS read at a
    // wave-uniform address (a broadcast: no cross-lane moves, no lane
    // selection): from the ring of the previous wave of the group, or from
    // in_stage, which holds one window of the global slot (or +inf: the pad
    // column of the first strip).  Lane 63's output of every step -- the
    // strip's right boundary -- is written by that lane alone to the ring of
    // the next wave, or to out_stage when it leaves the group through global
    // memory, from where whole windows are copied out.
    const bool has_in = in_global || in_lds;
    if (!has_in) sh.in_stage[lane] = Pair2<AT>{INF, INF};
    // boundary row t + 1 sits at in_src[(t + in_add) & in_mask]: ring slot
    // (t + 1) mod 128, or in_stage slot t - wb = t mod 64
    const Pair2<AT> *const in_src = in_lds ? &sh.ring[w > 0 ? w - 1 : 0][0] : &sh.in_stage[0];
    const int in_add = in_lds ? 1 : 0;
    const int in_mask = in_lds ? kRing - 1 : kWindow - 1;
    Pair2<AT> *const out_ring = out_lds ? &sh.ring[w < G - 1 ? w : 0][0] : &sh.out_stage[0];

    // The next global window is fetched ahead when it is already published:
    // its flag is read at the start of the window's second-to-last sub-chunk
    // (the load completes behind that sub-chunk's steps), checked at the last
    // one, and the window's rows are loaded there into registers, to be
    // staged in LDS at the next window's start (their latency, too, hides
    // behind a sub-chunk).  Otherwise the window start waits for the flag.
    // (Single-strip groups, where every strip hands over through global
    // memory, wait at each window start: fetching ahead there kept the
    // window's rows in scratch memory.)
    constexpr bool kAheadFetch = G > 1;
    const int q_last = (kWindow >> sub_shift) - 1;
    uint32_t ahead_flag = 0;
    bool ahead = false;
    Pair2<AT> ahead_rows{};
    for (int t0 = 0; t0 < T_run; t0 += kSub) {
        const int q = (t0 >> sub_shift) & ((kWindow >> sub_shift) - 1);  // sub-chunk within the window
        const int wb = t0 - q * kSub;                          // window start
        const int steps = T_run - t0 < kSub ? T_run - t0 : kSub;
        const bool flagged = !TILE || s > 0;  // a tile's left column is there from the start
        if (in_global && q == 0) {
            if (ahead) {
                sh.in_stage[lane] = ahead_rows;
            } else {
                if (flagged) {
                    const uint32_t need = (uint32_t)(t0 + kWindow < nA ? t0 + kWindow : nA);
                    wait_progress<false>(in_flag, need, err);
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                }
                // rows t0 + 1 .. t0 + 64 of the boundary: lane l's row to slot l
                const int rr = t0 + 1 + lane < nA ? t0 + 1 + lane : nA;
                sh.in_stage[lane] = in_slot[rr];
            }
            ahead = false;
        }
        // (the flag's value is taken wave-uniform only where it is used, so
        // the wave does not wait for the load where it is issued)
        if (kAheadFetch && in_global && flagged && q_last > 0 && q == q_last - 1)
            ahead_flag = __hip_atomic_load(in_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (kAheadFetch && in_global && q == q_last && wb + kWindow < T_run) {
            const int nb0 = wb + kWindow;  // the next window's start
            const uint32_t need = (uint32_t)(nb0 + kWindow < nA ? nb0 + kWindow : nA);
            if (!flagged || (q_last > 0 && wave_uniform(ahead_flag) >= need)) {
                if (flagged) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                const int rr = nb0 + 1 + lane < nA ? nb0 + 1 + lane : nA;
                ahead_rows = in_slot[rr];
                ahead = true;
            }
        }
        if (in_lds) {
            // the rows this sub-chunk reads, t0 + 1 .. t0 + kSub, are in the ring
            const uint32_t need = (uint32_t)(t0 + kSub < nA ? t0 + kSub : nA);
            wait_progress<true>(&sh.prod[w - 1], need, err);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        }
        if (out_lds) {
            // this sub-chunk writes rows up to t0 + steps - 64 into the ring,
            // over the slots of rows up to 128 earlier: the next wave must
            // have read those
            const int last_w = t0 + steps - kWave;
            if (last_w > kRing) wait_progress<true>(&sh.cons[w + 1], (uint32_t)(last_w - kRing), err);
        }

        // One step: sweep row t - lane with `use`, prefetch row t + kAhead -
        // lane into `fill`.  Steps rotate the row buffers, so the prefetched
        // row never has to be copied.  SP (tile sweeps): this sub-chunk holds
        // a step where top-row cells enter or boundary cells leave; the other
        // sub-chunks run without testing for them at every step.
        auto step = [&]<bool SP>(int i, Row<CT, DIMT> &use, Row<CT, DIMT> &fill) {
            const int t = t0 + i;
            load_row<CT, DIMT>(row_ptr, 0, fill);  // row t + kAhead - lane
            row_ptr += S;
            // boundary row t + 1, which lane 0 meets at the next step (read
            // before the cells so that its latency hides behind them)
            const Pair2<AT> nb = in_src[(t + in_add) & in_mask];

            AT left = sh_l, xl;
            if constexpr (TILE) {
                if constexpr (DIRS) {
                    uint64_t code;
                    if constexpr (REC == kRecTwed)
                        code = lane_row_dirs<CT, AT, DIMT, PM, K>(L, use, left, sh_xo, xl, ca.nu, ca.p, ca.invp);
                    else
                        code = lane_row_sibling<CT, AT, DIMT, PM, K, REC, true>(L, use, left, sh_xo, xl, ca.p,
                                                                                ca.invp);
                    store_dirs<K>(io.dirs + (((size_t)s * (size_t)T + (size_t)t) * kWave + lane) * K, code);
                } else {
                    if constexpr (REC == kRecTwed)
                        lane_row<CT, AT, DIMT, PM, K>(L, use, left, sh_xo, xl, ca.nu, ca.p, ca.invp, beta);
                    else
                        (void)lane_row_sibling<CT, AT, DIMT, PM, K, REC, false>(L, use, left, sh_xo, xl, ca.p,
                                                                                ca.invp);
                }
              if constexpr (SP) {
                // the lane sits on row 0: its top-row cells replace the pad state
                if (io.top != nullptr && t < kWave) {
                    const bool own = t == lane;
#pragma unroll
                    for (int j = 0; j < K; ++j) {
                        const Pair2<AT> v = io.top[c0 + j <= nB ? c0 + j : nB];
                        L.up[j] = own ? v.dp : L.up[j];
                        L.xp[j] = own ? v.x : L.xp[j];
                    }
                    left = own ? L.up[K - 1] : left;
                    xl = own ? L.xp[K - 1] : xl;
                }
                // rows stored at this step (every lane stores; lanes without
                // such a row write the dummy cells)
                const bool cap_last = io.bottom != nullptr && nA >= t - (kWave - 1) && nA <= t;
                int kr = 0;
                if (io.ckrow != nullptr) {
                    const int m = t / io.ck_rows * io.ck_rows;
                    kr = (m >= io.ck_rows && m >= t - (kWave - 1) && m < nA) ? m : 0;
                }
                if (cap_last || kr > 0) {
                    const int r = t - lane;
                    const bool own_last = cap_last && r == nA;
                    const bool own = own_last || (kr > 0 && r == kr);
                    Pair2<AT> *base = own_last ? io.bottom
                                               : io.ckrow + (size_t)(kr > 0 ? kr / io.ck_rows - 1 : 0) *
                                                                (size_t)(nB + 1);
#pragma unroll
                    for (int j = 0; j < K; ++j) {
                        Pair2<AT> *dst = (own && c0 + j <= nB) ? base + (c0 + j) : io.dummy + lane * K + j;
                        *dst = Pair2<AT>{L.up[j], L.xp[j]};
                    }
                }
                // column nB (lane lstar, column jstar of the last strip)
                if (io.right != nullptr && result_strip && t - lstar >= 1 && t - lstar <= nA) {
                    AT dp = L.up[0], x = L.xp[0];
#pragma unroll
                    for (int j = 1; j < K; ++j) {
                        if (j == jstar) {
                            dp = L.up[j];
                            x = L.xp[j];
                        }
                    }
                    io.right[t - lstar] = Pair2<AT>{lane_value(dp, lstar), lane_value(x, lstar)};
                }
              }
            } else {
                lane_row<CT, AT, DIMT, PM, K>(L, use, left, sh_xo, xl, ca.nu, ca.p, ca.invp, beta);
            }

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
            sh_xo = sh_x;
            sh_l = shift_in(left, nb.dp);
            sh_x = shift_in(xl, nb.x);
            if (has_out && lane == kWave - 1) {
                // Lane 63 holds row t - 63 of the strip's right boundary.
                // Rows -63 .. 0 of the first 64 steps land in the slots of
                // rows 65 .. 128, which are written again with those rows
                // (steps 128 .. 191) before anyone may read them.
                out_ring[(t - (kWave - 1)) & (kRing - 1)] = Pair2<AT>{left, xl};
            }
        };
        auto run = [&]<bool SP>() {
            int i = 0;
            if constexpr (kAhead == 1) {
                for (; i + 1 < steps; i += 2) {
                    step.template operator()<SP>(i, cur, nxt);
                    step.template operator()<SP>(i + 1, nxt, cur);
                }
                if (i < steps) {
                    step.template operator()<SP>(i, cur, nxt);
                    cur = nxt;
                }
            } else {
                // ring[k] holds row t + k (k < kAhead) at the start of each
                // run of kAhead + 1 steps; sub-chunks are multiples of that
                // run except at the end of the sweep, where the ring is
                // shifted step by step
                constexpr int R = kAhead + 1;
                for (; i + R <= steps; i += R) {
#pragma unroll
                    for (int k = 0; k < R; ++k)
                        step.template operator()<SP>(i + k, ring[k], ring[(k + kAhead) % R]);
                }
                for (; i < steps; ++i) {
                    step.template operator()<SP>(i, ring[0], ring[kAhead]);
#pragma unroll
                    for (int k = 0; k < kAhead; ++k) ring[k] = ring[k + 1];
                }
            }
        };
        if constexpr (TILE) {
            // does a lane reach row 0 (top row), nA (bottom row) or a
            // checkpoint row in this sub-chunk, or is this the strip that
            // hands out column nB at every step?
            const int r_lo = t0 - (kWave - 1), r_hi = t0 + steps - 1;  // rows the lanes touch
            bool sp = (io.top != nullptr && t0 < kWave) || (io.right != nullptr && result_strip) ||
                      (io.bottom != nullptr && nA >= r_lo && nA <= r_hi);
            if (io.ckrow != nullptr) {
                // the two multiples of ck_rows (>= 64) at or below r_hi cover
                // the at most 95 rows of the range
                const int m = r_hi / io.ck_rows * io.ck_rows;
                for (int q = m; q >= m - io.ck_rows; q -= io.ck_rows)
                    sp = sp || (q >= io.ck_rows && q >= r_lo && q < nA);
            }
            if (sp) run.template operator()<true>();
            else run.template operator()<false>();
        } else {
            run.template operator()<false>();
        }

        const int tend = t0 + steps;        // steps done so far
        const int last = tend - kWave;      // last boundary row complete
        if (in_lds) {
            // rows up to tend have been read
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __hip_atomic_store(&sh.cons[w], (uint32_t)(tend < nA ? tend : nA), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        if (out_lds && last >= 1) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __hip_atomic_store(&sh.prod[w], (uint32_t)(last < nA ? last : nA), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        if (out_global && (q == (kWindow >> sub_shift) - 1 || tend >= T)) {
            // the window's rows, tend - 127 + lane for lanes kWave - (tend -
            // wb) .. 63, from out_stage to the slot (lanes without a row of
            // this window write slot row 0, which no consumer reads: no
            // lane-conditional branch)
            const int ws = tend - wb;
            int r = tend - 2 * kWave + 1 + lane;
            r = (lane >= kWave - ws && r >= 1 && r <= nA) ? r : 0;
            out_slot[r] = sh.out_stage[r > 0 ? (r & (kRing - 1)) : kRing];
            if (last >= 1) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                __hip_atomic_store(out_flag, (uint32_t)(last < nA ? last : nA), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        if constexpr (TILE) {
            // a checkpoint column at this strip's right edge, window by window
            if (ck_col != nullptr && (q == (kWindow >> sub_shift) - 1 || tend >= T)) {
                const int ws = tend - wb;
                const int r = tend - 2 * kWave + 1 + lane;
                const bool ok = lane >= kWave - ws && r >= 1 && r <= nA;
                *(ok ? ck_col + r : io.dummy + lane) = out_ring[ok ? (r & (kRing - 1)) : kRing];
            }
        }
    }
    if (result_strip) {
        // DP(nA, nB): column jstar of lane lstar after its sweep of row nA
        // (wave-uniform; every lane stores the same value)
        AT res = L.up[0];
#pragma unroll
        for (int j = 1; j < K; ++j)
            if (j == jstar) res = L.up[j];
        res = lane_value(res, lstar);
        if (kShifted<AT>) res = (AT)((double)res + (double)beta * (double)(nA + nB));
        if (load_progress(err) != 0u) res = __builtin_nan("");
        out[0] = res;
    }
}

// Persistent workgroups of G waves.  A workgroup claims a group g of G
// consecutive strips from an atomic ticket (wave 0 claims, LDS broadcasts),
// so the group it waits for has always been claimed by a running workgroup:
// no co-residency assumption, no deadlock.  Inside the group, wave w sweeps
// strip g*G + w: body(w, g, s).
//
// Two global slots suffice: group g+2 writes row r of its boundary only
// after group g+1 has read row r from the slot both use (it reads a row
// before its own last wave can produce that row).
template <typename AT, int G, typename Body>
__device__ __forceinline__ void claim_groups(GroupShared<AT, G> &sh, uint32_t *ticket, int nStrips, Body &&body)
{
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int nGroups = (nStrips + G - 1) / G;
    for (;;) {
        __syncthreads();  // the previous group is done with the LDS
        // Every thread takes part in the claim and only thread 0 counts, so
        // there is no branch around the atomic; wave 0's lane-0 value is the
        // group, published through LDS.
        const uint32_t mine = atomicAdd(ticket, threadIdx.x == 0 ? 1u : 0u);
        __hip_atomic_store(&sh.ticket[w], (uint32_t)__builtin_amdgcn_readlane((int)mine, 0), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_store(&sh.prod[w], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_store(&sh.cons[w], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __syncthreads();
        const int g = (int)__hip_atomic_load(&sh.ticket[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (g >= nGroups) break;
        const int s = g * G + w;
        if (s < nStrips) body(w, g, s);
    }
}

// Strips of one width: strip s starts at column 1 + s*64*K.
template <typename CT, typename AT, int DIMT, int PM, int K, int G, bool DUMP, bool TILE, int REC = kRecTwed,
          bool DIRS = false>
__global__ __launch_bounds__(kWave * G) void wavefront_kernel(const CT *__restrict__ rowsA,
                                                             const CT *__restrict__ rowsB, int nA, int nB,
                                                             CostArgs<CT> ca, Pair2<AT> *bnd, uint32_t *flags,
                                                             uint32_t *ticket, uint32_t *err, int nStrips,
                                                             const CT *beta_ptr, AT *out, AT *dump, int sub_shift,
                                                             TileIO<AT> io)
{
    __shared__ GroupShared<AT, G> sh;
    const CT beta = kShifted<AT> ? beta_ptr[0] : CT(0);
    claim_groups<AT, G>(sh, ticket, nStrips, [&](int w, int g, int s) {
        sweep_strip<CT, AT, DIMT, PM, K, G, DUMP, TILE, REC, DIRS>(sh, w, g, s, s * kWave * K, rowsA, rowsB, nA, nB,
                                                                   ca, bnd, flags, err, nStrips, beta, out, dump,
                                                                   sub_shift, io);
    });
}

// Strips of two widths: strips 0 .. s1-1 hold K columns per lane, the rest
// K2 < K.  A strip starts one pipeline lag (in its own steps) after the one
// before it and runs nA + 63 steps, so with every strip resident the sweep
// ends when the last strip does: narrower strips at the end of the row
// finish sooner, and the spare workgroup slots that uniform strips would
// leave idle take the extra strips.  Cells and their arithmetic do not
// depend on the strip widths.
template <typename CT, typename AT, int DIMT, int PM, int K, int K2, int G>
__global__ __launch_bounds__(kWave * G) void wavefront_mixed_kernel(const CT *__restrict__ rowsA,
                                                                   const CT *__restrict__ rowsB, int nA, int nB,
                                                                   CostArgs<CT> ca, Pair2<AT> *bnd, uint32_t *flags,
                                                                   uint32_t *ticket, uint32_t *err, int nStrips,
                                                                   int s1, const CT *beta_ptr, AT *out,
                                                                   int sub_shift)
{
    static_assert(K2 < K, "the second width is the narrower one");
    __shared__ GroupShared<AT, G> sh;
    const CT beta = kShifted<AT> ? beta_ptr[0] : CT(0);
    claim_groups<AT, G>(sh, ticket, nStrips, [&](int w, int g, int s) {
        if (s < s1)
            sweep_strip<CT, AT, DIMT, PM, K, G, false, false, kRecTwed, false>(
                sh, w, g, s, s * kWave * K, rowsA, rowsB, nA, nB, ca, bnd, flags, err, nStrips, beta, out,
                nullptr, sub_shift, TileIO<AT>{});
        else
            sweep_strip<CT, AT, DIMT, PM, K2, G, false, false, kRecTwed, false>(
                sh, w, g, s, s1 * kWave * K + (s - s1) * kWave * K2, rowsA, rowsB, nA, nB, ca, bnd, flags, err,
                nStrips, beta, out, nullptr, sub_shift, TileIO<AT>{});
    });
}

template <typename CT, typename AT, int DIMT, int PM, int K, int G, bool TILE, int REC = kRecTwed,
          bool DIRS = false>
int occupancy_kg()
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, wavefront_kernel<CT, AT, DIMT, PM, K, G, false, TILE, REC, DIRS>,
                                                     kWave * G, 0) != hipSuccess)
        return 0;
    return blocks;
}

template <typename CT, typename AT, int DIMT, int PM, int K, int G, bool TILE, int REC = kRecTwed,
          bool DIRS = false>
size_t scratch_kg()
{
    hipFuncAttributes attr{};
    if (hipFuncGetAttributes(&attr, reinterpret_cast<const void *>(wavefront_kernel<CT, AT, DIMT, PM, K, G, false, TILE, REC, DIRS>)) !=
        hipSuccess)
        return (size_t)-1;
    return attr.localSizeBytes;
}

template <typename CT, typename AT, int DIMT, int PM, int K, bool TILE>
int occupancy_k(int G)
{
    switch (G) {
    case 1: return occupancy_kg<CT, AT, DIMT, PM, K, 1, TILE>();
    case 4: return occupancy_kg<CT, AT, DIMT, PM, K, 4, TILE>();
    case 8: return occupancy_kg<CT, AT, DIMT, PM, K, 8, TILE>();
    default: return 0;
    }
}

}  // namespace twed

// twed_kernels.h -- host-side launch interface of the TWED kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace twed {

// Precision of one launch (resolved: no AUTO here).
enum Prec : int { kF64 = 0, kF32 = 1, kF32Acc64 = 2 };

// Recurrence of a strip sweep: TWED, or one of its siblings (dynamic time
// warping, edit distance, indel distance; lane_row_sibling in twed_device.h).
enum Rec : int { kRecTwed = 0, kRecDtw = 1, kRecEdit = 2, kRecIndel = 3 };

// Sample dimensions the kernels are compiled for; a call with dim d runs the
// smallest compiled DIMT >= d with the extra components zero.
int dimt_for(int dim);
// Elements per packed row for (precision, DIMT).
int row_stride(Prec prec, int dimt);
inline size_t cost_size(Prec p) { return p == kF64 ? 8 : 4; }
inline size_t acc_size(Prec p) { return p == kF32 ? 4 : 8; }

struct CostParams {
    double nu, lambda, p;
    int dim;   // real dimension
    int dimt;  // compiled dimension
    int pm;    // PMode
};

// Zero rows kept before and after every packed row buffer.  A sweep lane l
// reads row t - l at step t (t < n + 64), and the pair sweep prefetches rows
// up to kMaxRowAhead steps early, so the buffer ends with that many more.
constexpr int kRowPad = 64;
constexpr int kMaxRowAhead = 8;
constexpr int kRowPadTail = kRowPad + kMaxRowAhead;
// Bytes of a packed row buffer holding `rows` rows plus its padding.
inline size_t rows_bytes(Prec prec, int dimt, int64_t rows)
{
    return (size_t)(rows + kRowPad + kRowPadTail) * (size_t)row_stride(prec, dimt) * cost_size(prec);
}

// Writes packed rows (zero pad row first) and deletion costs for nSeries
// series.  `off` (device, nSeries+1 sample offsets) may be null for a single
// series of n samples.  Row block of series s starts at row off[s] + s.
// `rows` points after the front padding of a buffer of total_rows rows
// (rows_bytes); the padding rows are zeroed too.  Also zeroes `zero_words`
// 32-bit words at `zero_ptr` (may be null).  With first_prev (a single
// series only) X and T start one sample into a longer series: the deletion
// cost of row 1 is taken against the sample before X[0] instead of the pad.
// T may be null (every timestamp 0: the sibling recurrences use none).
hipError_t launch_stage(Prec prec, const CostParams &cp, const void *X, const void *T,
                        const int64_t *off, int64_t nSeries, int64_t n_single, int64_t max_len,
                        int64_t total_rows, void *rows, uint32_t *zero_ptr, int64_t zero_words, hipStream_t st,
                        bool first_prev = false);

// Single pair, persistent wave pipeline over strips of 64*K columns.
struct WavefrontArgs {
    const void *rowsA, *rowsB;
    int64_t nA, nB;
    void *bnd;          // 2 * (nA+1) pairs (dp, x) of the accumulator type
    uint32_t *flags;    // nStrips words, zero
    uint32_t *ticket;   // two words, zero: ticket, then the wait-timeout error word
    int64_t nStrips;
    const void *beta;   // one cost element: FP32 cost offset (read in FP32 mode)
    void *out;          // one accumulator element
    void *dump;         // optional (nA+1)*(nB+1) accumulators
    int grid;           // workgroups
    int group;          // waves (consecutive strips) per workgroup: 1, 4 or 8
    int sub_shift;      // in-group handoff every 1 << sub_shift rows (3, 4 or 5)
    int s1;             // two strip widths (launch_wavefront_mixed): strips before s1 hold K columns per lane
};
hipError_t launch_wavefront(Prec prec, const CostParams &cp, int K, const WavefrontArgs &a, hipStream_t st);
// Strips of two widths (wavefront_mixed.hip): layout m sweeps strips 0 .. a.s1-1
// with kMixedLayouts[m].wide columns per lane and the others with .narrow,
// in workgroups of .group strips.
struct MixedLayout {
    int wide, narrow, group;
};
constexpr MixedLayout kMixedLayouts[] = {{8, 7, 8}};
constexpr int kNumMixedLayouts = 1;
// True if the two-width sweep of this layout is compiled for this
// (precision, dimension, distance).
bool wavefront_mixed_compiled(Prec prec, const CostParams &cp, int layout);
hipError_t launch_wavefront_mixed(Prec prec, const CostParams &cp, int layout, const WavefrontArgs &a,
                                  hipStream_t st);
int wavefront_mixed_max_workers(Prec prec, const CostParams &cp, int layout);
size_t wavefront_mixed_scratch_bytes(Prec prec, const CostParams &cp, int layout);
// FP32 pairs longer than this get a per-diagonal cost offset.
constexpr int64_t kOffsetMinLength = 4096;
// Writes the FP32 cost offset of one staged pair to beta (one cost element).
hipError_t launch_offset(Prec prec, const CostParams &cp, const void *rowsA, int64_t nA, const void *rowsB,
                         int64_t nB, void *beta, hipStream_t st);
// Resident workgroups of G waves for one wavefront instantiation.
int wavefront_max_workers(Prec prec, const CostParams &cp, int K, int G);
// Per-lane scratch (register spill) bytes of one wavefront instantiation.
size_t wavefront_scratch_bytes(Prec prec, const CostParams &cp, int K, int G);

// Boundaries and extra outputs of a tile sweep (device pointers to (DP, X)
// cell pairs of FP64; any may be null).  See TileIO in wavefront_impl.h.
struct TileArgs {
    const void *top;    // row 0 of the block, columns 0..nB (null: pad row)
    const void *left;   // column 0 of the block, rows 0..nA (null: pad column)
    void *bottom;       // row nA, columns 0..nB
    void *right;        // column nB, rows 0..nA
    void *ckrow;        // rows ck_rows, 2*ck_rows, ... < nA, nB + 1 cells each
    void *ckcol;        // columns ck_cols, 2*ck_cols, ... < nB, nA + 1 cells each
    void *dummy;        // 512 cells of scratch
    uint8_t *dirs;      // moves, nStrips * (nA + 64) * 64 * K bytes (recording kernels, K = 1)
    int ck_rows;        // >= 64
    int ck_cols;        // a multiple of the strip width 64*K
};
// The tile sweep (FP64 accumulators: kF64 or kF32Acc64).  `a` as for the
// pair sweep, with rowsA / rowsB at the rows of the block's row 0 / column 0.
hipError_t launch_tile(Prec prec, const CostParams &cp, int K, const WavefrontArgs &a, const TileArgs &t,
                       hipStream_t st);
size_t tile_scratch_bytes(Prec prec, const CostParams &cp, int K, int G);
int tile_max_workers(Prec prec, const CostParams &cp, int K, int G);
// Column 0 of the output rows and row 0 of the output columns (copied from
// the inputs or set to the +inf pad); launched after every tile sweep.
hipError_t launch_tile_edges(int64_t nA, int64_t nB, const TileArgs &t, hipStream_t st);
// The tile sweep on a sibling recurrence (dp.hip; rec: 1 DTW, 2 edit
// distance, 3 indel distance), strips of K = 1, 2 or 8 columns per lane,
// groups of G = 1 or 8 strips; other configurations return hipErrorInvalidValue /
// (size_t)-1 / 0.
hipError_t launch_dp(int rec, Prec prec, const CostParams &cp, int K, const WavefrontArgs &a, const TileArgs &t,
                     hipStream_t st);
// Tile sweeps that record moves (t.dirs set; tile_dirs.hip): any recurrence,
// K = 1 only, G = 1, 4 or 8.  launch_tile / launch_dp with t.dirs set call
// these.
hipError_t launch_tile_dirs(Prec prec, const CostParams &cp, int K, const WavefrontArgs &a, const TileArgs &t,
                            hipStream_t st);
hipError_t launch_rec_dirs(int rec, Prec prec, const CostParams &cp, int K, const WavefrontArgs &a, const TileArgs &t,
                           hipStream_t st);
size_t rec_dirs_scratch_bytes(int rec, Prec prec, const CostParams &cp, int K, int G);
int rec_dirs_max_workers(int rec, Prec prec, const CostParams &cp, int K, int G);
size_t dp_scratch_bytes(int rec, Prec prec, const CostParams &cp, int K, int G);
int dp_max_workers(int rec, Prec prec, const CostParams &cp, int K, int G);

// Path read-back (path.hip).  st holds {r, c, cells written, status}.
hipError_t launch_walk_init(int64_t *st, int64_t nA, int64_t nB, hipStream_t s);
// Follows the moves of the block (nAt x nBt cells) whose row 0 / column 0
// are global row r0 / column c0 (dirs in the tile sweep's order with strip
// width 64*K and T = nAt + 64 steps per strip) until the walk leaves it.
hipError_t launch_walk(const uint8_t *dirs, int64_t r0, int64_t c0, int64_t nAt, int64_t nBt, int K, int64_t T,
                       int64_t *st, int64_t *rev, int64_t cap, bool free_edges, hipStream_t s);
// n + 1 (DP, X) cells (i, i), i = 0..n: the boundary of edit / indel distances.
hipError_t launch_index_cells(void *cells, int64_t n, hipStream_t s);
// out[0] = (nA + nB - out[0]) / 2: the LCS length from the indel distance.
hipError_t launch_lcs_finish(double *out, int64_t nA, int64_t nB, hipStream_t s);
// Zeroes n 32-bit words (a kernel, so that it can be captured in a graph).
hipError_t launch_zero32(uint32_t *p, int64_t n, hipStream_t s);
// Reverses the st[2] cells of `path` in place and writes the count to len.
hipError_t launch_order(const int64_t *st, int64_t *path, int64_t *len, int64_t cap, hipStream_t s);

// Fills row 0 and column 0 of a dump matrix (0 at the corner, +inf elsewhere).
hipError_t launch_dump_border(Prec prec, void *dump, int64_t nA, int64_t nB, hipStream_t st);

// One launch per anti-diagonal over three diagonal vectors in device memory.
struct DiagonalArgs {
    const void *rowsA, *rowsB;
    int64_t nA, nB;
    void *z[3];         // three DP diagonals, nB+1 accumulators each
    void *x[3];         // three X = DP + e diagonals
    const void *beta;   // one cost element: FP32 cost offset (read in FP32 mode)
    void *out;
    void *dump;
};
hipError_t launch_diagonal(Prec prec, const CostParams &cp, const DiagonalArgs &a, hipStream_t st);

// Batched pairs: one wave per pair, shorter series across the lanes.
enum BatchMode : int { kSymmetric = 0, kRect = 1, kPairList = 2 };
struct BatchArgs {
    const void *rowsX, *rowsY;   // packed rows (with pad rows)
    const int64_t *offX, *offY;  // device sample offsets (nX+1, nY+1)
    const int32_t *order;        // symmetric: series order (longest first), nX entries
    const int64_t *pairs;        // pair-list mode
    int64_t nX, nY, nItems;
    int mode;
    void *D;
    uint32_t *ticket;            // one word, zero
    int grid;
    int chunk;                   // consecutive items per ticket (0 or 1: one)
    int64_t item0;               // first item of this launch (items item0 .. nItems-1)
    int kclass;                  // kernel of the pair widths swept (BatchClass)
};
// Pair widths (columns per lane K) a batch kernel sweeps; pairs outside its
// range are left to another launch.  One kernel for every width holds the
// registers of the widest, which limits it to two waves per SIMD; narrower
// kernels fit more.
enum BatchClass : int {
    kBatchAll = 0,     // K = 1 .. KMAX
    kBatchNarrow = 1,  // K = 1 .. min(8, KMAX)
    kBatchWide = 2     // K = 9 .. KMAX (one-component samples only)
};
constexpr int kBatchNarrowMax = 8;
constexpr int kWaveLanes = 64;  // lanes of a wave (gfx950 runs wave64)
hipError_t launch_batch(Prec prec, const CostParams &cp, const BatchArgs &a, hipStream_t st);
int batch_kmax(int dimt);
// One query of at most kLaneMaxQuery samples (staged rows rowsQ) against nY
// series: one lane per pair, D[j] = TWED(query, Y_j); ticket zeroed.  The
// series are the staged rows rowsY, or, with Yraw non-null, the caller's
// arrays Yraw (dim components per sample) and TYraw read directly.
constexpr int kLaneMaxQuery = 32;
hipError_t launch_batch_lane(Prec prec, const CostParams &cp, const void *rowsQ, int nQ, const void *rowsY,
                            const void *Yraw, const void *TYraw, const int64_t *offY, int64_t nY, void *D,
                            uint32_t *ticket, int grid, hipStream_t st);
int batch_max_workers(Prec prec, const CostParams &cp, int kclass = kBatchAll);
hipError_t launch_batch_diag_zero(Prec prec, void *D, int64_t n, hipStream_t st);
// dst[0] = src[0] on the device (accumulator type of prec).
hipError_t launch_copy_one(Prec prec, const void *src, void *dst, hipStream_t st);
// dst[i] = (double)src[i] for n floats.
hipError_t launch_widen(const float *src, double *dst, int64_t n, hipStream_t st);

}  // namespace twed

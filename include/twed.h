/*
 * twed.h -- C ABI of libtwed, Time Warp Edit Distance on AMD Instinct MI355X
 * (gfx950).
 *
 * The distance is the one defined in the paper's section "Time Warp Edit
 * Distance" (steps 1-6) with Marteau's cost terms: for series A (nA samples
 * of `dim` components, timestamps TA) and B (nB samples, TB), zero-padded at
 * index 0,
 *
 *   del_A(i)  = d(A'_i, A'_{i-1}) + nu*|TA'_i - TA'_{i-1}| + lambda
 *   del_B(j)  = d(B'_j, B'_{j-1}) + nu*|TB'_j - TB'_{j-1}| + lambda
 *   mat(i,j)  = d(A'_i, B'_j) + d(A'_{i-1}, B'_{j-1})
 *               + nu*(|TA'_i - TB'_j| + |TA'_{i-1} - TB'_{j-1}|)
 *   DP[0][0] = 0, DP[i][0] = DP[0][j] = +inf,
 *   DP[i][j] = min(DP[i-1][j] + del_A(i), DP[i][j-1] + del_B(j),
 *                  DP[i-1][j-1] + mat(i,j)),        TWED = DP[nA][nB],
 *
 * with d the Lp distance of degree p including its 1/p root (section
 * "cuTWED Implementation Remarks").  The library evaluates the DP by the
 * anti-diagonal band of the section "Improved Time Warp Edit Distance":
 * cell (row, col) lies on diagonal row+col at index col (Eq. (1), (2)); every
 * cell of a diagonal depends only on the two previous diagonals and is
 * updated in parallel, and only O(nA + nB) state is kept.
 *
 * Conventions for every entry point:
 *  - Array arguments named as device arrays are device pointers owned by the
 *    caller; the library never allocates or frees device memory.  Scratch
 *    memory comes from the caller's `workspace` (device, 256-byte aligned),
 *    whose size is given by the matching *_workspace_size() call.
 *  - Work is enqueued on `stream` (NULL = the default stream) and is
 *    asynchronous: results are valid once the stream has been synchronised.
 *  - Argument errors are detected on the host before any HIP call and
 *    returned synchronously; outputs are then left untouched.
 *  - A device fault is sticky in HIP: it surfaces as TWED_ERR_DEVICE from
 *    the next call or from twed_stream_check().
 *  - Calls are thread-safe when concurrent calls use distinct workspaces.
 *  - Inputs containing NaN give unspecified results.  Timestamps need not be
 *    sorted; the cost uses their absolute differences.
 */
#ifndef TWED_H_
#define TWED_H_

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TWED_OK = 0,
    TWED_ERR_INVALID = 1,     /* bad argument (null pointer, size < 1, nu < 0, ...) */
    TWED_ERR_UNSUPPORTED = 2, /* valid but not supported (dim too large, ...) */
    TWED_ERR_WORKSPACE = 3,   /* workspace missing, too small or misaligned */
    TWED_ERR_DEVICE = 4       /* a HIP call failed (possibly an earlier fault) */
} twed_status;

/* Arithmetic of a call (the paper's experiments are FP64; FP32 halves storage). */
typedef enum {
    TWED_F64 = 0,       /* f64 inputs, f64 costs, f64 accumulators, f64 results */
    TWED_F32 = 1,       /* f32 inputs, f32 costs, f32 accumulators, f32 results */
    TWED_F32_ACC64 = 2, /* f32 inputs, f32 costs, f64 accumulators, f64 results */
    TWED_AUTO = 3       /* f32 inputs, f64 results: F32_ACC64 when the longest
                           series of the call exceeds acc64_threshold samples,
                           otherwise F32 (whose result is widened to f64) */
} twed_precision;

/* How a single pair is swept. */
typedef enum {
    TWED_ALGO_AUTO = 0,      /* the library's choice (currently WAVEFRONT) */
    TWED_ALGO_WAVEFRONT = 1, /* persistent wave pipeline: each wave carries a
                                64-cell segment of the three-diagonal band in
                                registers across a strip of columns */
    TWED_ALGO_DIAGONAL = 2   /* one kernel launch per anti-diagonal with three
                                diagonal vectors in device memory, as in the
                                paper's implementation remarks (slow for long
                                series; kept as a cross-check) */
} twed_algo;

#define TWED_MAX_DIM 32

typedef struct {
    double nu;               /* stiffness, >= 0 and finite */
    double lambda;           /* deletion penalty, >= 0 and finite */
    double p;                /* Lp degree, >= 1 and finite */
    int32_t dim;             /* components per sample, 1..TWED_MAX_DIM */
    int32_t precision;       /* twed_precision */
    int32_t algo;            /* twed_algo (single pairs only) */
    int32_t strip_k;         /* 0 = auto; else columns per lane of the
                                wavefront sweep (1, 2, 4 or 8; 1 or 2 when
                                dim > 16) */
    int64_t acc64_threshold; /* TWED_AUTO switch-over length; <= 0 means 100000 */
} twed_params;

/* Fills *prm with nu = 0.001, lambda = 1, p = 1, dim = 1, TWED_F64, auto
   algorithm and threshold. */
void twed_params_default(twed_params *prm);

/* ---- one pair -------------------------------------------------------------
 * A: device, nA*dim samples, row-major (sample-major, components fastest);
 * TA: device, nA timestamps; likewise B, TB.  Element type: double for
 * TWED_F64, float otherwise.
 * out: device, one element: float for TWED_F32, double otherwise.
 * Errors: TWED_ERR_INVALID for nA < 1, nB < 1, null pointers, dim < 1,
 * nu < 0, lambda < 0, p < 1, non-finite parameters or an unknown precision /
 * algorithm; TWED_ERR_UNSUPPORTED for dim > TWED_MAX_DIM or nA, nB >= 2^31;
 * TWED_ERR_WORKSPACE if ws_bytes < twed_pair_workspace_size(...). */
size_t twed_pair_workspace_size(int64_t nA, int64_t nB, const twed_params *prm);

twed_status twed_pair(const void *A, const void *TA, int64_t nA,
                      const void *B, const void *TB, int64_t nB,
                      const twed_params *prm, void *out,
                      void *workspace, size_t ws_bytes, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation as twed_pair, bitwise equal to it, with no workspace argument.
 * Its scratch memory is a fixed array of TWED_PAIR_NOALLOC_SCRATCH_BYTES
 * bytes inside the library, one per GPU, held until the process ends; the
 * call allocates nothing (no hipMalloc, hipFree or allocating library
 * routine).  The first call on a device looks up that device's copy of the
 * array (hipGetSymbolAddress), so make the device current as for any HIP call.
 * Every call on one GPU shares its array, and the staging kernel clears what
 * must start at zero: calls on one GPU whose work overlaps (different streams
 * without ordering, other host threads) race and give wrong results; calls
 * ordered on one stream are safe.  Arguments and errors as twed_pair, plus
 * TWED_ERR_UNSUPPORTED (with a message naming the size) when the pair needs
 * more than TWED_PAIR_NOALLOC_SCRATCH_BYTES, i.e. when
 * twed_pair_workspace_size(nA, nB, prm) exceeds it.  Equal lengths that fit:
 * up to 698,495 samples (1-D F64), 1,396,183 (1-D F32), 523,927 (3-D F64 or
 * 8-D F32_ACC64). */
#define TWED_PAIR_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

twed_status twed_pair_noalloc(const void *A, const void *TA, int64_t nA,
                              const void *B, const void *TB, int64_t nB,
                              const twed_params *prm, void *out, hipStream_t stream);

/* Same as twed_pair, and also writes every DP cell to `dp` (device,
 * (nA+1)*(nB+1) elements of the result type, row-major, row stride nB+1,
 * row 0 and column 0 included).  Meant for validation on small problems:
 * the caller owns `dp`; no size limit is imposed beyond memory.  The
 * wavefront sweep runs with strips of at most 2 columns per lane here
 * (strip_k 3..8 gives TWED_ERR_UNSUPPORTED); TWED_AUTO is not accepted. */
twed_status twed_pair_matrix(const void *A, const void *TA, int64_t nA,
                             const void *B, const void *TB, int64_t nB,
                             const twed_params *prm, void *out, void *dp,
                             void *workspace, size_t ws_bytes, hipStream_t stream);

/* Measures the single-pair sweep configurations (strip width = columns per
 * lane, strips per workgroup) on this pair -- a prefix of A of up to 262,144
 * samples against all of B -- and remembers the fastest for this precision,
 * dimension, distance and nB in a host-side, process-wide cache; later
 * twed_pair calls with strip_k == 0 and the same key use it.  Arguments as
 * twed_pair (the same workspace size); the chosen values are written to
 * *strip_k and *group when those are not NULL.  Synchronises `stream`.
 * Results never depend on the configuration (every cell is evaluated with
 * the same arithmetic); only the time does.  Errors as twed_pair, plus
 * TWED_ERR_INVALID for algo == TWED_ALGO_DIAGONAL. */
twed_status twed_pair_tune(const void *A, const void *TA, int64_t nA,
                           const void *B, const void *TB, int64_t nB,
                           const twed_params *prm, void *workspace, size_t ws_bytes,
                           hipStream_t stream, int32_t *strip_k, int32_t *group);

/* The strip layout a twed_pair call with these arguments would sweep (no
 * device work; the device must be current).  Strips of *strip_k columns per
 * lane in workgroups of *group strips; when uniform strips would leave
 * workgroup slots of the device empty, the first *wide_strips strips hold
 * *strip_k columns per lane and the rest *strip_k - 1 (*wide_strips is 0
 * for uniform strips); *strips is the strip count.  A strip starts one
 * pipeline lag after its left neighbour (section "Improved Time Warp Edit
 * Distance": cell (r, c) needs the cell on its left), so narrower strips on
 * the right end sooner.  Any output pointer may be NULL.  Errors: as
 * twed_pair's argument checks, TWED_ERR_INVALID for algo ==
 * TWED_ALGO_DIAGONAL. */
twed_status twed_pair_config(int64_t nA, int64_t nB, const twed_params *prm, int32_t *strip_k,
                             int32_t *group, int64_t *wide_strips, int64_t *strips);

/* Empties the tuning cache (single-pair and batch choices). */
void twed_tune_clear(void);

/* ---- blocks of the DP matrix (section "Improved Time Warp Edit Distance":
 * the band of live cells is the whole state of the program, so a sweep can
 * stop at any row or column and resume from it) ------------------------------
 * A cell of the state: dp = DP(i, j) and x = DP(i, j) + e(i, j), where
 * e(i, j) = d(A'_i, B'_j) + nu*|TA'_i - TB'_j| (padded samples as in
 * twed_pair), the half of a match cost that the match into (i+1, j+1) takes
 * from row i.  Row 0 and column 0 are the pad: DP(0, 0) = 0, X(0, 0) = 0 and
 * +inf elsewhere on them. */
typedef struct {
    double dp;
    double x;
} twed_cell;

/* Sweeps the block of rows r0+1..r1 and columns c0+1..c1 of the DP matrix of
 * (A, B) (0 <= r0 < r1 <= nA, 0 <= c0 < c1 <= nB) from its top row and left
 * column, exactly as twed_pair sweeps those cells: tiles swept in dependency
 * order give the twed_pair value bitwise.  A, TA, B, TB are the whole series
 * (device, as twed_pair); the block reads samples r0..r1 and c0..c1.
 * top: device, c1-c0+1 cells of row r0 (columns c0..c1); NULL is the pad row
 *   and is allowed only for r0 == 0.
 * left: device, r1-r0+1 cells of column c0 (rows r0..r1); NULL is the pad
 *   column, only for c0 == 0.  When both are given, top[0] is the corner.
 * bottom (c1-c0+1 cells of row r1), right (r1-r0+1 cells of column c1) and
 *   corner (one double, DP(r1, c1)): device outputs, each may be NULL.
 * The caller owns every buffer.  Precision TWED_F64 or TWED_F32_ACC64
 * (FP64 cells); strip_k as for twed_pair.
 * Errors: as twed_pair, plus TWED_ERR_INVALID for a block outside the matrix
 * or a missing top row / left column, TWED_ERR_UNSUPPORTED for another
 * precision, TWED_ERR_WORKSPACE if ws_bytes <
 * twed_pair_tile_workspace_size(r1 - r0, c1 - c0, prm). */
size_t twed_pair_tile_workspace_size(int64_t rows, int64_t cols, const twed_params *prm);

twed_status twed_pair_tile(const void *A, const void *TA, int64_t nA,
                           const void *B, const void *TB, int64_t nB,
                           const twed_params *prm, int64_t r0, int64_t r1, int64_t c0, int64_t c1,
                           const twed_cell *top, const twed_cell *left,
                           twed_cell *bottom, twed_cell *right, double *corner,
                           void *workspace, size_t ws_bytes, hipStream_t stream);

/* One optimal alignment path of (A, B) (section "Time Warp Edit Distance":
 * the path follows by backtracking over the choices of the forward problem).
 * The cells (i, j) from (0, 0) to (nA, nB) go to `path` (device, capacity
 * 2*(nA + nB + 1) int64, i and j interleaved) and their number to *path_len
 * (device int64); out (device double) receives the distance.  Read back from
 * (nA, nB), each cell is left by the move whose candidate is the minimum,
 * preferring the match, then the deletion in A (from the cell above), then
 * the deletion in B.  Memory: one forward sweep keeps every `block`-th row
 * and (rounded up to the strip width) column; each block the path crosses
 * is swept again recording one byte per cell; block == 0 means 4096.
 * Precision TWED_F64 or TWED_F32_ACC64.  The call reads the walk's position
 * between blocks, so it synchronises `stream` and returns when the path is
 * complete; the blocks next to the one being walked are swept meanwhile on
 * non-blocking streams the call creates, orders after `stream` and waits
 * for before it returns.  Errors as twed_pair_tile, plus TWED_ERR_INVALID for NULL
 * outputs or block < 0, and TWED_ERR_DEVICE when no finite path exists. */
size_t twed_pair_path_workspace_size(int64_t nA, int64_t nB, const twed_params *prm, int64_t block);

twed_status twed_pair_path(const void *A, const void *TA, int64_t nA,
                           const void *B, const void *TB, int64_t nB,
                           const twed_params *prm, int64_t block,
                           double *out, int64_t *path, int64_t *path_len,
                           void *workspace, size_t ws_bytes, hipStream_t stream);

/* ---- sibling dynamic programs (section "Generalized Dynamic Programming
 * Extensions", its "Direct Extension: LCS": programs whose cells need only
 * the cells above, to the left and up-left run on the same band sweep) ------
 * TWED_DP_DTW   dynamic time warping: D(i, j) = d(A_i, B_j) + min(D(i-1, j),
 *               D(i, j-1), D(i-1, j-1)), D(0, 0) = 0, +inf on the rest of row
 *               0 and column 0; d is the Lp distance of twed_params (dim, p).
 * TWED_DP_EDIT  edit (Levenshtein) distance of two 1-D token sequences
 *               (samples compared for equality; dim must be 1).
 * TWED_DP_LCS   length of a longest common subsequence of two 1-D token
 *               sequences (dim 1), from the indel distance nA + nB - 2*LCS.
 * Timestamps, nu and lambda are not used.  Samples are double for TWED_F64
 * and float for TWED_F32_ACC64 (the only precisions; tokens should be exact
 * integers in that type); results are one double on the device. */
typedef enum {
    TWED_DP_DTW = 1,
    TWED_DP_EDIT = 2,
    TWED_DP_LCS = 3
} twed_dp_kind;

/* One pair.  Errors: TWED_ERR_INVALID for an unknown kind, null pointers or
 * empty series; TWED_ERR_UNSUPPORTED for dim != 1 with EDIT / LCS, another
 * precision, strip_k other than 0, 1, 2 or 8, or series >= 2^31;
 * TWED_ERR_WORKSPACE if ws_bytes < twed_dp_workspace_size(...). */
size_t twed_dp_workspace_size(int32_t kind, int64_t nA, int64_t nB, const twed_params *prm);

twed_status twed_dp(int32_t kind, const void *A, int64_t nA, const void *B, int64_t nB,
                    const twed_params *prm, double *out,
                    void *workspace, size_t ws_bytes, hipStream_t stream);

/* One optimal alignment of the pair, as twed_pair_path (same path format,
 * tie order, block checkpoints and stream synchronisation).  For the edit and
 * LCS kinds the path may run along row 0 or column 0; for LCS the diagonal
 * steps into cells (i, j) with A_i == B_j give a longest common subsequence.
 * out receives the value as twed_dp. */
size_t twed_dp_path_workspace_size(int32_t kind, int64_t nA, int64_t nB, const twed_params *prm,
                                   int64_t block);

twed_status twed_dp_path(int32_t kind, const void *A, int64_t nA, const void *B, int64_t nB,
                         const twed_params *prm, int64_t block,
                         double *out, int64_t *path, int64_t *path_len,
                         void *workspace, size_t ws_bytes, hipStream_t stream);

/* ---- many pairs (the paper's batch mode, section "cuTWED Implementation
 * Remarks"; the symmetric case computes only the upper triangle, as the
 * section "Validation using Real Datasets" anticipates) ---------------------
 * X: device, packed samples of nX series (sum of lengths x dim); TX: device,
 * packed timestamps; offX: HOST, nX+1 non-decreasing int64 offsets (in
 * samples) with offX[0] = 0 and every length >= 1.  Same for Y / TY / offY.
 * Y == NULL means Y = X (then TY and offY must be NULL and nY == nX): the
 * symmetric all-pairs matrix, computed on the upper triangle, mirrored, with
 * a zero diagonal.
 * pairs == NULL: D is the nX x nY matrix, row-major, D[i*nY + j] =
 *   TWED(X_i, Y_j).
 * pairs != NULL: device array of nPairs (i, j) int64 pairs (0 <= i < nX,
 *   0 <= j < nY); D[k] = TWED(X_{pairs[2k]}, Y_{pairs[2k+1]}).  A pair
 *   outside those ranges cannot be checked on the host; its D[k] is NaN.
 * D: device, element type as `out` of twed_pair.  Every entry is
 * bitwise equal to what twed_pair returns for the same two series
 * and parameters, whichever operand is longer.
 * Pairs whose shorter series is longer than twed_batch_max_short_length(dim)
 * run the single-pair sweep one after another.  In pair-list mode, when both
 * collections hold such series, the call reads the pair list back to the
 * host to find them: it then synchronises `stream` before it returns.
 * Errors as for twed_pair, plus TWED_ERR_INVALID for bad offsets. */
size_t twed_batch_workspace_size(const int64_t *offX, int64_t nX,
                                 const int64_t *offY, int64_t nY,
                                 const twed_params *prm);

twed_status twed_batch(const void *X, const void *TX, const int64_t *offX, int64_t nX,
                       const void *Y, const void *TY, const int64_t *offY, int64_t nY,
                       const int64_t *pairs, int64_t nPairs,
                       const twed_params *prm, void *D,
                       void *workspace, size_t ws_bytes, hipStream_t stream);

/* A batch of fixed shape prepared once and run many times (the paper's batch
 * mode, as twed_batch).  twed_batch_plan_create checks the offsets and
 * parameters, lays out `workspace` (twed_batch_workspace_size bytes; the
 * caller keeps it allocated and untouched while the plan lives) and copies
 * the offsets and the longest-first order of the series into it with a
 * synchronous copy.  offY == NULL plans the symmetric matrix of X (nY is
 * then ignored); nPairs > 0 plans a pair list of that length (D then holds
 * nPairs results), nPairs == 0 the full matrix.
 * twed_batch_plan_run then enqueues kernels only on `stream` (staging, which
 * also clears the work ticket, the sweeps, the mirror and the widening), so
 * a caller can capture it in a HIP graph and replay it (except a pair-list
 * plan whose two collections both hold series longer than
 * twed_batch_max_short_length(dim): its runs read the list back, see
 * twed_batch); X, TX, Y, TY, pairs
 * and D as for twed_batch, with the planned shapes (Y, TY NULL exactly for a
 * symmetric plan, pairs given exactly for a pair-list plan; Y and TY may
 * also be NULL for a plan whose Y twed_batch_plan_stage_y staged).  Runs on one
 * plan must not overlap: they share the workspace.  The plan is a host
 * object; twed_batch_plan_destroy frees it (not the workspace).
 * Errors: as twed_batch at creation; at a run, TWED_ERR_INVALID (on the
 * host, before any launch) for a NULL plan or arguments that do not match
 * the plan. */
typedef struct twed_batch_plan twed_batch_plan;

twed_status twed_batch_plan_create(const int64_t *offX, int64_t nX, const int64_t *offY, int64_t nY,
                                   int64_t nPairs, const twed_params *prm,
                                   void *workspace, size_t ws_bytes, twed_batch_plan **plan);

/* Stages Y, TY (the planned second collection) into the plan's workspace on
 * `stream`.  After it, twed_batch_plan_run with Y == TY == NULL reuses those
 * rows instead of staging Y again: a fixed collection queried many times is
 * packed once.  The staged rows stay valid until the next stage call or a
 * run that passes Y.  Symmetric plans: TWED_ERR_INVALID. */
twed_status twed_batch_plan_stage_y(twed_batch_plan *plan, const void *Y, const void *TY, hipStream_t stream);

twed_status twed_batch_plan_run(const twed_batch_plan *plan, const void *X, const void *TX,
                                const void *Y, const void *TY, const int64_t *pairs, void *D,
                                hipStream_t stream);

void twed_batch_plan_destroy(twed_batch_plan *plan);

/* Batch autotuner (the paper plans light auto-tuning of its kernels, section
 * "cuTWED Implementation Remarks").  A batch run is configured by: the
 * consecutive items a wave takes per work ticket (chunk), the resident
 * waves per compute unit, and, for a single query of at most 32 samples,
 * whether each lane sweeps a whole pair (lane_mode 1) or each wave does
 * (0).  By default rules choose them.  twed_batch_plan_tune runs the plan on
 * the given inputs (as twed_batch_plan_run, several times: D is
 * overwritten) under the rules' choice and then, one knob at a time, under
 * each candidate (lane mode; chunk 1..64; a quarter, half or three quarters
 * of the waves that fit), keeps the fastest (median of three runs) in the
 * plan, and caches it under the plan's size class: device (architecture and
 * compute units), precision, dimension, distance, mode (symmetric,
 * rectangular, pair list), and the mean series lengths of X and Y and the
 * number of pairs, each rounded down to a power of two.  Plans created
 * afterwards, and twed_batch calls, of the same class use the cached choice.
 * Synchronises `stream`.  Results never depend on the configuration: every
 * entry is the same bits.  The chosen values go to *chunk, *waves_per_cu
 * and *lane_mode when those are not NULL (0 / 0 / -1 mean the rule).
 * Errors as twed_batch_plan_run. */
twed_status twed_batch_plan_tune(twed_batch_plan *plan, const void *X, const void *TX,
                                 const void *Y, const void *TY, const int64_t *pairs, void *D,
                                 hipStream_t stream, int32_t *chunk, int32_t *waves_per_cu,
                                 int32_t *lane_mode);

/* The configuration a plan runs with (values as twed_batch_plan_tune's). */
twed_status twed_batch_plan_config(const twed_batch_plan *plan, int32_t *chunk, int32_t *waves_per_cu,
                                   int32_t *lane_mode);

/* Writes the tuning cache (single-pair choices of twed_pair_tune and batch
 * choices of twed_batch_plan_tune) to a text file, or merges such a file
 * into it, so that measurements survive the process.  Entries carry the
 * device they were measured on and apply only to that kind of device.
 * Errors: TWED_ERR_INVALID for a NULL path, a file that cannot be opened or
 * written, or (load) a malformed file, in which case nothing is merged. */
twed_status twed_tune_save(const char *path);
twed_status twed_tune_load(const char *path);

/* Longest shorter-operand length a pair may have to be swept by a single
 * wave inside the batched kernel (longer pairs use the single-pair sweep). */
int64_t twed_batch_max_short_length(int32_t dim);

/* ---- measurement helper (not part of the distance computation) -------------
 * Enqueues a loop of independent vector operations on `stream` so that the
 * caller, timing it, measures the chip's vector lane-operation rate: the
 * ceiling the sweeps' roofline fractions are taken against.  `waves` waves
 * of 64 lanes (a multiple of 4, at most 2^24) each run `iters` iterations
 * of eight independent chains of: kind 0 an FP32 fused multiply-add; 1 an
 * FP32 add then minimum; 2 an FP64 fused multiply-add; 3 an FP64 add then
 * minimum; 4 an FP32 square root; 5 an FP32 add; 6 an FP64 add; 7 an FP32
 * three-way minimum.  sink: device, waves*64 doubles (kinds 2, 3, 6) or
 * floats (the others), overwritten.  *lane_ops (host, may be NULL) receives
 * the lane operations issued (an add and a minimum count as two, a
 * three-way minimum as one).  Errors: TWED_ERR_INVALID for an unknown kind,
 * iters < 1, a bad wave count or a NULL sink. */
twed_status twed_probe_valu(int32_t kind, int64_t waves, int64_t iters, void *sink, double *lane_ops,
                            hipStream_t stream);

/* ---- status ---------------------------------------------------------------- */
const char *twed_status_string(twed_status s);
/* Message of the last error returned on the calling thread ("" if none). */
const char *twed_last_error(void);
/* Synchronises `stream` and reports TWED_ERR_DEVICE if it has failed. */
twed_status twed_stream_check(hipStream_t stream);
/* Library version string. */
const char *twed_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TWED_H_ */

// tile_capi.hip -- extern "C" entry points of the tile sweep and of the
// alignment path (host code: argument checks, workspace layout, dispatch).
//
// A block of the DP matrix is swept from its top row and left column of
// (DP, X = DP + e) cells (section "Improved Time Warp Edit Distance": the
// band is the whole state), which gives resumable sweeps of long pairs and
// the column shards a multi-GPU sweep would hand from GPU to GPU.  The path
// is read back block by block from moves recorded during a second sweep of
// each block the path crosses (section "Time Warp Edit Distance" names
// backtracking over the forward problem's choices).
#include "../../include/twed.h"
#include "capi_util.h"
#include "twed_kernels.h"

#include <algorithm>
#include <cstdint>
#include <cstdlib>

using namespace twed;
using namespace twed::capi;

namespace {

constexpr int64_t kTailWords = 4;      // work ticket, wait error word, two spare words
constexpr size_t kDummyCells = 512;    // 64 lanes x up to 8 columns
constexpr int64_t kDefaultBlock = 4096;
constexpr size_t kCell = 16;           // one (DP, X) pair of FP64

int simds()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1024;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 1024;
    return cus * 4;
}

bool tile_prec(const twed_params *prm, Prec *out)
{
    if (prm->precision == TWED_F64) *out = kF64;
    else if (prm->precision == TWED_F32_ACC64) *out = kF32Acc64;
    else return false;
    return true;
}

struct Sweep {
    int K, G;
};

// The widest strip whose kernel keeps to registers and still leaves about
// three strips for every four SIMDs (the rule of the pair sweep), in the
// widest non-spilling group that leaves work for half the CUs.
// The recurrence a sweep runs: kRecTwed, or a sibling (kRecDtw, kRecEdit,
// kRecIndel; see twed_device.h), whose kernels exist for K in {1, 8} and G
// in {1, 8} only.
size_t sweep_scratch(int rec, bool dirs, Prec prec, const CostParams &cp, int K, int G)
{
    if (dirs) return rec_dirs_scratch_bytes(rec, prec, cp, K, G);
    return rec == kRecTwed ? tile_scratch_bytes(prec, cp, K, G) : dp_scratch_bytes(rec, prec, cp, K, G);
}

int sweep_workers(int rec, bool dirs, Prec prec, const CostParams &cp, int K, int G)
{
    if (dirs) return rec_dirs_max_workers(rec, prec, cp, K, G);
    return rec == kRecTwed ? tile_max_workers(prec, cp, K, G) : dp_max_workers(rec, prec, cp, K, G);
}

// Move-recording sweeps (dirs) run strips of one column per lane.
Sweep tile_sweep(int rec, int strip_k, int64_t nB, Prec prec, const CostParams &cp, bool dirs = false)
{
    const bool sib = rec != kRecTwed && !dirs;
    int K = 1;
    if (dirs) {
        K = 1;
    } else if (strip_k > 0) {
        K = strip_k;
    } else {
        const int64_t want = (int64_t)simds() * 3 / 4;
        for (int k : {8, 4, 2}) {
            if (sib && k == 4) continue;
            const int64_t strips = (nB + 64 * k - 1) / (64 * k);
            if (strips >= want && sweep_scratch(rec, dirs, prec, cp, k, 1) == 0) {
                K = k;
                break;
            }
        }
    }
    // Groups: in-group handoffs go through LDS, which shortens the pipeline,
    // so the widest group that still leaves work for half the CUs; a
    // move-recording sweep of one block is latency-bound, not width-bound,
    // and takes the widest group that has a few groups to pipeline.
    const int64_t nStrips = (nB + 64 * K - 1) / (64 * K);
    const int64_t cus = std::max(1, simds() / 4);
    const int64_t want_groups = dirs ? 2 : std::max<int64_t>(1, cus / 2);
    int G = 1;
    for (int g : {8, 4}) {
        if (sib && g != 8) continue;
        if ((nStrips + g - 1) / g >= want_groups && nStrips >= g && sweep_scratch(rec, dirs, prec, cp, K, g) == 0) {
            G = g;
            break;
        }
    }
    // TWED_WAVEFRONT_GROUP (1, 4 or 8) overrides the group of plain TWED
    // tile sweeps for tuning runs
    if (const char *env = std::getenv("TWED_WAVEFRONT_GROUP")) {
        const int g = std::atoi(env);
        if (!sib && !dirs && (g == 1 || g == 4 || g == 8) && sweep_scratch(rec, dirs, prec, cp, K, g) == 0) G = g;
    }
    return Sweep{K, G};
}

// Staged rows, handoff slots, flags and scratch of one sweep of nA x nB.
struct SweepBuffers {
    void *rowsA, *rowsB, *bnd, *dummy, *tmp;
    uint32_t *flags;
    int64_t zero_words;
};

void take_sweep(Carver &c, SweepBuffers &b, Prec prec, int dimt, int64_t nA, int64_t nB)
{
    b.rowsA = take_rows(c, prec, dimt, nA + 1);
    b.rowsB = take_rows(c, prec, dimt, nB + 1);
    b.bnd = c.take((size_t)2 * (size_t)(nA + 1) * kCell);
    b.zero_words = (nB + 63) / 64 + kTailWords;
    b.flags = (uint32_t *)c.take((size_t)b.zero_words * 4);
    b.dummy = c.take(kDummyCells * kCell);
    b.tmp = c.take(8);
}

twed_status run_tile(int rec, Prec prec, const CostParams &cp, Sweep sw, const void *rowsA, const void *rowsB,
                     int64_t nA, int64_t nB, const SweepBuffers &b, const TileArgs &t, void *out, hipStream_t st)
{
    WavefrontArgs w{};
    w.rowsA = rowsA;
    w.rowsB = rowsB;
    w.nA = nA;
    w.nB = nB;
    w.bnd = b.bnd;
    w.flags = b.flags;
    w.ticket = b.flags + (b.zero_words - kTailWords);
    w.beta = w.ticket + 2;
    w.nStrips = (nB + 64 * sw.K - 1) / (64 * sw.K);
    w.out = out;
    w.dump = nullptr;
    w.group = sw.G;
    w.sub_shift = 4;
    const int workers = sweep_workers(rec, t.dirs != nullptr, prec, cp, sw.K, sw.G);
    if (workers <= 0) return fail(TWED_ERR_DEVICE, "occupancy query failed");
    w.grid = (int)std::min<int64_t>((w.nStrips + sw.G - 1) / sw.G, workers);
    const hipError_t e = rec == kRecTwed ? launch_tile(prec, cp, sw.K, w, t, st)
                                         : launch_dp(rec, prec, cp, sw.K, w, t, st);
    if (e != hipSuccess) return fail_hip(e, "tile sweep launch");
    return TWED_OK;
}

twed_status check_series(const void *A, const void *TA, int64_t nA, const void *B, const void *TB, int64_t nB)
{
    if (!A || !TA || !B || !TB) return fail(TWED_ERR_INVALID, "NULL array argument");
    if (nA < 1 || nB < 1) return fail(TWED_ERR_INVALID, "series lengths must be >= 1");
    if (nA > kMaxLen || nB > kMaxLen) return fail(TWED_ERR_UNSUPPORTED, "series longer than 2^31 - 130");
    return TWED_OK;
}

size_t row_bytes(Prec prec, int dimt) { return (size_t)row_stride(prec, dimt) * cost_size(prec); }

// ---- path layout ---------------------------------------------------------------

struct PathGeometry {
    Sweep fwd, blk;
    int64_t H, Wc, nr, nc;
};

PathGeometry path_geometry(int rec, const twed_params *prm, int64_t nA, int64_t nB, int64_t block, Prec prec,
                           const CostParams &cp)
{
    PathGeometry g{};
    const int64_t want = block > 0 ? block : kDefaultBlock;
    g.fwd = tile_sweep(rec, prm->strip_k, nB, prec, cp);
    const int64_t W = 64 * (int64_t)g.fwd.K;
    g.H = std::max<int64_t>(64, want);
    g.Wc = (std::max(want, W) + W - 1) / W * W;
    g.nr = (nA - 1) / g.H;
    g.nc = (nB - 1) / g.Wc;
    g.blk = tile_sweep(rec, 0, std::min(g.Wc, nB), prec, cp, true);
    return g;
}

// Edit and indel distances start from finite row 0 / column 0 (i, i).
bool finite_edges(int rec) { return rec == kRecEdit || rec == kRecIndel; }

// Blocks recomputed with moves at once: the block the walk is in and the
// three it can leave into (up, left, up-left), each in its own slot.
constexpr int kPathSlots = 4;

struct PathLayout {
    SweepBuffers b;
    SweepBuffers slot[kPathSlots];  // boundary, flags, dummy and result of one block sweep
    void *dirs[kPathSlots];
    void *ckrow, *ckcol, *row0, *col0;
    int64_t *st;
    size_t total;
};

PathLayout path_layout(char *base, int rec, const twed_params *prm, int64_t nA, int64_t nB, const PathGeometry &g,
                       Prec prec)
{
    Carver c{base};
    PathLayout L{};
    take_sweep(c, L.b, prec, dimt_for(prm->dim), nA, nB);
    L.st = (int64_t *)c.take(4 * sizeof(int64_t));
    if (finite_edges(rec)) {
        L.row0 = c.take((size_t)(nB + 1) * kCell);
        L.col0 = c.take((size_t)(nA + 1) * kCell);
    }
    L.ckrow = c.take((size_t)g.nr * (size_t)(nB + 1) * kCell);
    L.ckcol = c.take((size_t)g.nc * (size_t)(nA + 1) * kCell);
    const int64_t Wb = 64 * (int64_t)g.blk.K;
    const int64_t bh = std::min(g.H, nA), bw = std::min(g.Wc, nB);
    const int64_t strips = (bw + Wb - 1) / Wb;
    for (int k = 0; k < kPathSlots; ++k) {
        SweepBuffers &u = L.slot[k];
        u.rowsA = L.b.rowsA;
        u.rowsB = L.b.rowsB;
        u.bnd = c.take((size_t)2 * (size_t)(bh + 1) * kCell);
        u.zero_words = (bw + 63) / 64 + kTailWords;
        u.flags = (uint32_t *)c.take((size_t)u.zero_words * 4);
        u.dummy = c.take(kDummyCells * kCell);
        u.tmp = c.take(8);
        L.dirs[k] = c.take((size_t)strips * (size_t)(bh + 64) * (size_t)Wb);
    }
    L.total = c.used;
    return L;
}

// Side streams and events of the backward pass; the destructor waits for
// their work (speculative block sweeps may still run) before releasing them.
struct PathStreams {
    hipStream_t s[kPathSlots] = {};
    hipEvent_t done[kPathSlots] = {};
    hipEvent_t fwd = nullptr;
    hipError_t create()
    {
        hipError_t e = hipEventCreateWithFlags(&fwd, hipEventDisableTiming);
        for (int k = 0; k < kPathSlots && e == hipSuccess; ++k) {
            e = hipStreamCreateWithFlags(&s[k], hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&done[k], hipEventDisableTiming);
        }
        return e;
    }
    ~PathStreams()
    {
        for (int k = 0; k < kPathSlots; ++k) {
            if (s[k]) {
                (void)hipStreamSynchronize(s[k]);
                (void)hipStreamDestroy(s[k]);
            }
            if (done[k]) (void)hipEventDestroy(done[k]);
        }
        if (fwd) (void)hipEventDestroy(fwd);
    }
};

// The path of one pair under recurrence `rec` (A/TA/B/TB as staged by
// twed_pair; TA, TB null for the siblings).  Runs after argument checks.
twed_status path_impl(int rec, const void *A, const void *TA, int64_t nA, const void *B, const void *TB, int64_t nB,
                      const twed_params *prm, int64_t block, double *out, int64_t *path, int64_t *path_len,
                      void *workspace, size_t ws_bytes, Prec prec, hipStream_t st)
{
    twed_status s;
    const CostParams cp = cost_params(prm);
    const PathGeometry g = path_geometry(rec, prm, nA, nB, block, prec, cp);
    if (g.H > 0x40000000LL || g.Wc > 0x40000000LL) return fail(TWED_ERR_UNSUPPORTED, "block too large");
    if ((s = check_workspace(workspace, ws_bytes, path_layout(nullptr, rec, prm, nA, nB, g, prec).total)) != TWED_OK)
        return s;
    const PathLayout L = path_layout((char *)workspace, rec, prm, nA, nB, g, prec);
    const SweepBuffers &b = L.b;
    hipError_t e;
#define TRY(call, what)                                \
    do {                                               \
        e = (call);                                    \
        if (e != hipSuccess) return fail_hip(e, what); \
    } while (0)
    // forward sweep of the whole pair, keeping checkpoint rows and columns
    TRY(launch_stage(prec, cp, A, TA, nullptr, 1, nA, nA, nA + 1, b.rowsA, b.flags, b.zero_words, st), "staging");
    TRY(launch_stage(prec, cp, B, TB, nullptr, 1, nB, nB, nB + 1, b.rowsB, nullptr, 0, st), "staging");
    if (finite_edges(rec)) {
        TRY(launch_index_cells(L.row0, nB, st), "boundary");
        TRY(launch_index_cells(L.col0, nA, st), "boundary");
    }
    TileArgs t{};
    t.top = L.row0;
    t.left = L.col0;
    t.dummy = b.dummy;
    t.ckrow = g.nr > 0 ? L.ckrow : nullptr;
    t.ckcol = g.nc > 0 ? L.ckcol : nullptr;
    t.ck_rows = (int)g.H;
    t.ck_cols = (int)g.Wc;
    s = run_tile(rec, prec, cp, g.fwd, b.rowsA, b.rowsB, nA, nB, b, t, out, st);
    if (s != TWED_OK) return s;
    // Backwards, block by block: sweep the block again recording moves, walk
    // it.  While the walk runs on the caller's stream, the blocks it can
    // leave into are swept on side streams, so that the next walk finds its
    // moves ready: the sweep of a block (latency-bound one-column strips on
    // a few CUs) then overlaps the walk of the one before.
    const int64_t cap = nA + nB + 1;
    TRY(launch_walk_init(L.st, nA, nB, st), "walk set-up");
    const size_t rb = row_bytes(prec, dimt_for(prm->dim));
    PathStreams ps;
    TRY(ps.create(), "stream set-up");
    TRY(hipEventRecord(ps.fwd, st), "event record");
    for (int k = 0; k < kPathSlots; ++k) TRY(hipStreamWaitEvent(ps.s[k], ps.fwd, 0), "stream wait");
    int64_t held[kPathSlots][2];
    for (int k = 0; k < kPathSlots; ++k) held[k][0] = held[k][1] = -1;
    // sweeps block (br, bc) with moves into slot k on side stream k
    auto sweep_block = [&](int k, int64_t br, int64_t bc) -> twed_status {
        const int64_t r0 = br * g.H, r1 = std::min(r0 + g.H, nA);
        const int64_t c0 = bc * g.Wc, c1 = std::min(c0 + g.Wc, nB);
        const SweepBuffers &sb = L.slot[k];
        hipError_t e2 = launch_zero32(sb.flags, sb.zero_words, ps.s[k]);
        if (e2 != hipSuccess) return fail_hip(e2, "flag reset");
        TileArgs u{};
        u.dummy = sb.dummy;
        if (br > 0)
            u.top = (const char *)L.ckrow + ((size_t)(br - 1) * (size_t)(nB + 1) + (size_t)c0) * kCell;
        else if (L.row0)
            u.top = (const char *)L.row0 + (size_t)c0 * kCell;
        if (bc > 0)
            u.left = (const char *)L.ckcol + ((size_t)(bc - 1) * (size_t)(nA + 1) + (size_t)r0) * kCell;
        else if (L.col0)
            u.left = (const char *)L.col0 + (size_t)r0 * kCell;
        u.dirs = (uint8_t *)L.dirs[k];
        const twed_status s2 = run_tile(rec, prec, cp, g.blk, (const char *)b.rowsA + r0 * rb,
                                        (const char *)b.rowsB + c0 * rb, r1 - r0, c1 - c0, sb, u, sb.tmp, ps.s[k]);
        if (s2 != TWED_OK) return s2;
        e2 = hipEventRecord(ps.done[k], ps.s[k]);
        if (e2 != hipSuccess) return fail_hip(e2, "event record");
        held[k][0] = br;
        held[k][1] = bc;
        return TWED_OK;
    };
    int64_t hst[4] = {0, 0, 0, 0};
    const int64_t max_blocks = g.nr + g.nc + 3;
    for (int64_t it = 0;; ++it) {
        TRY(hipMemcpyAsync(hst, L.st, sizeof(hst), hipMemcpyDeviceToHost, st), "walk state read");
        TRY(hipStreamSynchronize(st), "walk state read");
        if (hst[3] == 1) break;
        if (hst[3] != 0 || it > max_blocks || hst[0] < 1 || hst[1] < 1)
            return fail(TWED_ERR_DEVICE, "the path could not be followed (non-finite distance or a timed-out sweep)");
        const int64_t br = (hst[0] - 1) / g.H, bc = (hst[1] - 1) / g.Wc;
        // this block first, then the up, left and up-left neighbours
        int64_t want[kPathSlots][2];
        int nw = 0;
        want[nw][0] = br, want[nw][1] = bc, ++nw;
        if (br > 0) want[nw][0] = br - 1, want[nw][1] = bc, ++nw;
        if (bc > 0) want[nw][0] = br, want[nw][1] = bc - 1, ++nw;
        if (br > 0 && bc > 0) want[nw][0] = br - 1, want[nw][1] = bc - 1, ++nw;
        auto slot_of = [&](int64_t qr, int64_t qc) {
            for (int k = 0; k < kPathSlots; ++k)
                if (held[k][0] == qr && held[k][1] == qc) return k;
            return -1;
        };
        // slots whose block is not wanted may be overwritten (slot k's
        // earlier sweep is ordered before the new one on stream k, and every
        // walk that read it has finished: the caller's stream was synchronised)
        bool keep[kPathSlots] = {};
        for (int w = 0; w < nw; ++w) {
            const int k = slot_of(want[w][0], want[w][1]);
            if (k >= 0) keep[k] = true;
        }
        for (int w = 0; w < nw; ++w) {
            if (slot_of(want[w][0], want[w][1]) >= 0) continue;
            int k = 0;
            while (keep[k]) ++k;  // nw <= kPathSlots, so a free slot exists
            keep[k] = true;
            if ((s = sweep_block(k, want[w][0], want[w][1])) != TWED_OK) return s;
        }
        const int kc = slot_of(br, bc);
        const int64_t r0 = br * g.H, r1 = std::min(r0 + g.H, nA);
        const int64_t c0 = bc * g.Wc, c1 = std::min(c0 + g.Wc, nB);
        TRY(hipStreamWaitEvent(st, ps.done[kc], 0), "stream wait");
        TRY(launch_walk((const uint8_t *)L.dirs[kc], r0, c0, r1 - r0, c1 - c0, g.blk.K, (r1 - r0) + 64, L.st, path,
                        cap, finite_edges(rec), st),
            "walk");
    }
    // later work on the caller's stream (and its reuse of the workspace)
    // stays behind speculative sweeps still running
    for (int k = 0; k < kPathSlots; ++k)
        if (held[k][0] >= 0) TRY(hipStreamWaitEvent(st, ps.done[k], 0), "stream wait");
    TRY(launch_order(L.st, path, path_len, cap, st), "path order");
    // the path and its length are complete when the call returns
    TRY(hipStreamSynchronize(st), "path order");
#undef TRY
    return TWED_OK;
}

// The recurrence of a twed_dp kind, or -1.
int rec_of(int32_t kind)
{
    switch (kind) {
    case TWED_DP_DTW: return kRecDtw;
    case TWED_DP_EDIT: return kRecEdit;
    case TWED_DP_LCS: return kRecIndel;
    default: return -1;
    }
}

twed_status check_dp(int32_t kind, const twed_params *prm, Prec *prec)
{
    twed_status s = check_params(prm);
    if (s != TWED_OK) return s;
    if (rec_of(kind) < 0) return fail(TWED_ERR_INVALID, "unknown twed_dp_kind");
    if (kind != TWED_DP_DTW && prm->dim != 1)
        return fail(TWED_ERR_UNSUPPORTED, "edit distance and LCS compare 1-D samples (dim = 1)");
    if (!(prm->strip_k == 0 || prm->strip_k == 1 || prm->strip_k == 2 || prm->strip_k == 8))
        return fail(TWED_ERR_UNSUPPORTED, "twed_dp takes strip_k 0, 1, 2 or 8");
    if (!tile_prec(prm, prec)) return fail(TWED_ERR_UNSUPPORTED, "twed_dp takes TWED_F64 or TWED_F32_ACC64");
    return TWED_OK;
}

}  // namespace

extern "C" {

size_t twed_pair_tile_workspace_size(int64_t rows, int64_t cols, const twed_params *prm)
{
    Prec prec;
    if (rows < 1 || cols < 1 || rows > kMaxLen || cols > kMaxLen) return 0;
    if (check_params(prm) != TWED_OK || !tile_prec(prm, &prec)) return 0;
    Carver c{nullptr};
    SweepBuffers b{};
    take_sweep(c, b, prec, dimt_for(prm->dim), rows, cols);
    return c.used;
}

twed_status twed_pair_tile(const void *A, const void *TA, int64_t nA, const void *B, const void *TB, int64_t nB,
                           const twed_params *prm, int64_t r0, int64_t r1, int64_t c0, int64_t c1,
                           const twed_cell *top, const twed_cell *left, twed_cell *bottom, twed_cell *right,
                           double *corner, void *workspace, size_t ws_bytes, hipStream_t st)
{
    last_error().clear();
    twed_status s = check_params(prm);
    if (s != TWED_OK) return s;
    if ((s = check_series(A, TA, nA, B, TB, nB)) != TWED_OK) return s;
    if (!(0 <= r0 && r0 < r1 && r1 <= nA && 0 <= c0 && c0 < c1 && c1 <= nB))
        return fail(TWED_ERR_INVALID, "the block must satisfy 0 <= r0 < r1 <= nA and 0 <= c0 < c1 <= nB");
    if (r0 > 0 && !top) return fail(TWED_ERR_INVALID, "a block below row 0 needs its top row");
    if (c0 > 0 && !left) return fail(TWED_ERR_INVALID, "a block right of column 0 needs its left column");
    Prec prec;
    if (!tile_prec(prm, &prec)) return fail(TWED_ERR_UNSUPPORTED, "tiles take TWED_F64 or TWED_F32_ACC64");
    const int64_t nAt = r1 - r0, nBt = c1 - c0;
    const size_t need = twed_pair_tile_workspace_size(nAt, nBt, prm);
    if ((s = check_workspace(workspace, ws_bytes, need)) != TWED_OK) return s;
    Carver c{(char *)workspace};
    SweepBuffers b{};
    const int dimt = dimt_for(prm->dim);
    take_sweep(c, b, prec, dimt, nAt, nBt);
    const CostParams cp = cost_params(prm);
    const size_t es = cost_size(prec) * (size_t)prm->dim, ts = cost_size(prec);
    hipError_t e = launch_stage(prec, cp, (const char *)A + r0 * es, (const char *)TA + r0 * ts, nullptr, 1, nAt,
                                nAt, nAt + 1, b.rowsA, b.flags, b.zero_words, st, r0 > 0);
    if (e != hipSuccess) return fail_hip(e, "staging launch");
    e = launch_stage(prec, cp, (const char *)B + c0 * es, (const char *)TB + c0 * ts, nullptr, 1, nBt, nBt, nBt + 1,
                     b.rowsB, nullptr, 0, st, c0 > 0);
    if (e != hipSuccess) return fail_hip(e, "staging launch");
    TileArgs t{};
    t.top = top;
    t.left = left;
    t.bottom = bottom;
    t.right = right;
    t.dummy = b.dummy;
    return run_tile(kRecTwed, prec, cp, tile_sweep(kRecTwed, prm->strip_k, nBt, prec, cp), b.rowsA, b.rowsB, nAt,
                    nBt, b, t, corner ? (void *)corner : b.tmp, st);
}

size_t twed_pair_path_workspace_size(int64_t nA, int64_t nB, const twed_params *prm, int64_t block)
{
    Prec prec;
    if (nA < 1 || nB < 1 || nA > kMaxLen || nB > kMaxLen || block < 0) return 0;
    if (check_params(prm) != TWED_OK || !tile_prec(prm, &prec)) return 0;
    const CostParams cp = cost_params(prm);
    const PathGeometry g = path_geometry(kRecTwed, prm, nA, nB, block, prec, cp);
    return path_layout(nullptr, kRecTwed, prm, nA, nB, g, prec).total;
}

twed_status twed_pair_path(const void *A, const void *TA, int64_t nA, const void *B, const void *TB, int64_t nB,
                           const twed_params *prm, int64_t block, double *out, int64_t *path, int64_t *path_len,
                           void *workspace, size_t ws_bytes, hipStream_t st)
{
    last_error().clear();
    twed_status s = check_params(prm);
    if (s != TWED_OK) return s;
    if ((s = check_series(A, TA, nA, B, TB, nB)) != TWED_OK) return s;
    if (!out || !path || !path_len) return fail(TWED_ERR_INVALID, "NULL output argument");
    if (block < 0) return fail(TWED_ERR_INVALID, "block must be >= 0");
    Prec prec;
    if (!tile_prec(prm, &prec)) return fail(TWED_ERR_UNSUPPORTED, "the path takes TWED_F64 or TWED_F32_ACC64");
    return path_impl(kRecTwed, A, TA, nA, B, TB, nB, prm, block, out, path, path_len, workspace, ws_bytes, prec, st);
}

size_t twed_dp_workspace_size(int32_t kind, int64_t nA, int64_t nB, const twed_params *prm)
{
    Prec prec;
    if (nA < 1 || nB < 1 || nA > kMaxLen || nB > kMaxLen) return 0;
    if (check_dp(kind, prm, &prec) != TWED_OK) return 0;
    Carver c{nullptr};
    SweepBuffers b{};
    take_sweep(c, b, prec, dimt_for(prm->dim), nA, nB);
    c.take((size_t)(nA + nB + 2) * kCell);
    return c.used;
}

twed_status twed_dp(int32_t kind, const void *A, int64_t nA, const void *B, int64_t nB, const twed_params *prm,
                    double *out, void *workspace, size_t ws_bytes, hipStream_t st)
{
    last_error().clear();
    Prec prec;
    twed_status s = check_dp(kind, prm, &prec);
    if (s != TWED_OK) return s;
    if (!A || !B || !out) return fail(TWED_ERR_INVALID, "NULL array argument");
    if (nA < 1 || nB < 1) return fail(TWED_ERR_INVALID, "series lengths must be >= 1");
    if (nA > kMaxLen || nB > kMaxLen) return fail(TWED_ERR_UNSUPPORTED, "series longer than 2^31 - 130");
    if ((s = check_workspace(workspace, ws_bytes, twed_dp_workspace_size(kind, nA, nB, prm))) != TWED_OK) return s;
    const int rec = rec_of(kind);
    Carver c{(char *)workspace};
    SweepBuffers b{};
    take_sweep(c, b, prec, dimt_for(prm->dim), nA, nB);
    void *row0 = c.take((size_t)(nB + 1) * kCell);
    void *col0 = c.take((size_t)(nA + 1) * kCell);
    const CostParams cp = cost_params(prm);
    hipError_t e = launch_stage(prec, cp, A, nullptr, nullptr, 1, nA, nA, nA + 1, b.rowsA, b.flags, b.zero_words, st);
    if (e != hipSuccess) return fail_hip(e, "staging launch");
    e = launch_stage(prec, cp, B, nullptr, nullptr, 1, nB, nB, nB + 1, b.rowsB, nullptr, 0, st);
    if (e != hipSuccess) return fail_hip(e, "staging launch");
    TileArgs t{};
    t.dummy = b.dummy;
    if (finite_edges(rec)) {
        if ((e = launch_index_cells(row0, nB, st)) != hipSuccess) return fail_hip(e, "boundary");
        if ((e = launch_index_cells(col0, nA, st)) != hipSuccess) return fail_hip(e, "boundary");
        t.top = row0;
        t.left = col0;
    }
    s = run_tile(rec, prec, cp, tile_sweep(rec, prm->strip_k, nB, prec, cp), b.rowsA, b.rowsB, nA, nB, b, t, out, st);
    if (s != TWED_OK) return s;
    if (kind == TWED_DP_LCS && (e = launch_lcs_finish(out, nA, nB, st)) != hipSuccess) return fail_hip(e, "LCS");
    return TWED_OK;
}

size_t twed_dp_path_workspace_size(int32_t kind, int64_t nA, int64_t nB, const twed_params *prm, int64_t block)
{
    Prec prec;
    if (nA < 1 || nB < 1 || nA > kMaxLen || nB > kMaxLen || block < 0) return 0;
    if (check_dp(kind, prm, &prec) != TWED_OK) return 0;
    const int rec = rec_of(kind);
    const CostParams cp = cost_params(prm);
    const PathGeometry g = path_geometry(rec, prm, nA, nB, block, prec, cp);
    return path_layout(nullptr, rec, prm, nA, nB, g, prec).total;
}

twed_status twed_dp_path(int32_t kind, const void *A, int64_t nA, const void *B, int64_t nB, const twed_params *prm,
                         int64_t block, double *out, int64_t *path, int64_t *path_len, void *workspace,
                         size_t ws_bytes, hipStream_t st)
{
    last_error().clear();
    Prec prec;
    twed_status s = check_dp(kind, prm, &prec);
    if (s != TWED_OK) return s;
    if (!A || !B) return fail(TWED_ERR_INVALID, "NULL array argument");
    if (nA < 1 || nB < 1) return fail(TWED_ERR_INVALID, "series lengths must be >= 1");
    if (nA > kMaxLen || nB > kMaxLen) return fail(TWED_ERR_UNSUPPORTED, "series longer than 2^31 - 130");
    if (!out || !path || !path_len) return fail(TWED_ERR_INVALID, "NULL output argument");
    if (block < 0) return fail(TWED_ERR_INVALID, "block must be >= 0");
    s = path_impl(rec_of(kind), A, nullptr, nA, B, nullptr, nB, prm, block, out, path, path_len, workspace, ws_bytes,
                  prec, st);
    if (s != TWED_OK) return s;
    if (kind == TWED_DP_LCS) {
        const hipError_t e = launch_lcs_finish(out, nA, nB, st);
        if (e != hipSuccess) return fail_hip(e, "LCS");
    }
    return TWED_OK;
}

}  // extern "C"

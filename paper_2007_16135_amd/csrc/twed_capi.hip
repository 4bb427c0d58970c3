// twed_capi.hip -- the extern "C" boundary of libtwed: argument validation,
// workspace layout, precision policy, strip-width choice and dispatch.
//
// Host code only.  Every argument error is detected here before the first
// HIP call (section "Time Warp Edit Distance" fixes what a valid problem is:
// two non-empty series with timestamps, nu >= 0, lambda >= 0, an Lp degree).
#include "../../include/twed.h"
#include "capi_util.h"
#include "twed_kernels.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <mutex>
#include <tuple>
#include <cstdlib>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

using namespace twed;
using namespace twed::capi;

namespace twed {
namespace capi {
std::string &last_error()
{
    thread_local std::string msg;
    return msg;
}
}  // namespace capi
}  // namespace twed

namespace {

constexpr int64_t kDefaultAcc64Threshold = 100000;

// Resolved arithmetic of a call whose longest series has `maxlen` samples.
Prec resolve(const twed_params *prm, int64_t maxlen)
{
    switch (prm->precision) {
    case TWED_F64: return kF64;
    case TWED_F32: return kF32;
    case TWED_F32_ACC64: return kF32Acc64;
    default: {
        const int64_t thr = prm->acc64_threshold > 0 ? prm->acc64_threshold : kDefaultAcc64Threshold;
        return maxlen > thr ? kF32Acc64 : kF32;
    }
    }
}

// AUTO always returns f64; when it resolves to F32 the kernels write f32 into
// the workspace and a widening pass copies them out.
bool needs_widen(const twed_params *prm, Prec p) { return prm->precision == TWED_AUTO && p == kF32; }

int device_simds()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1024;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 1024;
    return cus * 4;
}

// Columns per lane of the wavefront sweep: the widest strip that still
// leaves about three strips for every four SIMDs, and whose kernel keeps
// everything in registers (wide strips of high-dimensional or general-Lp
// sweeps would spill).  Narrow strips fill more SIMDs but lengthen the
// pipeline (each strip starts 64 + 16 steps after the one before it) and
// pay the per-step work for fewer cells: on the 3-D n = 1e5 pair, strips of
// two columns (782 strips) sweep 1.36x faster in FP64 than strips of one
// (1,563 strips, two waves on some SIMDs).
int choose_k(const twed_params *prm, int64_t nB, Prec prec, const CostParams &cp)
{
    if (prm->strip_k > 0) return prm->strip_k;
    const int64_t want = (int64_t)device_simds() * 3 / 4;
    for (int k : {8, 4, 2}) {
        const int64_t strips = (nB + 64 * k - 1) / (64 * k);
        if (strips >= want && wavefront_scratch_bytes(prec, cp, k, 1) == 0) return k;
    }
    return 1;
}

// Words after the per-strip flags in the zeroed region: work ticket, wait
// timeout flag, and two words holding the FP32 cost offset.
constexpr int64_t kTailWords = 4;

struct PairLayout {
    void *rowsA, *rowsB, *bnd, *zero, *tmp_out;
    void *z[3], *x[3];
    int64_t nflags, zero_words;
    size_t total;
};

PairLayout pair_layout(char *base, int64_t nA, int64_t nB, const twed_params *prm, Prec prec)
{
    const int dimt = dimt_for(prm->dim);
    const size_t cs = cost_size(prec), as = acc_size(prec);
    const size_t S = (size_t)row_stride(prec, dimt);
    Carver c{base};
    PairLayout L{};
    L.rowsA = take_rows(c, prec, dimt, nA + 1);
    L.rowsB = take_rows(c, prec, dimt, nB + 1);
    if (prm->algo == TWED_ALGO_DIAGONAL) {
        for (int i = 0; i < 3; ++i) L.z[i] = c.take((size_t)(nB + 1) * as);
        for (int i = 0; i < 3; ++i) L.x[i] = c.take((size_t)(nB + 1) * as);
        L.bnd = nullptr;
        L.nflags = 0;
    } else {
        L.bnd = c.take((size_t)2 * (size_t)(nA + 1) * 2 * as);
        L.nflags = (nB + 63) / 64;  // flags for the narrowest strips
    }
    // zeroed words: flags, then ticket, error word and the FP32 cost offset
    L.zero_words = L.nflags + kTailWords;
    L.zero = c.take((size_t)L.zero_words * 4);
    L.tmp_out = c.take(8);
    L.total = c.used;
    return L;
}

// ---- sweep configuration and its tuning cache ---------------------------------------
//
// A single-pair sweep is configured by the strip width K (columns per lane),
// the group size G (strips per workgroup) and the in-group handoff interval.
// The defaults come from occupancy rules; twed_pair_tune measures the
// candidates on the caller's own pair and caches the fastest per
// (precision, dimension, distance, nB), which later calls with strip_k = 0
// use.
struct SweepChoice {
    int K, G, sub_shift;
};

// Identity of the current device in the tuning caches (architecture name and
// compute-unit count), so that a saved cache serves only the same hardware.
std::string device_id()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);
    return arch + "-cu" + std::to_string(prop.multiProcessorCount);
}

using TuneKey = std::tuple<std::string, int, int, int, int64_t>;

std::mutex &tune_mutex()
{
    static std::mutex m;
    return m;
}

std::map<TuneKey, SweepChoice> &tune_cache()
{
    static std::map<TuneKey, SweepChoice> c;
    return c;
}

bool tuned_choice(Prec prec, const CostParams &cp, int64_t nB, SweepChoice *out)
{
    std::lock_guard<std::mutex> lock(tune_mutex());
    const auto it = tune_cache().find(TuneKey{device_id(), (int)prec, cp.dimt, cp.pm, nB});
    if (it == tune_cache().end()) return false;
    *out = it->second;
    return true;
}

// ---- strips of two widths ---------------------------------------------------------------
//
// With every strip resident, strip s starts lag_s of its own steps after
// strip s-1 and then runs nA + 63 steps: the lag is 64 + 16 inside a group
// (the lane skew and the in-group handoff interval) and 64 + 64 where the
// boundary leaves the group through a global window.  A step of K columns
// per lane costs about K + 1/2 cells of time (the boundary shifts, loads and
// stores of the step).  The sweep ends when its last strip of either width
// ends.  choose_mixed_split returns the number s1 of wide strips of a layout
// that minimises that end with at most `slots` strips in all (every strip
// resident), or 0 when no split beats uniform strips of the wide width by
// 1% (or when uniform strips would not all be resident either).
int64_t choose_mixed_split(const MixedLayout &L, int64_t nA, int64_t nB, int64_t slots)
{
    const int K = L.wide, K2 = L.narrow, G = L.group;
    constexpr double h = 0.5, lag_in = 80.0, lag_out = 128.0;
    auto lags = [&](int64_t n) { return lag_in * (double)n + (lag_out - lag_in) * (double)(n / G); };
    const double run = (double)(nA + 63);
    const int64_t su = (nB + 64 * K - 1) / (64 * K);
    if (su > slots) return 0;
    double best = 0.99 * ((K + h) * lags(su - 1) + run * (K + h));
    int64_t best_s1 = 0;
    for (int64_t s1 = 1; s1 < su; ++s1) {
        const int64_t S = s1 + (nB - 64 * K * s1 + 64 * K2 - 1) / (64 * K2);
        if (S > slots) continue;
        const double end_wide = (K + h) * lags(s1 - 1) + run * (K + h);
        const double start_last = (K + h) * lags(s1) + (K2 + h) * (lags(S - 1) - lags(s1));
        const double end = std::max(end_wide, start_last + run * (K2 + h));
        if (end < best) {
            best = end;
            best_s1 = s1;
        }
    }
    return best_s1;
}

// Configuration of one single-pair strip sweep.
struct SweepPlan {
    int K, G, sub_shift;
    int layout;       // two-width layout (kMixedLayouts), when s1 > 0
    int64_t s1;       // wide strips of a two-width sweep (0: uniform strips of K)
    int64_t nStrips;
    int grid;         // workgroups launched
};

twed_status plan_pair_sweep(Prec prec, const CostParams &cp, const twed_params *prm, int64_t nA, int64_t nB,
                            bool dump, const SweepChoice *force, SweepPlan *plan)
{
    SweepChoice tuned{};
    const bool have_tuned = !force && !dump && prm->strip_k == 0 && tuned_choice(prec, cp, nB, &tuned);
    int K = force ? force->K : (have_tuned ? tuned.K : choose_k(prm, nB, prec, cp));
    if (dump) {
        // cell dumps exist for narrow strips only (a validation aid)
        if (prm->strip_k > 2) return fail(TWED_ERR_UNSUPPORTED, "twed_pair_matrix takes strip_k 0, 1 or 2");
        K = std::min(K, 2);
    }
    plan->K = K;
    plan->s1 = 0;
    plan->nStrips = (nB + 64 * K - 1) / (64 * K);
    // Strips per workgroup: in-group handoffs go through LDS, one in G
    // through global memory.  The widest group that still leaves about
    // three groups for every four CUs and whose kernel keeps to registers
    // (eight waves put two on each SIMD, which halves the registers a lane
    // may hold: too few for the widest high-dimensional strips); cell dumps
    // use single-wave groups.
    // TWED_WAVEFRONT_GROUP
    // (1, 4 or 8) and TWED_WAVEFRONT_SUB (in-group handoff rows: 8, 16 or 32)
    // override the choices for tuning runs.
    const int64_t cus = std::max(1, device_simds() / 4);
    plan->G = 1;
    for (int G : {8, 4})
        if (plan->nStrips * 4 >= (int64_t)G * cus * 3 && wavefront_scratch_bytes(prec, cp, K, G) == 0) {
            plan->G = G;
            break;
        }
    if (dump) plan->G = 1;
    if (const char *env = std::getenv("TWED_WAVEFRONT_GROUP")) {
        const int G = std::atoi(env);
        if ((G == 1 || G == 4 || G == 8) && !dump) plan->G = G;
    }
    plan->sub_shift = 4;
    if (const char *env = std::getenv("TWED_WAVEFRONT_SUB")) {
        const int v = std::atoi(env);
        if (v == 8 || v == 16 || v == 32) plan->sub_shift = v == 8 ? 3 : (v == 16 ? 4 : 5);
    }
    if (have_tuned) {
        plan->G = tuned.G;
        plan->sub_shift = tuned.sub_shift;
    }
    if (force) {
        plan->G = force->G;
        plan->sub_shift = force->sub_shift;
    }
    // Strips of two widths where the widest strips in groups of eight would
    // leave workgroup slots empty: the first compiled, register-resident
    // layout of kMixedLayouts that beats uniform strips.
    // TWED_WAVEFRONT_LAYOUT picks one layout (its index; -1 none) and
    // TWED_WAVEFRONT_MIXED the number of wide strips (0 none); results do not
    // depend on either.
    plan->layout = -1;
    if (!dump && K == 8 && plan->G == 8 && plan->nStrips > 1) {
        int only = -2;
        if (const char *env = std::getenv("TWED_WAVEFRONT_LAYOUT")) only = std::atoi(env);
        int64_t forced = -1;
        if (const char *env = std::getenv("TWED_WAVEFRONT_MIXED")) forced = std::max<int64_t>(0, std::atoll(env));
        for (int m = 0; m < kNumMixedLayouts && forced != 0; ++m) {
            if (only != -2 && m != only) continue;
            if (!wavefront_mixed_compiled(prec, cp, m) || wavefront_mixed_scratch_bytes(prec, cp, m) != 0) continue;
            const MixedLayout &L = kMixedLayouts[m];
            const int mworkers = wavefront_mixed_max_workers(prec, cp, m);
            if (mworkers <= 0) return fail(TWED_ERR_DEVICE, "occupancy query failed");
            const int64_t su = (nB + 64 * L.wide - 1) / (64 * L.wide);
            int64_t s1 = forced > 0 ? forced : choose_mixed_split(L, nA, nB, (int64_t)mworkers * L.group);
            s1 = std::min<int64_t>(s1, su - 1);
            if (s1 <= 0) continue;
            plan->layout = m;
            plan->K = L.wide;
            plan->G = L.group;
            plan->s1 = s1;
            plan->nStrips = s1 + (nB - 64 * L.wide * s1 + 64 * L.narrow - 1) / (64 * L.narrow);
            plan->grid = (int)std::min<int64_t>((plan->nStrips + L.group - 1) / L.group, mworkers);
            return TWED_OK;
        }
    }
    const int workers = wavefront_max_workers(prec, cp, K, plan->G);
    if (workers <= 0) return fail(TWED_ERR_DEVICE, "occupancy query failed");
    plan->grid = (int)std::min<int64_t>((plan->nStrips + plan->G - 1) / plan->G, workers);
    return TWED_OK;
}

// Runs the sweep of one pair whose rows are already staged.
// `tail` points at the kTailWords words after the flags (zeroed beforehand).
twed_status run_pair_sweep(Prec prec, const CostParams &cp, const twed_params *prm, const void *rowsA,
                           const void *rowsB, int64_t nA, int64_t nB, void *bnd, uint32_t *flags,
                           uint32_t *tail, const PairLayout *diag_layout, void *out, void *dump,
                           hipStream_t st, const SweepChoice *force = nullptr)
{
    hipError_t e;
    void *beta = tail + 2;
    if (prec == kF32 && std::max(nA, nB) > kOffsetMinLength) {
        e = launch_offset(prec, cp, rowsA, nA, rowsB, nB, beta, st);
        if (e != hipSuccess) return fail_hip(e, "offset launch");
    }
    if (prm->algo == TWED_ALGO_DIAGONAL) {
        if (!diag_layout) return fail(TWED_ERR_UNSUPPORTED, "no single-pair sweep available for this call");
        DiagonalArgs d{};
        d.rowsA = rowsA;
        d.rowsB = rowsB;
        d.nA = nA;
        d.nB = nB;
        for (int i = 0; i < 3; ++i) {
            d.z[i] = diag_layout->z[i];
            d.x[i] = diag_layout->x[i];
        }
        d.beta = beta;
        d.out = out;
        d.dump = dump;
        e = launch_diagonal(prec, cp, d, st);
        if (e != hipSuccess) return fail_hip(e, "diagonal sweep launch");
        return TWED_OK;
    }
    SweepPlan plan{};
    twed_status s = plan_pair_sweep(prec, cp, prm, nA, nB, dump != nullptr, force, &plan);
    if (s != TWED_OK) return s;
    WavefrontArgs w{};
    w.rowsA = rowsA;
    w.rowsB = rowsB;
    w.nA = nA;
    w.nB = nB;
    w.bnd = bnd;
    w.flags = flags;
    w.ticket = tail;
    w.beta = beta;
    w.nStrips = plan.nStrips;
    w.out = out;
    w.dump = dump;
    w.group = plan.G;
    w.sub_shift = plan.sub_shift;
    w.s1 = (int)plan.s1;
    w.grid = plan.grid;
    e = plan.s1 > 0 ? launch_wavefront_mixed(prec, cp, plan.layout, w, st) : launch_wavefront(prec, cp, plan.K, w, st);
    if (e != hipSuccess) return fail_hip(e, "wavefront sweep launch");
    return TWED_OK;
}

// Argument checks of a single-pair call (no HIP call).
twed_status check_pair_args(const void *A, const void *TA, int64_t nA, const void *B, const void *TB, int64_t nB,
                            const twed_params *prm, const void *out)
{
    twed_status s = check_params(prm);
    if (s != TWED_OK) return s;
    if (!A || !TA || !B || !TB || !out) return fail(TWED_ERR_INVALID, "NULL array argument");
    if (nA < 1 || nB < 1) return fail(TWED_ERR_INVALID, "series lengths must be >= 1");
    if (nA > kMaxLen || nB > kMaxLen) return fail(TWED_ERR_UNSUPPORTED, "series longer than 2^31 - 130");
    return TWED_OK;
}

twed_status pair_impl(const void *A, const void *TA, int64_t nA, const void *B, const void *TB, int64_t nB,
                      const twed_params *prm, void *out, void *dp, void *ws, size_t ws_bytes, hipStream_t st)
{
    twed_status s = check_pair_args(A, TA, nA, B, TB, nB, prm, out);
    if (s != TWED_OK) return s;
    const Prec prec = resolve(prm, std::max(nA, nB));
    const PairLayout need = pair_layout(nullptr, nA, nB, prm, prec);
    s = check_workspace(ws, ws_bytes, need.total);
    if (s != TWED_OK) return s;

    const PairLayout L = pair_layout((char *)ws, nA, nB, prm, prec);
    const CostParams cp = cost_params(prm);
    uint32_t *flags = (uint32_t *)L.zero;
    uint32_t *tail = flags + L.nflags;
    hipError_t e;
    // stage A (zeroing flags and ticket on the way), then B
    e = launch_stage(prec, cp, A, TA, nullptr, 1, nA, nA, nA + 1, L.rowsA, flags, L.zero_words, st);
    if (e != hipSuccess) return fail_hip(e, "staging launch");
    e = launch_stage(prec, cp, B, TB, nullptr, 1, nB, nB, nB + 1, L.rowsB, nullptr, 0, st);
    if (e != hipSuccess) return fail_hip(e, "staging launch");
    if (dp) {
        e = launch_dump_border(prec, dp, nA, nB, st);
        if (e != hipSuccess) return fail_hip(e, "dump border launch");
    }
    const bool widen = needs_widen(prm, prec);
    void *kout = widen ? L.tmp_out : out;
    if (widen && dp) return fail(TWED_ERR_UNSUPPORTED, "twed_pair_matrix does not take TWED_AUTO");
    s = run_pair_sweep(prec, cp, prm, L.rowsA, L.rowsB, nA, nB, L.bnd, flags, tail, &L, kout, dp, st);
    if (s != TWED_OK) return s;
    if (widen) {
        e = launch_widen((const float *)kout, (double *)out, 1, st);
        if (e != hipSuccess) return fail_hip(e, "widen launch");
    }
    return TWED_OK;
}

// ---- the scratch array of the no-allocation pair call ---------------------------------
//
// One fixed device array per GPU stands in for the caller's workspace, so that
// callers that cannot allocate (code under graph capture, serving loops)
// still have one.  Host code never passes the array's name to a kernel: the
// name is a host-side stand-in, and the device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
constexpr size_t kNoAllocBytes = TWED_PAIR_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;

std::mutex &scratch_mutex()
{
    static std::mutex m;
    return m;
}

// Device address of `scratch` on the current device.
twed_status noalloc_scratch(void **out)
{
    static void *addr[kMaxDevices];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(TWED_ERR_UNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lock(scratch_mutex());
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return fail_hip(e, "hipGetSymbolAddress(scratch)");
        if (!p || ((uintptr_t)p) % kAlign) return fail(TWED_ERR_DEVICE, "scratch array address not 256-byte aligned");
        addr[dev] = p;
    }
    *out = addr[dev];
    return TWED_OK;
}

// ---- batch ----------------------------------------------------------------------

struct BatchLayout {
    void *rowsX, *rowsY, *offX, *offY, *order, *zero, *bnd, *flags, *tmpD;
    size_t total;
};

BatchLayout batch_layout(char *base, int64_t totX, int64_t nX, int64_t maxX, int64_t totY, int64_t nY,
                         int64_t maxY, bool symmetric, int64_t nOut, const twed_params *prm, Prec prec)
{
    const int dimt = dimt_for(prm->dim);
    const size_t cs = cost_size(prec), as = acc_size(prec);
    const size_t S = (size_t)row_stride(prec, dimt);
    Carver c{base};
    BatchLayout L{};
    L.rowsX = take_rows(c, prec, dimt, totX + nX);
    L.rowsY = symmetric ? L.rowsX : take_rows(c, prec, dimt, totY + nY);
    L.offX = c.take((size_t)(nX + 1) * 8);
    L.offY = symmetric ? L.offX : c.take((size_t)(nY + 1) * 8);
    L.order = c.take((size_t)nX * 4);
    L.zero = c.take(8);  // batch tickets: one per launch of the sweep
    // single-pair sweep state for pairs too long for one wave
    const int64_t maxlen = std::max(maxX, maxY);
    const int64_t kshort = twed_batch_max_short_length(prm->dim);
    if (std::min(maxX, maxY) > kshort) {
        L.bnd = c.take((size_t)2 * (size_t)(maxlen + 1) * 2 * as);
        L.flags = c.take((size_t)((maxlen + 63) / 64 + kTailWords) * 4);
    }
    if (needs_widen(prm, prec)) L.tmpD = c.take((size_t)nOut * 4);
    L.total = c.used;
    return L;
}

// ---- batch: preparation (host), upload and enqueue --------------------------------
//
// twed_batch = prepare + upload + enqueue in one call.  A twed_batch_plan
// keeps the prepared state so that later runs enqueue kernels only (and can
// therefore be captured in a HIP graph).
// A batch run is configured by the number of consecutive items a wave takes
// per work ticket, the resident waves per compute unit, and whether a single
// short query runs one lane per pair.  The defaults come from rules;
// twed_batch_plan_tune measures the candidates on a plan's own inputs and
// caches the fastest under the plan's size class, which later plans and
// twed_batch calls of that class use.
struct BatchConfig {
    int chunk = 0;         // items per ticket (0: rule)
    int waves_per_cu = 0;  // resident waves per compute unit (0: all that fit)
    int lane_mode = -1;    // single short query: 1 lane per pair (1), wave per pair (0), rule (-1)
};

// Size class: device, precision, compiled dimension, distance, mode, and the
// mean lengths of X and Y and the item count rounded down to powers of two.
using BatchKey = std::tuple<std::string, int, int, int, int, int, int, int>;

std::map<BatchKey, BatchConfig> &batch_cache()
{
    static std::map<BatchKey, BatchConfig> c;
    return c;
}

int floor_log2(double v) { return v < 2.0 ? 0 : (int)std::floor(std::log2(v)); }

struct BatchPlan {
    twed_params prm;
    Prec prec;
    CostParams cp;
    BatchLayout L;
    std::vector<int64_t> offX, offY;  // host copies (offY empty when symmetric)
    std::vector<int32_t> order;       // longest-first order (symmetric)
    int64_t nX, nY, maxX, maxY, totX, totY, nPairs;
    bool sym, list;
    bool y_staged = false;  // rows of Y staged by twed_batch_plan_stage_y
    BatchKey key;
    BatchConfig cfg;
};

int64_t batch_items(const BatchPlan &P)
{
    return P.list ? P.nPairs : (P.sym ? P.nX * (P.nX - 1) / 2 : P.nX * P.nY);
}

BatchKey batch_key(const BatchPlan &P)
{
    const int mode = P.list ? kPairList : (P.sym ? kSymmetric : kRect);
    return BatchKey{device_id(), (int)P.prec, P.cp.dimt, P.cp.pm, mode,
                    floor_log2((double)P.totX / (double)P.nX), floor_log2((double)P.totY / (double)P.nY),
                    floor_log2((double)std::max<int64_t>(1, batch_items(P)))};
}

// A single query short enough for one lane per pair (rectangular mode).
bool lane_eligible(const BatchPlan &P) { return !P.sym && !P.list && P.nX == 1 && P.maxX <= kLaneMaxQuery; }

twed_status batch_prepare(const int64_t *offX, int64_t nX, const int64_t *offY, int64_t nY, bool sym, bool list,
                          int64_t nPairs, const twed_params *prm, void *workspace, size_t ws_bytes, BatchPlan &P)
{
    twed_status s = check_params(prm);
    if (s != TWED_OK) return s;
    int64_t maxX, totX, maxY, totY;
    s = check_offsets(offX, nX, &maxX, &totX);
    if (s != TWED_OK) return s;
    if (sym) {
        if (offY) return fail(TWED_ERR_INVALID, "Y == NULL requires TY == NULL and offY == NULL");
        if (nY != nX) return fail(TWED_ERR_INVALID, "Y == NULL requires nY == nX");
        maxY = maxX;
        totY = totX;
    } else {
        s = check_offsets(offY, nY, &maxY, &totY);
        if (s != TWED_OK) return s;
    }
    if (list && nPairs < 0) return fail(TWED_ERR_INVALID, "nPairs must be >= 0");
    if (nX * nY > (int64_t(1) << 40)) return fail(TWED_ERR_UNSUPPORTED, "too many pairs");
    const Prec prec = resolve(prm, std::max(maxX, maxY));
    const BatchLayout need = batch_layout(nullptr, totX, nX, maxX, totY, nY, maxY, sym, nX * nY, prm, prec);
    s = check_workspace(workspace, ws_bytes, need.total);
    if (s != TWED_OK) return s;
    P.prm = *prm;
    P.prec = prec;
    P.cp = cost_params(prm);
    P.L = batch_layout((char *)workspace, totX, nX, maxX, totY, nY, maxY, sym, nX * nY, prm, prec);
    P.offX.assign(offX, offX + nX + 1);
    if (!sym) P.offY.assign(offY, offY + nY + 1);
    P.order.clear();
    if (sym) {
        P.order.resize((size_t)nX);
        std::iota(P.order.begin(), P.order.end(), 0);
        std::stable_sort(P.order.begin(), P.order.end(), [&](int32_t a, int32_t b) {
            return offX[a + 1] - offX[a] > offX[b + 1] - offX[b];
        });
    }
    P.nX = nX;
    P.nY = nY;
    P.maxX = maxX;
    P.maxY = maxY;
    P.totX = totX;
    P.totY = totY;
    P.nPairs = list ? nPairs : 0;
    P.sym = sym;
    P.list = list;
    P.key = batch_key(P);
    P.cfg = BatchConfig{};
    {
        std::lock_guard<std::mutex> lock(tune_mutex());
        const auto it = batch_cache().find(P.key);
        if (it != batch_cache().end()) P.cfg = it->second;
    }
    return TWED_OK;
}

// Copies the offsets and the order to the workspace (asynchronous unless
// `sync`, in which case the copies have completed on return).
twed_status batch_upload(const BatchPlan &P, hipStream_t st, bool sync)
{
    const BatchLayout &L = P.L;
    hipError_t e;
    if (sync) {
        e = hipMemcpy(L.offX, P.offX.data(), (size_t)(P.nX + 1) * 8, hipMemcpyHostToDevice);
        if (e == hipSuccess && !P.sym) e = hipMemcpy(L.offY, P.offY.data(), (size_t)(P.nY + 1) * 8,
                                                    hipMemcpyHostToDevice);
        if (e == hipSuccess && P.sym) e = hipMemcpy(L.order, P.order.data(), (size_t)P.nX * 4, hipMemcpyHostToDevice);
    } else {
        e = hipMemcpyAsync(L.offX, P.offX.data(), (size_t)(P.nX + 1) * 8, hipMemcpyHostToDevice, st);
        if (e == hipSuccess && !P.sym) e = hipMemcpyAsync(L.offY, P.offY.data(), (size_t)(P.nY + 1) * 8,
                                                         hipMemcpyHostToDevice, st);
        if (e == hipSuccess && P.sym) e = hipMemcpyAsync(L.order, P.order.data(), (size_t)P.nX * 4,
                                                        hipMemcpyHostToDevice, st);
    }
    if (e != hipSuccess) return fail_hip(e, "offset upload");
    return TWED_OK;
}

// Kernels only: staging (which also clears the work ticket), the sweeps, the
// mirror of the symmetric case and the widening of TWED_AUTO results.  With
// Y == NULL in the rectangular and pair-list cases the rows of Y staged
// earlier are used as they are.
twed_status batch_enqueue(const BatchPlan &P, const void *X, const void *TX, const void *Y, const void *TY,
                          const int64_t *pairs, void *D, hipStream_t st)
{
    const BatchLayout &L = P.L;
    const twed_params *prm = &P.prm;
    const Prec prec = P.prec;
    const CostParams &cp = P.cp;
    const int64_t nX = P.nX, nY = P.nY, maxX = P.maxX, maxY = P.maxY, totX = P.totX, totY = P.totY;
    const int64_t nPairs = P.nPairs;
    const bool sym = P.sym;
    const int64_t *offX = P.offX.data();
    const int64_t *offY = sym ? nullptr : P.offY.data();
    const int64_t kshort = twed_batch_max_short_length(prm->dim);
    if (P.list && nPairs == 0) return TWED_OK;
    twed_status s = TWED_OK;
    hipError_t e;
    e = launch_stage(prec, cp, X, TX, (const int64_t *)L.offX, nX, 0, maxX, totX + nX, L.rowsX,
                     (uint32_t *)L.zero, 2, st);
    if (e != hipSuccess) return fail_hip(e, "staging launch");
    // one short query reads the caller's collection as it is (no staging
    // pass); every other sweep reads staged rows
    const bool lane = lane_eligible(P) && P.cfg.lane_mode != 0;
    if (!sym && Y && !lane) {
        e = launch_stage(prec, cp, Y, TY, (const int64_t *)L.offY, nY, 0, maxY, totY + nY, L.rowsY, nullptr, 0,
                         st);
        if (e != hipSuccess) return fail_hip(e, "staging launch");
    }
    const bool widen = needs_widen(prm, prec);
    void *Dk = widen ? L.tmpD : D;
    const int64_t nOut = pairs ? nPairs : nX * nY;

    BatchArgs b{};
    b.rowsX = L.rowsX;
    b.rowsY = L.rowsY;
    b.offX = (const int64_t *)L.offX;
    b.offY = (const int64_t *)L.offY;
    b.order = (const int32_t *)L.order;
    b.pairs = pairs;
    b.nX = nX;
    b.nY = nY;
    b.mode = pairs ? kPairList : (sym ? kSymmetric : kRect);
    b.nItems = pairs ? nPairs : (sym ? nX * (nX - 1) / 2 : nX * nY);
    b.D = Dk;
    b.ticket = (uint32_t *)L.zero;
    if (b.nItems > 0xffffffffLL) return fail(TWED_ERR_UNSUPPORTED, "more than 2^32 - 1 pairs in one call");
    // Width classes: a pair's K (columns per lane) is ceil(shorter length /
    // 64).  Only pairs of K <= 8 need no more than the narrow kernel; in the
    // symmetric case the longest-first order puts every pair of K > 8 (both
    // series longer than 512 samples) before the others, so the items split
    // into a wide launch and a narrow one.
    const int kmax = batch_kmax(cp.dimt);
    const int64_t k_need = (std::min(maxX, maxY) + kWaveLanes - 1) / kWaveLanes;
    int64_t split = 0;  // symmetric: items [0, split) hold the pairs of K > 8
    int kclass = kBatchAll;
    if (k_need <= kBatchNarrowMax || kmax <= kBatchNarrowMax) {
        kclass = kBatchNarrow;
    } else if (sym) {
        int64_t J = 0;  // first series (in the order) of at most 512 samples
        while (J < nX && offX[P.order[J] + 1] - offX[P.order[J]] > (int64_t)kBatchNarrowMax * kWaveLanes) ++J;
        split = J * (J - 1) / 2;
        kclass = -1;  // two launches
    }
    const int cus = std::max(1, device_simds() / 4);
    auto workers_of = [&](int cls) {
        int wk = batch_max_workers(prec, cp, cls);
        if (P.cfg.waves_per_cu > 0) wk = std::min(wk, P.cfg.waves_per_cu * cus);
        return wk;
    };
    int workers = workers_of(kclass < 0 ? kBatchNarrow : kclass);
    if (workers <= 0) return fail(TWED_ERR_DEVICE, "occupancy query failed");
    if (sym) {
        e = launch_batch_diag_zero(prec, Dk, nX, st);
        if (e != hipSuccess) return fail_hip(e, "diagonal zero launch");
    }
    if (b.nItems > 0 && lane) {
        // one short query: a lane per pair
        e = launch_batch_lane(prec, cp, L.rowsX, (int)maxX, L.rowsY, Y, TY, (const int64_t *)L.offY, nY, Dk,
                              (uint32_t *)L.zero, (int)std::min<int64_t>((nY + 63) / 64, workers), st);
        if (e != hipSuccess) return fail_hip(e, "batch launch");
    } else if (b.nItems > 0) {
        int64_t chunk = P.cfg.chunk;
        if (chunk <= 0) {
            // items per ticket: about 64k cells of work per ticket for short
            // pairs, while leaving at least four tickets per wave
            const double cells = (double)totX / (double)nX * (double)totY / (double)nY;
            chunk = std::max<int64_t>(1, std::min<int64_t>(32, (int64_t)(65536.0 / std::max(cells, 1.0))));
            chunk = std::min<int64_t>(chunk, std::max<int64_t>(1, b.nItems / (4 * (int64_t)workers)));
        }
        b.chunk = (int)chunk;
        if (kclass >= 0) {
            b.kclass = kclass;
            b.grid = (int)std::min<int64_t>((b.nItems + chunk - 1) / chunk, workers);
            e = launch_batch(prec, cp, b, st);
            if (e != hipSuccess) return fail_hip(e, "batch launch");
        } else {
            // the wide pairs first (longest first), then the narrow ones on
            // the second ticket
            BatchArgs w = b;
            w.kclass = kBatchWide;
            w.nItems = split;
            const int wide_workers = workers_of(kBatchWide);
            if (wide_workers <= 0) return fail(TWED_ERR_DEVICE, "occupancy query failed");
            w.grid = (int)std::min<int64_t>((split + chunk - 1) / chunk, wide_workers);
            if (split > 0) {
                e = launch_batch(prec, cp, w, st);
                if (e != hipSuccess) return fail_hip(e, "batch launch");
            }
            BatchArgs nrw = b;
            nrw.kclass = kBatchNarrow;
            nrw.item0 = split;
            nrw.ticket = (uint32_t *)L.zero + 1;
            nrw.grid = (int)std::min<int64_t>((b.nItems - split + chunk - 1) / chunk, workers);
            if (b.nItems > split) {
                e = launch_batch(prec, cp, nrw, st);
                if (e != hipSuccess) return fail_hip(e, "batch launch");
            }
        }
    }

    // listed pairs whose shorter series exceeds one wave (the batch kernel
    // leaves them): the list is read back and each runs the single-pair sweep
    if (pairs && std::min(maxX, maxY) > kshort) {
        s = sweep_long_listed_pairs(prec, cp, prm, L.rowsX, offX, nX, L.rowsY, sym ? offX : offY, nY, pairs, nPairs,
                                    L.bnd, std::max(maxX, maxY), Dk, st);
        if (s != TWED_OK) return s;
    }
    // pairs whose shorter series exceeds one wave: single-pair sweeps
    if (!pairs && std::min(maxX, maxY) > kshort) {
        const size_t S = (size_t)row_stride(prec, cp.dimt), cs = cost_size(prec), as = acc_size(prec);
        const int64_t maxlen = std::max(maxX, maxY);
        const int64_t nflags = (maxlen + 63) / 64, zero_words = nflags + kTailWords;
        const int64_t *offYh = sym ? offX : offY;
        for (int64_t i = 0; i < nX; ++i) {
            const int64_t li = offX[i + 1] - offX[i];
            if (li <= kshort) continue;
            for (int64_t j = sym ? i + 1 : 0; j < nY; ++j) {
                const int64_t lj = offYh[j + 1] - offYh[j];
                if (lj <= kshort) continue;
                const char *ra = (const char *)L.rowsX + (size_t)(offX[i] + i) * S * cs;
                const char *rb = (const char *)L.rowsY + (size_t)(offYh[j] + j) * S * cs;
                // the longer series streams, the shorter spreads over the lanes
                const bool swap = lj > li;
                const int64_t nA = swap ? lj : li, nB = swap ? li : lj;
                // zero flags and ticket (the staging kernel's zeroing pass)
                e = launch_stage(prec, cp, X, TX, (const int64_t *)L.offX, 0, 0, 0, totX + nX, L.rowsX,
                                 (uint32_t *)L.flags, zero_words, st);
                if (e != hipSuccess) return fail_hip(e, "flag reset launch");
                uint32_t *flags = (uint32_t *)L.flags;
                char *dst = (char *)Dk + (size_t)(i * nY + j) * as;
                s = run_pair_sweep(prec, cp, prm, swap ? rb : ra, swap ? ra : rb, nA, nB, L.bnd, flags,
                                   flags + nflags, nullptr, dst, nullptr, st);
                if (s != TWED_OK) return s;
                if (sym) {
                    e = launch_copy_one(prec, dst, (char *)Dk + (size_t)(j * nY + i) * as, st);
                    if (e != hipSuccess) return fail_hip(e, "mirror launch");
                }
            }
        }
    }
    if (widen) {
        e = launch_widen((const float *)Dk, (double *)D, nOut, st);
        if (e != hipSuccess) return fail_hip(e, "widen launch");
    }
    return TWED_OK;
}

}  // namespace

namespace twed {
namespace capi {

size_t long_pair_state_bytes(Prec prec, int64_t maxlen)
{
    const size_t as = acc_size(prec);
    return align_up((size_t)2 * (size_t)(maxlen + 1) * 2 * as) +
           align_up((size_t)((maxlen + 63) / 64 + kTailWords) * 4);
}

twed_status sweep_long_listed_pairs(Prec prec, const CostParams &cp, const twed_params *prm, const void *rowsX,
                                    const int64_t *offX, int64_t nX, const void *rowsY, const int64_t *offY,
                                    int64_t nY, const int64_t *pairs, int64_t nPairs, void *state,
                                    int64_t maxlen, void *D, hipStream_t st)
{
    if (nPairs <= 0) return TWED_OK;
    std::vector<int64_t> hp((size_t)nPairs * 2);
    hipError_t e = hipMemcpyAsync(hp.data(), pairs, (size_t)nPairs * 16, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail_hip(e, "pair list read-back");
    const int64_t kshort = twed_batch_max_short_length(prm->dim);
    const size_t S = (size_t)row_stride(prec, cp.dimt), cs = cost_size(prec), as = acc_size(prec);
    const int64_t nflags = (maxlen + 63) / 64, zero_words = nflags + kTailWords;
    void *bnd = state;
    uint32_t *flags = (uint32_t *)((char *)state + align_up((size_t)2 * (size_t)(maxlen + 1) * 2 * as));
    for (int64_t k = 0; k < nPairs; ++k) {
        const int64_t i = hp[2 * k], j = hp[2 * k + 1];
        if (i < 0 || i >= nX || j < 0 || j >= nY) continue;  // NaN, written by the batch kernel
        const int64_t li = offX[i + 1] - offX[i], lj = offY[j + 1] - offY[j];
        if (std::min(li, lj) <= kshort) continue;  // swept by the batch kernel
        const char *ra = (const char *)rowsX + (size_t)(offX[i] + i) * S * cs;
        const char *rb = (const char *)rowsY + (size_t)(offY[j] + j) * S * cs;
        const bool swap = lj > li;  // the longer series streams
        e = launch_zero32(flags, zero_words, st);
        if (e != hipSuccess) return fail_hip(e, "flag reset launch");
        twed_status s = run_pair_sweep(prec, cp, prm, swap ? rb : ra, swap ? ra : rb, swap ? lj : li,
                                       swap ? li : lj, bnd, flags, flags + nflags, nullptr,
                                       (char *)D + (size_t)k * as, nullptr, st);
        if (s != TWED_OK) return s;
    }
    return TWED_OK;
}

}  // namespace capi
}  // namespace twed

extern "C" {

void twed_params_default(twed_params *prm)
{
    if (!prm) return;
    std::memset(prm, 0, sizeof(*prm));
    prm->nu = 0.001;
    prm->lambda = 1.0;
    prm->p = 1.0;
    prm->dim = 1;
    prm->precision = TWED_F64;
    prm->algo = TWED_ALGO_AUTO;
    prm->strip_k = 0;
    prm->acc64_threshold = 0;
}

size_t twed_pair_workspace_size(int64_t nA, int64_t nB, const twed_params *prm)
{
    if (check_params(prm) != TWED_OK || nA < 1 || nB < 1 || nA > kMaxLen || nB > kMaxLen) return 0;
    return pair_layout(nullptr, nA, nB, prm, resolve(prm, std::max(nA, nB))).total;
}

twed_status twed_pair(const void *A, const void *TA, int64_t nA, const void *B, const void *TB, int64_t nB,
                      const twed_params *prm, void *out, void *workspace, size_t ws_bytes, hipStream_t stream)
{
    last_error().clear();
    return pair_impl(A, TA, nA, B, TB, nB, prm, out, nullptr, workspace, ws_bytes, stream);
}

twed_status twed_pair_config(int64_t nA, int64_t nB, const twed_params *prm, int32_t *strip_k, int32_t *group,
                             int64_t *wide_strips, int64_t *strips)
{
    last_error().clear();
    twed_status s = check_params(prm);
    if (s != TWED_OK) return s;
    if (nA < 1 || nB < 1) return fail(TWED_ERR_INVALID, "series lengths must be >= 1");
    if (nA > kMaxLen || nB > kMaxLen) return fail(TWED_ERR_UNSUPPORTED, "series longer than 2^31 - 130");
    if (prm->algo == TWED_ALGO_DIAGONAL) return fail(TWED_ERR_INVALID, "the per-diagonal sweep has no strips");
    SweepPlan plan{};
    s = plan_pair_sweep(resolve(prm, std::max(nA, nB)), cost_params(prm), prm, nA, nB, false, nullptr, &plan);
    if (s != TWED_OK) return s;
    if (strip_k) *strip_k = plan.K;
    if (group) *group = plan.G;
    if (wide_strips) *wide_strips = plan.s1;
    if (strips) *strips = plan.nStrips;
    return TWED_OK;
}

twed_status twed_pair_noalloc(const void *A, const void *TA, int64_t nA, const void *B, const void *TB,
                              int64_t nB, const twed_params *prm, void *out, hipStream_t stream)
{
    last_error().clear();
    twed_status s = check_pair_args(A, TA, nA, B, TB, nB, prm, out);
    if (s != TWED_OK) return s;
    const size_t need = pair_layout(nullptr, nA, nB, prm, resolve(prm, std::max(nA, nB))).total;
    if (need > kNoAllocBytes) {
        char msg[160];
        std::snprintf(msg, sizeof msg,
                      "pair needs %zu bytes of scratch; twed_pair_noalloc holds %zu (use twed_pair with a workspace)",
                      need, kNoAllocBytes);
        return fail(TWED_ERR_UNSUPPORTED, msg);
    }
    void *ws = nullptr;
    s = noalloc_scratch(&ws);
    if (s != TWED_OK) return s;
    return pair_impl(A, TA, nA, B, TB, nB, prm, out, nullptr, ws, kNoAllocBytes, stream);
}

twed_status twed_pair_matrix(const void *A, const void *TA, int64_t nA, const void *B, const void *TB, int64_t nB,
                             const twed_params *prm, void *out, void *dp, void *workspace, size_t ws_bytes,
                             hipStream_t stream)
{
    last_error().clear();
    if (!dp) return fail(TWED_ERR_INVALID, "dp is NULL");
    return pair_impl(A, TA, nA, B, TB, nB, prm, out, dp, workspace, ws_bytes, stream);
}

static twed_status twed_pair_tune_body(const void *A, const void *TA, int64_t nA, const void *B, const void *TB, int64_t nB,
                                       const twed_params *prm, void *workspace, size_t ws_bytes, hipStream_t st,
                                       int32_t *strip_k, int32_t *group)
{
    last_error().clear();
    twed_status s = check_params(prm);
    if (s != TWED_OK) return s;
    if (!A || !TA || !B || !TB) return fail(TWED_ERR_INVALID, "NULL array argument");
    if (nA < 1 || nB < 1) return fail(TWED_ERR_INVALID, "series lengths must be >= 1");
    if (nA > kMaxLen || nB > kMaxLen) return fail(TWED_ERR_UNSUPPORTED, "series longer than 2^31 - 130");
    if (prm->algo == TWED_ALGO_DIAGONAL) return fail(TWED_ERR_INVALID, "only the wavefront sweep is tuned");
    const Prec prec = resolve(prm, std::max(nA, nB));
    const PairLayout need = pair_layout(nullptr, nA, nB, prm, prec);
    s = check_workspace(workspace, ws_bytes, need.total);
    if (s != TWED_OK) return s;
    const PairLayout L = pair_layout((char *)workspace, nA, nB, prm, prec);
    const CostParams cp = cost_params(prm);
    uint32_t *flags = (uint32_t *)L.zero;
    uint32_t *tail = flags + L.nflags;
    hipError_t e;
    // the cost per row is uniform, so a prefix of A long enough to cover the
    // pipeline's fill and drain ranks the candidates
    const int64_t rows = std::min<int64_t>(nA, 262144);
    e = launch_stage(prec, cp, B, TB, nullptr, 1, nB, nB, nB + 1, L.rowsB, nullptr, 0, st);
    if (e != hipSuccess) return fail_hip(e, "staging launch");
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if ((e = hipEventCreate(&ev0)) != hipSuccess || (e = hipEventCreate(&ev1)) != hipSuccess) {
        if (ev0) hipEventDestroy(ev0);
        return fail_hip(e, "event create");
    }
    SweepChoice best{0, 0, 4};
    float best_ms = 0.f;
    twed_params p1 = *prm;
    p1.strip_k = 0;
    for (int K : {8, 4, 2, 1}) {
        if (wavefront_scratch_bytes(prec, cp, K, 1) != 0) continue;
        const int64_t strips = (nB + 64 * K - 1) / (64 * K);
        for (int G : {8, 4, 1}) {
            if (G > 1 && (strips < 2 * G || wavefront_scratch_bytes(prec, cp, K, G) != 0)) continue;
            const SweepChoice c{K, G, 4};
            // restaging A zeroes the flags and the ticket for this run
            e = launch_stage(prec, cp, A, TA, nullptr, 1, rows, rows, rows + 1, L.rowsA, flags, L.zero_words, st);
            if (e == hipSuccess) e = hipEventRecord(ev0, st);
            if (e != hipSuccess) break;
            s = run_pair_sweep(prec, cp, &p1, L.rowsA, L.rowsB, rows, nB, L.bnd, flags, tail, &L, L.tmp_out,
                               nullptr, st, &c);
            if (s != TWED_OK) break;
            if ((e = hipEventRecord(ev1, st)) != hipSuccess || (e = hipEventSynchronize(ev1)) != hipSuccess) break;
            float ms = 0.f;
            if ((e = hipEventElapsedTime(&ms, ev0, ev1)) != hipSuccess) break;
            if (best.K == 0 || ms < best_ms) {
                best = c;
                best_ms = ms;
            }
        }
        if (e != hipSuccess || s != TWED_OK) break;
    }
    hipEventDestroy(ev0);
    hipEventDestroy(ev1);
    if (s != TWED_OK) return s;
    if (e != hipSuccess) return fail_hip(e, "tuning run");
    if (best.K == 0) return fail(TWED_ERR_UNSUPPORTED, "no sweep configuration fits this pair");
    {
        std::lock_guard<std::mutex> lock(tune_mutex());
        tune_cache()[TuneKey{device_id(), (int)prec, cp.dimt, cp.pm, nB}] = best;
    }
    if (strip_k) *strip_k = best.K;
    if (group) *group = best.G;
    return TWED_OK;
}

twed_status twed_pair_tune(const void *A, const void *TA, int64_t nA, const void *B, const void *TB, int64_t nB,
                           const twed_params *prm, void *workspace, size_t ws_bytes, hipStream_t st,
                           int32_t *strip_k, int32_t *group)
{
    return no_throw([&] {
        return twed_pair_tune_body(A, TA, nA, B, TB, nB, prm, workspace, ws_bytes, st, strip_k, group);
    });
}

void twed_tune_clear(void)
{
    std::lock_guard<std::mutex> lock(tune_mutex());
    tune_cache().clear();
    batch_cache().clear();
}

int64_t twed_batch_max_short_length(int32_t dim)
{
    const int dimt = dimt_for(dim < 1 ? 1 : dim);
    if (dimt < 0) return 0;
    return (int64_t)64 * batch_kmax(dimt);
}

size_t twed_batch_workspace_size(const int64_t *offX, int64_t nX, const int64_t *offY, int64_t nY,
                                 const twed_params *prm)
{
    if (check_params(prm) != TWED_OK) return 0;
    int64_t maxX, totX, maxY, totY;
    if (check_offsets(offX, nX, &maxX, &totX) != TWED_OK) return 0;
    const bool sym = offY == nullptr;
    if (sym) {
        maxY = maxX;
        totY = totX;
        nY = nX;
    } else if (check_offsets(offY, nY, &maxY, &totY) != TWED_OK) {
        return 0;
    }
    const Prec prec = resolve(prm, std::max(maxX, maxY));
    // the output count is unknown here for pair lists: size for the larger
    const int64_t nOut = nX * nY;
    return batch_layout(nullptr, totX, nX, maxX, totY, nY, maxY, sym, nOut, prm, prec).total;
}

static twed_status twed_batch_body(const void *X, const void *TX, const int64_t *offX, int64_t nX, const void *Y,
                                   const void *TY, const int64_t *offY, int64_t nY, const int64_t *pairs, int64_t nPairs,
                                   const twed_params *prm, void *D, void *workspace, size_t ws_bytes, hipStream_t st)
{
    last_error().clear();
    if (!prm) return fail(TWED_ERR_INVALID, "params is NULL");
    if (!X || !TX || !D) return fail(TWED_ERR_INVALID, "NULL array argument");
    const bool sym = Y == nullptr;
    if (sym && TY) return fail(TWED_ERR_INVALID, "Y == NULL requires TY == NULL and offY == NULL");
    if (!sym && !TY) return fail(TWED_ERR_INVALID, "NULL array argument");
    BatchPlan P;
    twed_status s = batch_prepare(offX, nX, offY, nY, sym, pairs != nullptr, nPairs, prm, workspace, ws_bytes, P);
    if (s != TWED_OK) return s;
    if (P.list && nPairs == 0) return TWED_OK;
    s = batch_upload(P, st, false);
    if (s != TWED_OK) return s;
    return batch_enqueue(P, X, TX, Y, TY, pairs, D, st);
}

twed_status twed_batch(const void *X, const void *TX, const int64_t *offX, int64_t nX, const void *Y,
                       const void *TY, const int64_t *offY, int64_t nY, const int64_t *pairs, int64_t nPairs,
                       const twed_params *prm, void *D, void *workspace, size_t ws_bytes, hipStream_t st)
{
    return no_throw([&] {
        return twed_batch_body(X, TX, offX, nX, Y, TY, offY, nY, pairs, nPairs, prm, D, workspace, ws_bytes, st);
    });
}

}  // extern "C"

struct twed_batch_plan {
    BatchPlan p;
};

extern "C" {

static twed_status twed_batch_plan_create_body(const int64_t *offX, int64_t nX, const int64_t *offY, int64_t nY, int64_t nPairs,
                                               const twed_params *prm, void *workspace, size_t ws_bytes, twed_batch_plan **out)
{
    last_error().clear();
    if (!out) return fail(TWED_ERR_INVALID, "out is NULL");
    if (!prm) return fail(TWED_ERR_INVALID, "params is NULL");
    if (nPairs < 0) return fail(TWED_ERR_INVALID, "nPairs must be >= 0");
    twed_batch_plan *plan = new (std::nothrow) twed_batch_plan();
    if (!plan) return fail(TWED_ERR_DEVICE, "host allocation failed");
    if (!offY) nY = nX;  // symmetric plan: nY is ignored, as in twed_batch_workspace_size
    twed_status s = batch_prepare(offX, nX, offY, nY, offY == nullptr, nPairs > 0, nPairs, prm, workspace, ws_bytes,
                                  plan->p);
    if (s == TWED_OK) s = batch_upload(plan->p, nullptr, true);
    if (s != TWED_OK) {
        delete plan;
        return s;
    }
    *out = plan;
    return TWED_OK;
}

twed_status twed_batch_plan_create(const int64_t *offX, int64_t nX, const int64_t *offY, int64_t nY, int64_t nPairs,
                                   const twed_params *prm, void *workspace, size_t ws_bytes, twed_batch_plan **out)
{
    return no_throw([&] {
        return twed_batch_plan_create_body(offX, nX, offY, nY, nPairs, prm, workspace, ws_bytes, out);
    });
}

twed_status twed_batch_plan_run(const twed_batch_plan *plan, const void *X, const void *TX, const void *Y,
                                const void *TY, const int64_t *pairs, void *D, hipStream_t st)
{
    last_error().clear();
    if (!plan) return fail(TWED_ERR_INVALID, "plan is NULL");
    if (!X || !TX || !D) return fail(TWED_ERR_INVALID, "NULL array argument");
    const BatchPlan &P = plan->p;
    if ((Y == nullptr) != (TY == nullptr)) return fail(TWED_ERR_INVALID, "Y and TY must both be given or both NULL");
    if (P.sym && Y) return fail(TWED_ERR_INVALID, "a symmetric plan takes no Y");
    if (!P.sym && !Y && !P.y_staged)
        return fail(TWED_ERR_INVALID, "Y is NULL but twed_batch_plan_stage_y has not staged it");
    if (P.list != (pairs != nullptr)) return fail(TWED_ERR_INVALID, "pairs given exactly when the plan has nPairs > 0");
    return batch_enqueue(P, X, TX, Y, TY, pairs, D, st);
}

twed_status twed_batch_plan_stage_y(twed_batch_plan *plan, const void *Y, const void *TY, hipStream_t st)
{
    last_error().clear();
    if (!plan) return fail(TWED_ERR_INVALID, "plan is NULL");
    if (!Y || !TY) return fail(TWED_ERR_INVALID, "NULL array argument");
    BatchPlan &P = plan->p;
    if (P.sym) return fail(TWED_ERR_INVALID, "a symmetric plan takes no Y");
    const hipError_t e = launch_stage(P.prec, P.cp, Y, TY, (const int64_t *)P.L.offY, P.nY, 0, P.maxY,
                                      P.totY + P.nY, P.L.rowsY, nullptr, 0, st);
    if (e != hipSuccess) return fail_hip(e, "staging launch");
    P.y_staged = true;
    return TWED_OK;
}

void twed_batch_plan_destroy(twed_batch_plan *plan) { delete plan; }

twed_status twed_batch_plan_config(const twed_batch_plan *plan, int32_t *chunk, int32_t *waves_per_cu,
                                   int32_t *lane_mode)
{
    last_error().clear();
    if (!plan) return fail(TWED_ERR_INVALID, "plan is NULL");
    const BatchConfig &c = plan->p.cfg;
    if (chunk) *chunk = c.chunk;
    if (waves_per_cu) *waves_per_cu = c.waves_per_cu;
    if (lane_mode) *lane_mode = c.lane_mode;
    return TWED_OK;
}

static twed_status twed_batch_plan_tune_body(twed_batch_plan *plan, const void *X, const void *TX, const void *Y,
                                             const void *TY, const int64_t *pairs, void *D, hipStream_t st,
                                             int32_t *chunk, int32_t *waves_per_cu, int32_t *lane_mode)
{
    twed_status s = twed_batch_plan_run(plan, X, TX, Y, TY, pairs, D, st);  // validates; warm-up run
    if (s != TWED_OK) return s;
    BatchPlan &P = plan->p;
    const BatchConfig start = P.cfg;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipError_t e;
    if ((e = hipEventCreate(&ev0)) != hipSuccess || (e = hipEventCreate(&ev1)) != hipSuccess) {
        if (ev0) hipEventDestroy(ev0);
        return fail_hip(e, "event create");
    }
    // time of one run under configuration c (median of three)
    auto time_of = [&](const BatchConfig &c, float *ms_out) -> twed_status {
        P.cfg = c;
        float t[3];
        for (int r = 0; r < 3; ++r) {
            if ((e = hipEventRecord(ev0, st)) != hipSuccess) return fail_hip(e, "event record");
            twed_status s2 = batch_enqueue(P, X, TX, Y, TY, pairs, D, st);
            if (s2 != TWED_OK) return s2;
            if ((e = hipEventRecord(ev1, st)) != hipSuccess || (e = hipEventSynchronize(ev1)) != hipSuccess ||
                (e = hipEventElapsedTime(&t[r], ev0, ev1)) != hipSuccess)
                return fail_hip(e, "tuning run");
        }
        std::sort(t, t + 3);
        *ms_out = t[1];
        return TWED_OK;
    };
    BatchConfig best{};
    float best_ms = 0.f;
    auto consider = [&](const BatchConfig &c) -> twed_status {
        float ms = 0.f;
        twed_status s2 = time_of(c, &ms);
        if (s2 != TWED_OK) return s2;
        if (best_ms == 0.f || ms < best_ms) {
            best = c;
            best_ms = ms;
        }
        return TWED_OK;
    };
    // coordinate search: the rule's configuration, then the lane mode of a
    // single short query, the items per ticket, the resident waves per CU
    s = consider(BatchConfig{});
    if (s == TWED_OK && lane_eligible(P)) s = consider(BatchConfig{0, 0, 0});
    const bool lanes = lane_eligible(P) && best.lane_mode != 0;
    if (s == TWED_OK && !lanes) {
        const int64_t items = batch_items(P);
        for (int c : {1, 2, 4, 8, 16, 32, 64}) {
            if (c > 1 && c > items) break;
            BatchConfig t = best;
            t.chunk = c;
            if ((s = consider(t)) != TWED_OK) break;
        }
    }
    if (s == TWED_OK) {
        const int cus = std::max(1, device_simds() / 4);
        const int per_cu = batch_max_workers(P.prec, P.cp) / cus;
        for (int w : {per_cu / 4, per_cu / 2, (3 * per_cu) / 4}) {
            if (w < 1) continue;
            BatchConfig t = best;
            t.waves_per_cu = w;
            if ((s = consider(t)) != TWED_OK) break;
        }
    }
    hipEventDestroy(ev0);
    hipEventDestroy(ev1);
    if (s != TWED_OK) {
        P.cfg = start;
        return s;
    }
    P.cfg = best;
    {
        std::lock_guard<std::mutex> lock(tune_mutex());
        batch_cache()[P.key] = best;
    }
    if (chunk) *chunk = best.chunk;
    if (waves_per_cu) *waves_per_cu = best.waves_per_cu;
    if (lane_mode) *lane_mode = best.lane_mode;
    return TWED_OK;
}

twed_status twed_batch_plan_tune(twed_batch_plan *plan, const void *X, const void *TX, const void *Y, const void *TY,
                                 const int64_t *pairs, void *D, hipStream_t stream, int32_t *chunk,
                                 int32_t *waves_per_cu, int32_t *lane_mode)
{
    last_error().clear();
    return no_throw([&] {
        return twed_batch_plan_tune_body(plan, X, TX, Y, TY, pairs, D, stream, chunk, waves_per_cu, lane_mode);
    });
}

// Tuning cache file: a header line, then one line per entry,
//   pair  <device> <precision> <dimt> <pm> <nB> <K> <G> <sub_shift>
//   batch <device> <precision> <dimt> <pm> <mode> <lx> <ly> <items> <chunk> <waves_per_cu> <lane_mode>
static const char kTuneHeader[] = "libtwed-tune 1";

static twed_status twed_tune_save_body(const char *path)
{
    if (!path) return fail(TWED_ERR_INVALID, "path is NULL");
    std::string text = std::string(kTuneHeader) + "\n";
    {
        std::lock_guard<std::mutex> lock(tune_mutex());
        char line[512];
        for (const auto &kv : tune_cache()) {
            const auto &k = kv.first;
            std::snprintf(line, sizeof line, "pair %s %d %d %d %lld %d %d %d\n", std::get<0>(k).c_str(),
                          std::get<1>(k), std::get<2>(k), std::get<3>(k), (long long)std::get<4>(k), kv.second.K,
                          kv.second.G, kv.second.sub_shift);
            text += line;
        }
        for (const auto &kv : batch_cache()) {
            const auto &k = kv.first;
            std::snprintf(line, sizeof line, "batch %s %d %d %d %d %d %d %d %d %d %d\n", std::get<0>(k).c_str(),
                          std::get<1>(k), std::get<2>(k), std::get<3>(k), std::get<4>(k), std::get<5>(k),
                          std::get<6>(k), std::get<7>(k), kv.second.chunk, kv.second.waves_per_cu,
                          kv.second.lane_mode);
            text += line;
        }
    }
    FILE *f = std::fopen(path, "w");
    if (!f) return fail(TWED_ERR_INVALID, "cannot open the tuning cache file for writing");
    const bool ok = std::fwrite(text.data(), 1, text.size(), f) == text.size();
    if (std::fclose(f) != 0 || !ok) return fail(TWED_ERR_INVALID, "cannot write the tuning cache file");
    return TWED_OK;
}

twed_status twed_tune_save(const char *path)
{
    last_error().clear();
    return no_throw([&] { return twed_tune_save_body(path); });
}

static twed_status twed_tune_load_body(const char *path)
{
    if (!path) return fail(TWED_ERR_INVALID, "path is NULL");
    FILE *f = std::fopen(path, "r");
    if (!f) return fail(TWED_ERR_INVALID, "cannot open the tuning cache file");
    std::map<TuneKey, SweepChoice> pairs;
    std::map<BatchKey, BatchConfig> batches;
    char line[512];
    bool header = false, bad = false;
    while (std::fgets(line, sizeof line, f)) {
        std::string l(line);
        while (!l.empty() && (l.back() == '\n' || l.back() == '\r')) l.pop_back();
        if (!header) {
            header = l == kTuneHeader;
            if (!header) bad = true;
            if (bad) break;
            continue;
        }
        if (l.empty()) continue;
        char kind[16], dev[128];
        int a[10];
        long long n = 0;
        if (std::sscanf(l.c_str(), "%15s", kind) != 1) { bad = true; break; }
        if (std::strcmp(kind, "pair") == 0 &&
            std::sscanf(l.c_str(), "pair %127s %d %d %d %lld %d %d %d", dev, &a[0], &a[1], &a[2], &n, &a[3], &a[4],
                        &a[5]) == 8 &&
            (a[3] == 1 || a[3] == 2 || a[3] == 4 || a[3] == 8) && (a[4] == 1 || a[4] == 4 || a[4] == 8) &&
            a[5] >= 3 && a[5] <= 5) {
            pairs[TuneKey{dev, a[0], a[1], a[2], (int64_t)n}] = SweepChoice{a[3], a[4], a[5]};
        } else if (std::strcmp(kind, "batch") == 0 &&
                   std::sscanf(l.c_str(), "batch %127s %d %d %d %d %d %d %d %d %d %d", dev, &a[0], &a[1], &a[2],
                               &a[3], &a[4], &a[5], &a[6], &a[7], &a[8], &a[9]) == 11 &&
                   a[7] >= 0 && a[7] <= 4096 && a[8] >= 0 && a[8] <= 64 && a[9] >= -1 && a[9] <= 1) {
            batches[BatchKey{dev, a[0], a[1], a[2], a[3], a[4], a[5], a[6]}] = BatchConfig{a[7], a[8], a[9]};
        } else {
            bad = true;
            break;
        }
    }
    std::fclose(f);
    if (bad || !header) return fail(TWED_ERR_INVALID, "malformed tuning cache file");
    std::lock_guard<std::mutex> lock(tune_mutex());
    for (const auto &kv : pairs) tune_cache()[kv.first] = kv.second;
    for (const auto &kv : batches) batch_cache()[kv.first] = kv.second;
    return TWED_OK;
}

twed_status twed_tune_load(const char *path)
{
    last_error().clear();
    return no_throw([&] { return twed_tune_load_body(path); });
}

const char *twed_status_string(twed_status s)
{
    switch (s) {
    case TWED_OK: return "ok";
    case TWED_ERR_INVALID: return "invalid argument";
    case TWED_ERR_UNSUPPORTED: return "unsupported argument";
    case TWED_ERR_WORKSPACE: return "workspace too small or misaligned";
    case TWED_ERR_DEVICE: return "device error";
    default: return "unknown status";
    }
}

const char *twed_last_error(void) { return last_error().c_str(); }

twed_status twed_stream_check(hipStream_t stream)
{
    last_error().clear();
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail_hip(e, "stream synchronize");
    e = hipGetLastError();
    if (e != hipSuccess) return fail_hip(e, "pending error");
    return TWED_OK;
}

const char *twed_version(void) { return "libtwed 0.1 (gfx950)"; }

}  // extern "C"

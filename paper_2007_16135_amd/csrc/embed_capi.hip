// embed_capi.hip -- extern "C" boundary of the embedding network and the
// learned k-NN index: validation, workspace layout and launch order.
//
// Host code only.  The network's arithmetic is in cnn.hip, the candidate
// selection in knn.hip, and the exact re-rank is the batched TWED sweep of
// batch.hip in its pair-list mode.
#include "../../include/twed_knn.h"
#include "capi_util.h"
#include "cnn_kernels.h"
#include "twed_kernels.h"

#include <algorithm>
#include <atomic>
#include <cstring>
#include <new>
#include <vector>

using namespace twed;
using namespace twed::capi;
using namespace twed::cnn;

struct twed_knn_index {
    const float *DB, *TDB, *params;
    std::vector<int64_t> off;
    int64_t nDB, total, maxlen;
    twed_params prm;
    char *storage;
    size_t storage_bytes;
    bool built;
    // carved from storage
    uint16_t *emb16;
    float *sqnorm;
    int64_t *off_dev;
    void *rows;
};

namespace {

// Default rows of one forward chunk for large collections (whole series per
// chunk) and score-matrix bytes per query chunk of a k-NN call; both can be
// lowered (or raised) with twed_embed_set_limits.
constexpr int64_t kDefaultChunkRows = int64_t(1) << 22;
constexpr int64_t kDefaultScoreBytes = int64_t(1) << 30;
std::atomic<int64_t> g_chunk_rows{kDefaultChunkRows};
std::atomic<int64_t> g_score_bytes{kDefaultScoreBytes};

struct Weights {
    uint16_t *wt[kLayers], *wb[kLayers];
};

void take_weights(Carver &c, Weights &w)
{
    for (int l = 0; l < kLayers; ++l) {
        w.wt[l] = (uint16_t *)c.take((size_t)layer_w_count(l) * 2);
        w.wb[l] = (uint16_t *)c.take((size_t)layer_w_count(l) * 2);
    }
}

hipError_t make_weights(const float *params, const Weights &w, hipStream_t st)
{
    for (int l = 0; l < kLayers; ++l) {
        hipError_t e = launch_weight_copies(params + layer_offset(l), kChan[l], kChan[l + 1], w.wt[l], w.wb[l], st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Activations of a chunk of `rows` packed rows.  With `keep` every layer's
// input stays (training); otherwise layers 1 and 3 share a buffer.
struct Acts {
    uint32_t *row_info;
    int32_t *row_series;
    uint16_t *feat;
    uint16_t *h[3];  // inputs of layers 2, 3, 4
    float *y4;
};

void take_acts(Carver &c, Acts &a, int64_t rows, bool keep)
{
    a.row_info = (uint32_t *)c.take((size_t)rows * 4);
    a.row_series = keep ? (int32_t *)c.take((size_t)rows * 4) : nullptr;
    a.feat = (uint16_t *)c.take((size_t)rows * 2 * 2);
    a.h[0] = (uint16_t *)c.take((size_t)rows * 64 * 2);
    a.h[1] = (uint16_t *)c.take((size_t)rows * 64 * 2);
    a.h[2] = keep ? (uint16_t *)c.take((size_t)rows * 64 * 2) : a.h[0];
    a.y4 = (float *)c.take((size_t)rows * kC4 * 4);
}

// y = conv(h; W_l) + b_l as an implicit GEMM over R packed rows.
hipError_t conv_forward(int l, const float *params, const Weights &w, const Acts &a, const uint16_t *in, void *out,
                        int64_t R, hipStream_t st)
{
    GemmArgs g;
    g.M = (int)R;
    g.N = kChan[l + 1];
    g.K = kKsize * kChan[l];
    g.a_mode = kAConv;
    g.A = in;
    g.conv_C = kChan[l];
    g.row_info = a.row_info;
    g.B = w.wt[l];
    g.ldb_k = 1;
    g.ldb_n = g.K;
    g.C = out;
    g.ldc = g.N;
    g.bias = params + layer_offset(l) + layer_w_count(l);
    g.relu = l < kLayers - 1;
    return launch_gemm(l < kLayers - 1 ? kOutBF16 : kOutF32, g, 1, st);
}

// Forward pass of nS series (device offsets `off` into X, packed rows from
// row_base) -> embeddings.
hipError_t forward(const float *params, const Weights &w, const Acts &a, const float *X, const int64_t *off, int nS,
                   int64_t row_base, int64_t R, int maxlen, float *emb, uint16_t *emb16, float *sqnorm,
                   hipStream_t st)
{
    hipError_t e = launch_features(X, off, nS, row_base, R, maxlen, a.row_info, a.row_series, a.feat, st);
    if (e != hipSuccess) return e;
    const uint16_t *in = a.feat;
    for (int l = 0; l < kLayers; ++l) {
        void *out = l < kLayers - 1 ? (void *)a.h[l] : (void *)a.y4;
        e = conv_forward(l, params, w, a, in, out, R, st);
        if (e != hipSuccess) return e;
        if (l < kLayers - 1) in = a.h[l];
    }
    return launch_pool(a.y4, off, nS, row_base, R, emb, emb16, sqnorm, st);
}

// Rows of the activation buffers: the whole collection if it fits the
// chunk limit, else the limit, but never less than the longest series (a
// series is never split across chunks).
int64_t chunk_rows_for(int64_t total, int64_t maxlen)
{
    return std::min(total, std::max(g_chunk_rows.load(std::memory_order_relaxed), maxlen));
}

// Chunked forward over a whole collection (host offsets offH, device offD).
hipError_t forward_all(const float *params, const Weights &w, const Acts &a, const float *X, const int64_t *offH,
                       const int64_t *offD, int64_t n, int64_t cap, float *emb, uint16_t *emb16, float *sqnorm,
                       hipStream_t st)
{
    int64_t s0 = 0;
    while (s0 < n) {
        int64_t s1 = s0 + 1;
        int maxlen = (int)(offH[s0 + 1] - offH[s0]);
        while (s1 < n && offH[s1 + 1] - offH[s0] <= cap) {
            maxlen = std::max(maxlen, (int)(offH[s1 + 1] - offH[s1]));
            ++s1;
        }
        const int64_t R = offH[s1] - offH[s0];
        hipError_t e = forward(params, w, a, X, offD + s0, (int)(s1 - s0), offH[s0], R, maxlen,
                               emb ? emb + s0 * kEmb : nullptr, emb16 ? emb16 + s0 * kEmb : nullptr,
                               sqnorm ? sqnorm + s0 : nullptr, st);
        if (e != hipSuccess) return e;
        s0 = s1;
    }
    return hipSuccess;
}

twed_status check_network_offsets(const int64_t *off, int64_t n, int64_t *maxlen, int64_t *total)
{
    twed_status s = check_offsets(off, n, maxlen, total);
    if (s != TWED_OK) return s;
    if (*maxlen > kMaxSeriesLen) return fail(TWED_ERR_UNSUPPORTED, "series longer than twed_embed_max_length()");
    if (n > 0x7fffffffLL) return fail(TWED_ERR_UNSUPPORTED, "more than 2^31 - 1 series");
    return TWED_OK;
}

struct EmbedLayout {
    int64_t *off;
    Weights w;
    Acts a;
    float *emb, *demb;
    void *dy[3];  // bf16 gradients: [R][64] twice (ping-pong), [R][4]
    float *wpart;  // per-workgroup weight-gradient partials
    size_t total;
};

EmbedLayout embed_layout(char *base, int64_t n, int64_t total, int64_t maxlen, int64_t nPairs)
{
    Carver c{base};
    EmbedLayout L{};
    L.off = (int64_t *)c.take((size_t)(n + 1) * 8);
    take_weights(c, L.w);
    const bool train = nPairs > 0;
    take_acts(c, L.a, train ? total : chunk_rows_for(total, maxlen), train);
    if (train) {
        L.emb = (float *)c.take((size_t)n * kEmb * 4);
        L.demb = (float *)c.take((size_t)n * kEmb * 4);
        L.dy[0] = c.take((size_t)total * 64 * 2);
        L.dy[1] = c.take((size_t)total * 64 * 2);
        L.dy[2] = c.take((size_t)total * kC4 * 2);
        L.wpart = (float *)c.take(conv_wgrad_partial_bytes(total));
    }
    L.total = c.used;
    return L;
}

// Split-K factor for a weight-gradient GEMM over R rows.
int splitk_for(int64_t R, int tiles)
{
    int64_t z = (R + 511) / 512;
    const int64_t cap = std::max<int64_t>(1, 2048 / std::max(1, tiles));
    return (int)std::max<int64_t>(1, std::min(z, cap));
}

}  // namespace

namespace {

bool knn_params_ok(const twed_params *prm)
{
    if (check_params(prm) != TWED_OK) return false;
    if (prm->dim != 1) {
        fail(TWED_ERR_UNSUPPORTED, "the k-NN index takes 1-D series (dim = 1)");
        return false;
    }
    if (prm->precision != TWED_F32) {
        fail(TWED_ERR_UNSUPPORTED, "the k-NN index re-ranks in TWED_F32");
        return false;
    }
    return true;
}

struct IndexLayout {
    uint16_t *emb16;
    float *sqnorm;
    int64_t *off;
    void *rows;
    size_t total;
};

IndexLayout index_layout(char *base, int64_t nDB, int64_t total)
{
    Carver c{base};
    IndexLayout L{};
    L.emb16 = (uint16_t *)c.take((size_t)nDB * kEmb * 2);
    L.sqnorm = (float *)c.take((size_t)nDB * 4);
    L.off = (int64_t *)c.take((size_t)(nDB + 1) * 8);
    L.rows = take_rows(c, kF32, dimt_for(1), total + nDB);
    L.total = c.used;
    return L;
}

struct BuildLayout {
    Weights w;
    Acts a;
    size_t total;
};

BuildLayout build_layout(char *base, int64_t total, int64_t maxlen)
{
    Carver c{base};
    BuildLayout L{};
    take_weights(c, L.w);
    take_acts(c, L.a, chunk_rows_for(total, maxlen), false);
    L.total = c.used;
    return L;
}

int64_t queries_per_chunk(int64_t nQ, int64_t nDB)
{
    const int64_t bytes = g_score_bytes.load(std::memory_order_relaxed);
    return std::max<int64_t>(1, std::min<int64_t>(nQ, bytes / (nDB * 4)));
}

struct KnnLayout {
    int64_t *offQ;
    void *rowsQ;
    uint32_t *ticket;
    Weights w;
    Acts a;
    uint16_t *emb16;
    float *sqnorm, *scores, *dist;
    int32_t *cand;
    int64_t *pairs;
    void *long_state;  // single-pair sweep state, when queries and database both hold long series
    size_t total;
};

KnnLayout knn_layout(char *base, int64_t nQ, int64_t totQ, int64_t maxQ, int64_t nDB, int64_t maxDB,
                     int64_t n_cand)
{
    Carver c{base};
    KnnLayout L{};
    L.offQ = (int64_t *)c.take((size_t)(nQ + 1) * 8);
    L.rowsQ = take_rows(c, kF32, dimt_for(1), totQ + nQ);
    L.ticket = (uint32_t *)c.take(4);
    take_weights(c, L.w);
    take_acts(c, L.a, chunk_rows_for(totQ, maxQ), false);
    L.emb16 = (uint16_t *)c.take((size_t)nQ * kEmb * 2);
    L.sqnorm = (float *)c.take((size_t)nQ * 4);
    L.scores = (float *)c.take((size_t)queries_per_chunk(nQ, nDB) * nDB * 4);
    L.cand = (int32_t *)c.take((size_t)nQ * n_cand * 4);
    L.pairs = (int64_t *)c.take((size_t)nQ * n_cand * 16);
    L.dist = (float *)c.take((size_t)nQ * n_cand * 4);
    L.long_state = std::min(maxQ, maxDB) > twed_batch_max_short_length(1)
                       ? c.take(long_pair_state_bytes(kF32, std::max(maxQ, maxDB)))
                       : nullptr;
    L.total = c.used;
    return L;
}

}  // namespace

extern "C" {

int64_t twed_embed_param_count(void) { return kParamCount; }

int64_t twed_embed_max_length(void) { return kMaxSeriesLen; }

void twed_embed_set_limits(int64_t chunk_rows, int64_t score_bytes)
{
    g_chunk_rows.store(chunk_rows > 0 ? chunk_rows : kDefaultChunkRows, std::memory_order_relaxed);
    g_score_bytes.store(score_bytes > 0 ? score_bytes : kDefaultScoreBytes, std::memory_order_relaxed);
}

size_t twed_embed_workspace_size(const int64_t *off, int64_t nSeries, int64_t nPairs)
{
    int64_t maxlen, total;
    if (nPairs < 0 || check_network_offsets(off, nSeries, &maxlen, &total) != TWED_OK) return 0;
    return embed_layout(nullptr, nSeries, total, maxlen, nPairs).total;
}

twed_status twed_embed_forward(const float *params, const float *X, const int64_t *off, int64_t nSeries, float *emb,
                               void *workspace, size_t ws_bytes, hipStream_t st)
{
    last_error().clear();
    if (!params || !X || !emb) return fail(TWED_ERR_INVALID, "NULL array argument");
    int64_t maxlen, total;
    twed_status s = check_network_offsets(off, nSeries, &maxlen, &total);
    if (s != TWED_OK) return s;
    s = check_workspace(workspace, ws_bytes, embed_layout(nullptr, nSeries, total, maxlen, 0).total);
    if (s != TWED_OK) return s;
    const EmbedLayout L = embed_layout((char *)workspace, nSeries, total, maxlen, 0);
    hipError_t e = hipMemcpyAsync(L.off, off, (size_t)(nSeries + 1) * 8, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return fail_hip(e, "offset upload");
    e = make_weights(params, L.w, st);
    if (e != hipSuccess) return fail_hip(e, "weight copies");
    e = forward_all(params, L.w, L.a, X, off, L.off, nSeries, chunk_rows_for(total, maxlen), emb, nullptr, nullptr,
                    st);
    if (e != hipSuccess) return fail_hip(e, "forward launch");
    return TWED_OK;
}

twed_status twed_embed_loss_grad(const float *params, const float *X, const int64_t *off, int64_t nSeries,
                                 const int32_t *pairs, const float *target, int64_t nPairs, float *loss, float *grad,
                                 float *emb, void *workspace, size_t ws_bytes, hipStream_t st)
{
    last_error().clear();
    if (!params || !X || !pairs || !target || !loss || !grad) return fail(TWED_ERR_INVALID, "NULL array argument");
    if (nPairs < 1) return fail(TWED_ERR_INVALID, "nPairs must be >= 1");
    if (nPairs > 0x7fffffffLL) return fail(TWED_ERR_UNSUPPORTED, "more than 2^31 - 1 pairs");
    int64_t maxlen, total;
    twed_status s = check_network_offsets(off, nSeries, &maxlen, &total);
    if (s != TWED_OK) return s;
    if (total > 0x7fffffffLL) return fail(TWED_ERR_UNSUPPORTED, "more than 2^31 - 1 samples in one training batch");
    s = check_workspace(workspace, ws_bytes, embed_layout(nullptr, nSeries, total, maxlen, nPairs).total);
    if (s != TWED_OK) return s;
    const EmbedLayout L = embed_layout((char *)workspace, nSeries, total, maxlen, nPairs);
    const Acts &a = L.a;
    const int64_t R = total;
    float *E = emb ? emb : L.emb;
    hipError_t e;
#define TRY(call, what)                       \
    do {                                      \
        e = (call);                           \
        if (e != hipSuccess) return fail_hip(e, what); \
    } while (0)
    TRY(hipMemcpyAsync(L.off, off, (size_t)(nSeries + 1) * 8, hipMemcpyHostToDevice, st), "offset upload");
    TRY(make_weights(params, L.w, st), "weight copies");
    TRY(forward(params, L.w, a, X, L.off, (int)nSeries, 0, R, (int)maxlen, E, nullptr, nullptr, st), "forward");
    TRY(launch_fill(L.demb, nSeries * kEmb, 0.f, st), "fill");
    TRY(launch_fill(grad, kParamCount, 0.f, st), "fill");
    TRY(launch_fill(loss, 1, 0.f, st), "fill");
    TRY(launch_pair_loss(E, pairs, target, (int)nPairs, (int)nSeries, L.demb, loss, st), "pair loss");
    uint16_t *dy_out = (uint16_t *)L.dy[2];
    TRY(launch_pool_bwd(L.demb, a.row_info, a.row_series, R, dy_out, st), "pool backward");
    const uint16_t *inputs[kLayers] = {a.feat, a.h[0], a.h[1], a.h[2]};
    for (int l = kLayers - 1; l >= 0; --l) {
        const int cin = kChan[l], cout = kChan[l + 1];
        float *gW = grad + layer_offset(l);
        float *gb = gW + layer_w_count(l);
        // dW_l[(tap, c)][n] = sum_r h_l[r + tap - 2][c] dy_l[r][n], db_l[n] = sum_r dy_l[r][n]
        if (conv_staged_enabled() && conv_wgrad_fits(cin, cout)) {
            TRY(launch_conv_wgrad(cin, cout, inputs[l], a.row_info, dy_out, R, L.wpart, gW, st), "weight gradient");
        } else {
            GemmArgs g;
            g.M = kKsize * cin;
            g.N = cout;
            g.K = (int)R;
            g.a_mode = kAConvT;
            g.A = inputs[l];
            g.conv_C = cin;
            g.row_info = a.row_info;
            g.B = dy_out;
            g.ldb_k = cout;
            g.ldb_n = 1;
            g.C = gW;
            g.ldc = cout;
            const int tiles = ((g.M + 63) / 64) * ((g.N + 63) / 64);
            TRY(launch_gemm(kOutAtomic, g, splitk_for(R, tiles), st), "weight gradient");
            TRY(launch_colsum(dy_out, R, cout, gb, st), "bias gradient");
        }
        if (l == 0) break;
        // dy_{l-1}[r][c] = sum_{u, n} dy_l[r + u - 2][n] W_l[4 - u][c][n], times [h_l > 0]
        uint16_t *dy_in = (uint16_t *)L.dy[l & 1];
        GemmArgs d;
        d.M = (int)R;
        d.N = cin;
        d.K = kKsize * cout;
        d.a_mode = kAConv;
        d.A = dy_out;
        d.conv_C = cout;
        d.row_info = a.row_info;
        d.B = L.w.wb[l];
        d.ldb_k = 1;
        d.ldb_n = d.K;
        d.C = dy_in;
        d.ldc = cin;
        d.mask = inputs[l];
        TRY(launch_gemm(kOutBF16, d, 1, st), "data gradient");
        dy_out = dy_in;
    }
#undef TRY
    return TWED_OK;
}

twed_status twed_embed_adamw(float *params, float *m, float *v, const float *grad, int64_t step, float lr,
                             float weight_decay, hipStream_t st)
{
    last_error().clear();
    if (!params || !m || !v || !grad) return fail(TWED_ERR_INVALID, "NULL array argument");
    if (step < 1) return fail(TWED_ERR_INVALID, "step must be >= 1");
    if (!(lr >= 0.f) || !(weight_decay >= 0.f)) return fail(TWED_ERR_INVALID, "lr and weight_decay must be >= 0");
    hipError_t e = launch_adamw(params, m, v, grad, kParamCount, lr, weight_decay, step, st);
    if (e != hipSuccess) return fail_hip(e, "adamw launch");
    return TWED_OK;
}

size_t twed_knn_index_storage_size(const int64_t *offDB, int64_t nDB, const twed_params *prm)
{
    int64_t maxlen, total;
    if (!knn_params_ok(prm) || check_network_offsets(offDB, nDB, &maxlen, &total) != TWED_OK) return 0;
    return index_layout(nullptr, nDB, total).total;
}

static twed_status twed_knn_index_create_body(const void *DB, const void *TDB, const int64_t *offDB, int64_t nDB,
                                              const float *params, const twed_params *prm, void *storage, size_t storage_bytes,
                                              twed_knn_index **out)
{
    last_error().clear();
    if (!out) return fail(TWED_ERR_INVALID, "out is NULL");
    if (!DB || !TDB || !params) return fail(TWED_ERR_INVALID, "NULL array argument");
    if (!knn_params_ok(prm)) return check_params(prm) != TWED_OK ? check_params(prm) : TWED_ERR_UNSUPPORTED;
    int64_t maxlen, total;
    twed_status s = check_network_offsets(offDB, nDB, &maxlen, &total);
    if (s != TWED_OK) return s;
    const IndexLayout need = index_layout(nullptr, nDB, total);
    if (storage_bytes < need.total) return fail(TWED_ERR_WORKSPACE, "storage smaller than twed_knn_index_storage_size()");
    if (!storage || ((uintptr_t)storage) % kAlign) return fail(TWED_ERR_WORKSPACE, "storage NULL or not 256-byte aligned");
    twed_knn_index *ix = new (std::nothrow) twed_knn_index();
    if (!ix) return fail(TWED_ERR_DEVICE, "host allocation failed");
    ix->DB = (const float *)DB;
    ix->TDB = (const float *)TDB;
    ix->params = params;
    ix->off.assign(offDB, offDB + nDB + 1);
    ix->nDB = nDB;
    ix->total = total;
    ix->maxlen = maxlen;
    ix->prm = *prm;
    ix->storage = (char *)storage;
    ix->storage_bytes = storage_bytes;
    ix->built = false;
    const IndexLayout L = index_layout((char *)storage, nDB, total);
    ix->emb16 = L.emb16;
    ix->sqnorm = L.sqnorm;
    ix->off_dev = L.off;
    ix->rows = L.rows;
    *out = ix;
    return TWED_OK;
}

twed_status twed_knn_index_create(const void *DB, const void *TDB, const int64_t *offDB, int64_t nDB,
                                  const float *params, const twed_params *prm, void *storage, size_t storage_bytes,
                                  twed_knn_index **out)
{
    return no_throw([&] {
        return twed_knn_index_create_body(DB, TDB, offDB, nDB, params, prm, storage, storage_bytes, out);
    });
}

size_t twed_knn_index_build_workspace_size(const twed_knn_index *ix)
{
    if (!ix) return 0;
    return build_layout(nullptr, ix->total, ix->maxlen).total;
}

twed_status twed_knn_index_build(twed_knn_index *ix, void *workspace, size_t ws_bytes, hipStream_t st)
{
    last_error().clear();
    if (!ix) return fail(TWED_ERR_INVALID, "index is NULL");
    twed_status s = check_workspace(workspace, ws_bytes, build_layout(nullptr, ix->total, ix->maxlen).total);
    if (s != TWED_OK) return s;
    const BuildLayout L = build_layout((char *)workspace, ix->total, ix->maxlen);
    hipError_t e = hipMemcpyAsync(ix->off_dev, ix->off.data(), (size_t)(ix->nDB + 1) * 8, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return fail_hip(e, "offset upload");
    const CostParams cp = cost_params(&ix->prm);
    e = launch_stage(kF32, cp, ix->DB, ix->TDB, ix->off_dev, ix->nDB, 0, ix->maxlen, ix->total + ix->nDB, ix->rows,
                     nullptr, 0, st);
    if (e != hipSuccess) return fail_hip(e, "staging launch");
    e = make_weights(ix->params, L.w, st);
    if (e != hipSuccess) return fail_hip(e, "weight copies");
    e = forward_all(ix->params, L.w, L.a, ix->DB, ix->off.data(), ix->off_dev, ix->nDB,
                    chunk_rows_for(ix->total, ix->maxlen), nullptr, ix->emb16, ix->sqnorm, st);
    if (e != hipSuccess) return fail_hip(e, "forward launch");
    ix->built = true;
    return TWED_OK;
}

size_t twed_knn_workspace_size(const twed_knn_index *ix, const int64_t *offQ, int64_t nQ, int32_t k, int32_t n_cand)
{
    int64_t maxlen, total;
    if (!ix || k < 1 || n_cand < k || n_cand > ix->nDB) return 0;
    if (check_network_offsets(offQ, nQ, &maxlen, &total) != TWED_OK) return 0;
    return knn_layout(nullptr, nQ, total, maxlen, ix->nDB, ix->maxlen, n_cand).total;
}

twed_status twed_knn(const twed_knn_index *ix, const void *Q, const void *TQ, const int64_t *offQ, int64_t nQ,
                     int32_t k, int32_t n_cand, int64_t *ids, float *dist, void *workspace, size_t ws_bytes,
                     hipStream_t st)
{
    last_error().clear();
    if (!ix) return fail(TWED_ERR_INVALID, "index is NULL");
    if (!ix->built) return fail(TWED_ERR_INVALID, "index not built (twed_knn_index_build)");
    if (!Q || !TQ || !ids || !dist) return fail(TWED_ERR_INVALID, "NULL array argument");
    if (k < 1 || n_cand < k || n_cand > ix->nDB) return fail(TWED_ERR_INVALID, "need 1 <= k <= n_cand <= nDB");
    int64_t maxQ, totQ;
    twed_status s = check_network_offsets(offQ, nQ, &maxQ, &totQ);
    if (s != TWED_OK) return s;
    const int64_t nItems = nQ * (int64_t)n_cand;
    if (nItems > 0xffffffffLL) return fail(TWED_ERR_UNSUPPORTED, "more than 2^32 - 1 query-candidate pairs");
    s = check_workspace(workspace, ws_bytes, knn_layout(nullptr, nQ, totQ, maxQ, ix->nDB, ix->maxlen, n_cand).total);
    if (s != TWED_OK) return s;
    const KnnLayout L = knn_layout((char *)workspace, nQ, totQ, maxQ, ix->nDB, ix->maxlen, n_cand);
    const CostParams cp = cost_params(&ix->prm);
    hipError_t e;
#define TRY(call, what)                                \
    do {                                               \
        e = (call);                                    \
        if (e != hipSuccess) return fail_hip(e, what); \
    } while (0)
    TRY(hipMemcpyAsync(L.offQ, offQ, (size_t)(nQ + 1) * 8, hipMemcpyHostToDevice, st), "offset upload");
    // queries staged for the sweep (zeroing the batch ticket), then embedded
    TRY(launch_stage(kF32, cp, Q, TQ, L.offQ, nQ, 0, maxQ, totQ + nQ, L.rowsQ, L.ticket, 1, st), "staging");
    TRY(make_weights(ix->params, L.w, st), "weight copies");
    TRY(forward_all(ix->params, L.w, L.a, (const float *)Q, offQ, L.offQ, nQ, chunk_rows_for(totQ, maxQ), nullptr,
                    L.emb16, L.sqnorm, st),
        "forward");
    // squared embedding distances and the n_cand smallest per query
    const int64_t qc = queries_per_chunk(nQ, ix->nDB);
    for (int64_t q0 = 0; q0 < nQ; q0 += qc) {
        const int64_t nq = std::min(qc, nQ - q0);
        GemmArgs g;
        g.M = (int)nq;
        g.N = (int)ix->nDB;
        g.K = kEmb;
        g.a_mode = kAPlain;
        g.A = L.emb16 + q0 * kEmb;
        g.lda_m = kEmb;
        g.lda_k = 1;
        g.B = ix->emb16;
        g.ldb_k = 1;
        g.ldb_n = kEmb;
        g.C = L.scores;
        g.ldc = ix->nDB;
        g.row_norm = L.sqnorm + q0;
        g.col_norm = ix->sqnorm;
        TRY(launch_gemm(kOutDist, g, 1, st), "score launch");
        TRY(launch_topk_select(L.scores, ix->nDB, (int)nq, (int)ix->nDB, n_cand, L.cand + q0 * n_cand, st),
            "selection launch");
    }
    // exact FP32 TWED of every (query, candidate) pair
    TRY(launch_make_pairs(L.cand, (int)nQ, n_cand, (int)ix->nDB, 0, L.pairs, st), "pair list");
    BatchArgs b{};
    b.rowsX = L.rowsQ;
    b.rowsY = ix->rows;
    b.offX = L.offQ;
    b.offY = ix->off_dev;
    b.order = nullptr;
    b.pairs = L.pairs;
    b.nX = nQ;
    b.nY = ix->nDB;
    b.nItems = nItems;
    b.mode = kPairList;
    b.D = L.dist;
    b.ticket = L.ticket;
    // pairs of at most 8 columns per lane (both series of at most 512
    // samples) run the narrow kernel, which fits more waves per SIMD
    const int64_t k_need = (std::min(maxQ, ix->maxlen) + kWaveLanes - 1) / kWaveLanes;
    b.kclass = k_need <= kBatchNarrowMax ? kBatchNarrow : kBatchAll;
    const int workers = batch_max_workers(kF32, cp, b.kclass);
    if (workers <= 0) return fail(TWED_ERR_DEVICE, "occupancy query failed");
    b.grid = (int)std::min<int64_t>(nItems, workers);
    TRY(launch_batch(kF32, cp, b, st), "re-rank launch");
    if (L.long_state) {
        // pairs of two series longer than one wave's strip: single-pair sweeps
        s = sweep_long_listed_pairs(kF32, cp, &ix->prm, L.rowsQ, offQ, nQ, ix->rows, ix->off.data(), ix->nDB,
                                    L.pairs, nItems, L.long_state, std::max(maxQ, ix->maxlen), L.dist, st);
        if (s != TWED_OK) return s;
    }
    TRY(launch_final_topk(L.dist, L.cand, (int)nQ, n_cand, k, ids, dist, st), "final selection");
#undef TRY
    return TWED_OK;
}

void twed_knn_index_destroy(twed_knn_index *ix) { delete ix; }

}  // extern "C"

/*
 * twed_knn.h -- learned k-nearest-neighbour search under TWED, and the
 * embedding network behind it (libtwed, gfx950).
 *
 * The paper motivates TWED as a proper metric for machine-learning and
 * exploratory work over large collections of series (Introduction), and its
 * validation section singles out collections meant for database indexing;
 * an exhaustive k-NN query there costs one full TWED per database series.
 * This interface adds a learned pruning stage that the paper does not have:
 * a small 1-D convolutional network maps every series to a 128-d embedding
 * whose Euclidean distances are trained to follow TWED; a query takes the
 * n_cand database series nearest in the embedding, computes their exact
 * TWED (the batched sweep of twed.h, FP32) and returns the k best.  The
 * exact TWED decides the answer; the network only chooses what to measure.
 *
 * Network (fixed shape; series values only, timestamps are not an input):
 *   features   f_t = (x_t / 8, L / 256) for a series of L samples
 *   4 layers   kernel 5, same padding inside the series, channels
 *              2 -> 64 -> 64 -> 64 -> 4, ReLU after layers 1-3
 *   pooling    segment s = 0..31 covers t in [floor(s L/32), floor((s+1) L/32));
 *              embedding[4 s + c] = mean of layer-4 channel c over segment s
 *              (0 for an empty segment: series shorter than 32 samples)
 *   loss       for a pair (a, b) with TWED d: p = sqrt(|e_a - e_b|^2 + 1e-6),
 *              (log(1 + p) - log(1 + d))^2, averaged over the pairs
 * Arithmetic: BF16 operands on the matrix cores with FP32 accumulation, FP32
 * master weights, biases, pooling, loss and optimiser state.
 *
 * Parameters are one flat FP32 vector of twed_embed_param_count() elements:
 * for each layer, W with shape (5, C_in, C_out) row-major, then b (C_out).
 *
 * Conventions are those of twed.h: device arrays are caller-owned, scratch
 * comes from a 256-byte aligned caller workspace, work is enqueued on
 * `stream`, argument errors are returned before any HIP call.
 */
#ifndef TWED_KNN_H_
#define TWED_KNN_H_

#include "twed.h"

#ifdef __cplusplus
extern "C" {
#endif

#define TWED_EMBED_DIM 128

/* ---- embedding network ------------------------------------------------------ */

/* Number of FP32 parameters (43,076). */
int64_t twed_embed_param_count(void);

/* Longest series the network accepts (65,535 samples). */
int64_t twed_embed_max_length(void);

/* Memory bounds of the embedding forward pass and of twed_knn.  The forward
 * pass over a collection embeds whole series, at most chunk_rows samples at
 * a time (activation workspace about 0.3 KB per sample; a chunk always
 * holds at least the longest series); twed_knn scores at most
 * max(1, score_bytes / (4 nDB)) queries against the database at a time.
 * 0 or a negative value restores the default (2^22 samples, 2^30 bytes).
 * Process-wide; it changes the workspace sizes reported afterwards.  A call
 * whose workspace was sized under a smaller limit than the one in force
 * fails with TWED_ERR_WORKSPACE.  Results do not depend on the limits. */
void twed_embed_set_limits(int64_t chunk_rows, int64_t score_bytes);

/* Workspace bytes for twed_embed_forward (nPairs = 0) or
 * twed_embed_loss_grad (nPairs pairs) over the collection `off` (host,
 * nSeries+1 offsets).  0 if the offsets are invalid. */
size_t twed_embed_workspace_size(const int64_t *off, int64_t nSeries, int64_t nPairs);

/* Embeddings of nSeries packed 1-D series.
 * params: device, twed_embed_param_count() floats.
 * X: device, off[nSeries] floats (values; no timestamps).
 * off: HOST, nSeries+1 offsets, off[0] = 0, every length in [1, max_length].
 * emb: device, nSeries x 128 floats, row-major.
 * Errors: TWED_ERR_INVALID for null pointers or bad offsets,
 * TWED_ERR_UNSUPPORTED for a series longer than twed_embed_max_length(),
 * TWED_ERR_WORKSPACE for a short or misaligned workspace. */
twed_status twed_embed_forward(const float *params, const float *X, const int64_t *off, int64_t nSeries,
                               float *emb, void *workspace, size_t ws_bytes, hipStream_t stream);

/* Mean pair loss over nPairs pairs of the collection and its gradient.
 * pairs: device, nPairs (a, b) int32 pairs of series indices; a pair with
 *        an index outside [0, nSeries) contributes nothing.
 * target: device, nPairs TWED values (>= 0).
 * loss: device, one float (overwritten).  grad: device, param_count floats
 * (overwritten).  emb: optional device nSeries x 128 floats (embeddings of
 * the forward pass), may be NULL.  nPairs >= 1. */
twed_status twed_embed_loss_grad(const float *params, const float *X, const int64_t *off, int64_t nSeries,
                                 const int32_t *pairs, const float *target, int64_t nPairs, float *loss,
                                 float *grad, float *emb, void *workspace, size_t ws_bytes, hipStream_t stream);

/* One AdamW step (beta1 0.9, beta2 0.999, eps 1e-8, decoupled weight decay)
 * on the flat parameters: step is the 1-based step count used for the bias
 * corrections; m and v are the device moment vectors (zero before step 1). */
twed_status twed_embed_adamw(float *params, float *m, float *v, const float *grad, int64_t step, float lr,
                             float weight_decay, hipStream_t stream);

/* ---- k-NN index --------------------------------------------------------------- */

typedef struct twed_knn_index twed_knn_index;

/* Device bytes the index keeps for a database (`storage` below): the BF16
 * embeddings and their norms, device offsets and the database staged for
 * the batched sweep.  prm: dim must be 1 and precision TWED_F32. */
size_t twed_knn_index_storage_size(const int64_t *offDB, int64_t nDB, const twed_params *prm);

/* Creates an index over nDB packed 1-D FP32 series (DB values and TDB
 * timestamps: device; offDB: host, copied).  DB, TDB and params (device,
 * the trained network) are referenced, not copied: the caller keeps them
 * alive and unchanged until destroy.  storage: device, caller-owned,
 * twed_knn_index_storage_size() bytes, 256-byte aligned.  Host-only: no
 * device work until twed_knn_index_build.
 * Errors: TWED_ERR_INVALID (null pointers, bad offsets or params),
 * TWED_ERR_UNSUPPORTED (dim != 1, precision != TWED_F32, a series longer
 * than twed_embed_max_length(), more than 2^31 - 1 series). */
twed_status twed_knn_index_create(const void *DB, const void *TDB, const int64_t *offDB, int64_t nDB,
                                  const float *params, const twed_params *prm, void *storage,
                                  size_t storage_bytes, twed_knn_index **out);

size_t twed_knn_index_build_workspace_size(const twed_knn_index *index);

/* Embeds and stages the database into the index storage. */
twed_status twed_knn_index_build(twed_knn_index *index, void *workspace, size_t ws_bytes, hipStream_t stream);

/* Workspace bytes of twed_knn for these queries. */
size_t twed_knn_workspace_size(const twed_knn_index *index, const int64_t *offQ, int64_t nQ, int32_t k,
                               int32_t n_cand);

/* The k nearest database series of each of nQ queries (Q, TQ: device
 * packed FP32 values and timestamps; offQ: host offsets).
 * 1 <= k <= n_cand <= nDB.  Candidates: the n_cand smallest squared
 * embedding distances (ties to lower ids); then exact FP32 TWED of every
 * (query, candidate) pair; ids[q*k + r] / dist[q*k + r] (device, int64 /
 * float) are the r-th smallest (distance, id).  With n_cand = nDB the
 * answer is the exact k-NN.  When queries and database both hold series
 * longer than twed_batch_max_short_length(1), the candidate list is read
 * back to the host to sweep those pairs one by one (see twed_batch), and
 * the call synchronises `stream`.
 * Errors as twed_batch, plus TWED_ERR_INVALID for k or n_cand out of range
 * and an index that was not built. */
twed_status twed_knn(const twed_knn_index *index, const void *Q, const void *TQ, const int64_t *offQ, int64_t nQ,
                     int32_t k, int32_t n_cand, int64_t *ids, float *dist, void *workspace, size_t ws_bytes,
                     hipStream_t stream);

void twed_knn_index_destroy(twed_knn_index *index);

#ifdef __cplusplus
}
#endif
#endif /* TWED_KNN_H_ */

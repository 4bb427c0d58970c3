// capi_util.h -- host helpers shared by the extern "C" entry points:
// error reporting, workspace carving and argument checks.
#pragma once

#include "../../include/twed.h"
#include "twed_kernels.h"

#include <algorithm>
#include <cmath>
#include <stdint.h>
#include <string>

namespace twed {
namespace capi {

// Message of the last error on the calling thread (defined in twed_capi.hip).
std::string &last_error();

inline twed_status fail(twed_status s, const char *msg)
{
    last_error() = msg;
    return s;
}

// Runs the body of an entry point that allocates host memory (containers,
// messages): an allocation failure becomes TWED_ERR_DEVICE instead of an
// exception crossing the C ABI.
template <typename F>
inline twed_status no_throw(F &&body) noexcept
{
    try {
        return body();
    } catch (...) {
        try {
            last_error() = "host allocation failed";
        } catch (...) {
        }
        return TWED_ERR_DEVICE;
    }
}

inline twed_status fail_hip(hipError_t e, const char *where)
{
    last_error() = std::string(where) + ": " + hipGetErrorString(e);
    return TWED_ERR_DEVICE;
}

constexpr size_t kAlign = 256;
constexpr int64_t kMaxLen = (int64_t(1) << 31) - 2 * 64 - 2;

inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Sequential carve-out of a caller buffer; with base == nullptr it only
// counts bytes (the *_size() queries).
struct Carver {
    char *base;
    size_t used = 0;
    void *take(size_t bytes)
    {
        void *p = base ? base + used : nullptr;
        used += align_up(bytes);
        return p;
    }
};

// Packed rows with kRowPad zero rows before and kRowPadTail after; returns
// the row-0 pointer.
inline void *take_rows(Carver &c, Prec prec, int dimt, int64_t rows)
{
    char *p = (char *)c.take(rows_bytes(prec, dimt, rows));
    return p ? p + (size_t)kRowPad * (size_t)row_stride(prec, dimt) * cost_size(prec) : nullptr;
}

// Device bytes of the single-pair sweep state (boundary slots, then flags
// and tail words) for series of up to maxlen samples (twed_capi.hip).
size_t long_pair_state_bytes(Prec prec, int64_t maxlen);

// Pairs of a device pair list whose shorter series is too long for the
// batched kernel's single wave: reads the list back (synchronising `st`) and
// runs the single-pair sweep of each such pair into D[k] (accumulator type).
// rowsX / rowsY: staged rows; offX / offY: host offsets of nX / nY series;
// state: long_pair_state_bytes(prec, maxlen) bytes (twed_capi.hip).
twed_status sweep_long_listed_pairs(Prec prec, const CostParams &cp, const twed_params *prm, const void *rowsX,
                                    const int64_t *offX, int64_t nX, const void *rowsY, const int64_t *offY,
                                    int64_t nY, const int64_t *pairs, int64_t nPairs, void *state,
                                    int64_t maxlen, void *D, hipStream_t st);

inline bool finite_nonneg(double v) { return std::isfinite(v) && v >= 0.0; }

inline twed_status check_params(const twed_params *prm)
{
    if (!prm) return fail(TWED_ERR_INVALID, "params is NULL");
    if (!finite_nonneg(prm->nu)) return fail(TWED_ERR_INVALID, "nu must be finite and >= 0");
    if (!finite_nonneg(prm->lambda)) return fail(TWED_ERR_INVALID, "lambda must be finite and >= 0");
    if (!std::isfinite(prm->p) || prm->p < 1.0) return fail(TWED_ERR_INVALID, "p must be finite and >= 1");
    if (prm->dim < 1) return fail(TWED_ERR_INVALID, "dim must be >= 1");
    if (prm->dim > TWED_MAX_DIM) return fail(TWED_ERR_UNSUPPORTED, "dim exceeds TWED_MAX_DIM");
    if (prm->precision < TWED_F64 || prm->precision > TWED_AUTO)
        return fail(TWED_ERR_INVALID, "unknown precision");
    if (prm->algo < TWED_ALGO_AUTO || prm->algo > TWED_ALGO_DIAGONAL) return fail(TWED_ERR_INVALID, "unknown algo");
    if (!(prm->strip_k == 0 || prm->strip_k == 1 || prm->strip_k == 2 || prm->strip_k == 4 || prm->strip_k == 8))
        return fail(TWED_ERR_INVALID, "strip_k must be 0, 1, 2, 4 or 8");
    if (prm->dim > 16 && prm->strip_k > 2)
        return fail(TWED_ERR_UNSUPPORTED, "strip_k 4 and 8 are not available for dim > 16");
    return TWED_OK;
}

inline CostParams cost_params(const twed_params *prm)
{
    CostParams cp;
    cp.nu = prm->nu;
    cp.lambda = prm->lambda;
    cp.p = prm->p;
    cp.dim = prm->dim;
    cp.dimt = dimt_for(prm->dim);
    cp.pm = prm->dim == 1 ? 0 : (prm->p == 1.0 ? 0 : (prm->p == 2.0 ? 1 : 2));
    return cp;
}

inline twed_status check_workspace(const void *ws, size_t ws_bytes, size_t need)
{
    if (need > ws_bytes) return fail(TWED_ERR_WORKSPACE, "workspace smaller than the *_workspace_size() value");
    if (need == 0) return TWED_OK;
    if (!ws) return fail(TWED_ERR_WORKSPACE, "workspace is NULL");
    if (((uintptr_t)ws) % kAlign) return fail(TWED_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    return TWED_OK;
}

// Host CSR offsets: n >= 1 series, off[0] = 0, every length >= 1.
inline twed_status check_offsets(const int64_t *off, int64_t n, int64_t *maxlen, int64_t *total)
{
    if (!off) return fail(TWED_ERR_INVALID, "NULL offsets");
    if (n < 1) return fail(TWED_ERR_INVALID, "collection must hold at least one series");
    if (off[0] != 0) return fail(TWED_ERR_INVALID, "offsets must start at 0");
    int64_t mx = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t len = off[i + 1] - off[i];
        if (len < 1) return fail(TWED_ERR_INVALID, "every series must hold at least one sample");
        mx = std::max(mx, len);
    }
    if (mx > kMaxLen) return fail(TWED_ERR_UNSUPPORTED, "series longer than 2^31 - 130");
    *maxlen = mx;
    *total = off[n];
    return TWED_OK;
}

}  // namespace capi
}  // namespace twed

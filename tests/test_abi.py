"""The C ABI on the host: the library loads, exports every declared entry
point, and rejects bad arguments before any HIP call (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2007_16135_amd as tw
from paper_2007_16135_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("twed.h", "twed_knn.h")]

INVALID, UNSUPPORTED, WORKSPACE = binding.TWED_ERR_INVALID, binding.TWED_ERR_UNSUPPORTED, binding.TWED_ERR_WORKSPACE


@pytest.fixture(scope="module")
def L():
    return binding.load_library()


def declared_functions():
    src = "".join(open(h).read() for h in HEADERS)
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(twed_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert "twed_pair" in names and "twed_batch" in names
    for n in names:
        assert hasattr(L, n), f"{n} declared in include/ but not exported"
    assert set(binding.EXPORTS) <= set(names)


def test_params_struct_layout(L):
    # the binding's struct must match the header's field order and size
    prm = binding.TwedParams()
    L.twed_params_default(ctypes.byref(prm))
    assert ctypes.sizeof(prm) == 48
    assert prm.nu == 0.001 and prm.lambda_ == 1.0 and prm.p == 1.0 and prm.dim == 1
    assert prm.precision == 0 and prm.algo == 0 and prm.strip_k == 0


def test_status_strings(L):
    for s in range(5):
        assert L.twed_status_string(s)
    assert L.twed_version().startswith(b"libtwed")


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails validation


def _pair(L, prm, nA=10, nB=10, A=FAKE, TA=FAKE, B=FAKE, TB=FAKE, out=FAKE, ws=None, wsb=0):
    return L.twed_pair(A, TA, nA, B, TB, nB, ctypes.byref(prm) if prm is not None else None, out,
                       ws, wsb, None)


def test_pair_argument_errors(L):
    good = tw.make_params()
    assert _pair(L, None) == INVALID
    assert _pair(L, good, nA=0) == INVALID
    assert _pair(L, good, nB=-3) == INVALID
    assert _pair(L, good, A=None) == INVALID
    assert _pair(L, good, TB=None) == INVALID
    assert _pair(L, good, out=None) == INVALID
    for kw in [dict(nu=-1.0), dict(lam=-0.5), dict(p=0.5), dict(nu=float("nan")),
               dict(lam=float("inf")), dict(p=float("inf")), dict(dim=0)]:
        assert _pair(L, tw.make_params(**kw)) == INVALID, kw
    assert _pair(L, tw.make_params(dim=33)) == UNSUPPORTED
    assert _pair(L, tw.make_params(dim=20, strip_k=4)) == UNSUPPORTED
    assert _pair(L, tw.make_params(dim=32, strip_k=8)) == UNSUPPORTED
    # up to 32 components with strips of one or two columns: only the
    # missing workspace is reported
    for k in (0, 1, 2):
        assert _pair(L, tw.make_params(dim=28, strip_k=k)) == WORKSPACE
    assert _pair(L, tw.make_params(precision=7)) == INVALID
    assert _pair(L, tw.make_params(algo=5)) == INVALID
    assert _pair(L, tw.make_params(strip_k=3)) == INVALID
    assert _pair(L, good, nA=1 << 31) == UNSUPPORTED
    # valid arguments, no or short workspace
    assert _pair(L, good) == WORKSPACE
    need = L.twed_pair_workspace_size(10, 10, ctypes.byref(good))
    assert need > 0
    assert _pair(L, good, ws=FAKE, wsb=need - 1) == WORKSPACE
    assert _pair(L, good, ws=ctypes.c_void_p(0x1001), wsb=need) == WORKSPACE  # misaligned
    assert L.twed_last_error()


def test_pair_noalloc_host_checks(L):
    # argument errors as twed_pair; a pair whose workspace exceeds the fixed
    # scratch array is refused, with the sizes in the message, before any HIP
    # call
    good = tw.make_params()
    call = lambda prm, nA=10, nB=10, A=FAKE, out=FAKE: L.twed_pair_noalloc(
        A, FAKE, nA, FAKE, FAKE, nB, ctypes.byref(prm) if prm is not None else None, out, None)
    assert call(None) == INVALID
    assert call(good, nA=0) == INVALID
    assert call(good, A=None) == INVALID
    assert call(good, out=None) == INVALID
    assert call(tw.make_params(nu=-1.0)) == INVALID
    assert call(tw.make_params(dim=33)) == UNSUPPORTED
    limit = 64 << 20
    big = 1 << 21
    assert L.twed_pair_workspace_size(big, big, ctypes.byref(good)) > limit
    assert call(good, nA=big, nB=big) == UNSUPPORTED
    msg = L.twed_last_error().decode()
    assert "twed_pair_noalloc" in msg and str(limit) in msg


def test_pair_config_host_checks(L):
    """twed_pair_config validates its arguments before touching the device."""
    prm = binding.make_params(dim=8, precision="f32_acc64")
    k, g = ctypes.c_int32(-1), ctypes.c_int32(-1)
    w, n = ctypes.c_int64(-1), ctypes.c_int64(-1)
    outs = (ctypes.byref(k), ctypes.byref(g), ctypes.byref(w), ctypes.byref(n))
    assert L.twed_pair_config(0, 10, ctypes.byref(prm), *outs) == INVALID
    assert L.twed_pair_config(10, -1, ctypes.byref(prm), *outs) == INVALID
    assert L.twed_pair_config(10, 10, None, *outs) == INVALID
    assert L.twed_pair_config(1 << 31, 10, ctypes.byref(prm), *outs) == UNSUPPORTED
    bad = binding.make_params(p=0.5)
    assert L.twed_pair_config(10, 10, ctypes.byref(bad), *outs) == INVALID
    diag = binding.make_params(algo="diagonal")
    assert L.twed_pair_config(10, 10, ctypes.byref(diag), *outs) == INVALID
    assert (k.value, g.value, w.value, n.value) == (-1, -1, -1, -1)  # nothing written on error


def test_pair_matrix_needs_dp(L):
    good = tw.make_params()
    assert L.twed_pair_matrix(FAKE, FAKE, 4, FAKE, FAKE, 4, ctypes.byref(good), FAKE, None, None, 0,
                              None) == INVALID


def test_workspace_sizes(L):
    for prec in ("f64", "f32", "f32_acc64"):
        prm = tw.make_params(dim=3, precision=prec)
        s1 = L.twed_pair_workspace_size(1000, 1000, ctypes.byref(prm))
        s2 = L.twed_pair_workspace_size(100000, 100000, ctypes.byref(prm))
        assert 0 < s1 < s2
        # linear memory: O(nA + nB), not O(nA * nB)
        assert s2 < 100 * s1 * 1.5
    bad = tw.make_params(nu=-1)
    assert L.twed_pair_workspace_size(10, 10, ctypes.byref(bad)) == 0
    assert L.twed_pair_workspace_size(0, 10, ctypes.byref(tw.make_params())) == 0
    # the wavefront state for n = 1e6 (8-D, FP32 costs, FP64 accumulators)
    # stays within a few hundred MB
    prm = tw.make_params(dim=8, p=2, precision="f32_acc64")
    assert L.twed_pair_workspace_size(10**6, 10**6, ctypes.byref(prm)) < 200 * 2**20


def _batch(L, prm, offX, nX=None, offY=None, nY=None, X=FAKE, TX=FAKE, Y=None, TY=None, pairs=None, nP=0,
           D=FAKE, ws=None, wsb=0):
    ox = np.ascontiguousarray(offX, dtype=np.int64) if offX is not None else None
    oy = np.ascontiguousarray(offY, dtype=np.int64) if offY is not None else None
    px = ox.ctypes.data_as(binding._i64p) if ox is not None else None
    py = oy.ctypes.data_as(binding._i64p) if oy is not None else None
    if nX is None:
        nX = len(ox) - 1
    if nY is None:
        nY = nX if oy is None else len(oy) - 1
    return L.twed_batch(X, TX, px, nX, Y, TY, py, nY, pairs, nP, ctypes.byref(prm), D, ws, wsb, None)


def test_batch_argument_errors(L):
    prm = tw.make_params(precision="f32")
    assert _batch(L, prm, [0, 3, 5]) == WORKSPACE           # valid, no workspace
    assert _batch(L, prm, [1, 3, 5]) == INVALID             # must start at 0
    assert _batch(L, prm, [0, 3, 3]) == INVALID             # empty series
    assert _batch(L, prm, [0, 3, 2]) == INVALID             # decreasing
    assert _batch(L, prm, None, nX=2) == INVALID
    assert _batch(L, prm, [0, 3, 5], X=None) == INVALID
    assert _batch(L, prm, [0, 3, 5], D=None) == INVALID
    assert _batch(L, prm, [0, 3, 5], nY=3) == INVALID       # symmetric needs nY == nX
    assert _batch(L, prm, [0, 3, 5], nY=2, TY=FAKE) == INVALID
    assert _batch(L, prm, [0, 3, 5], offY=[0, 2], nY=1, Y=FAKE, TY=None) == INVALID
    assert _batch(L, prm, [0, 3, 5], offY=[0, 2], nY=1, Y=FAKE, TY=FAKE, pairs=FAKE, nP=-1) == INVALID
    # pair list with both collections holding over-long series: accepted
    # (such pairs run the single-pair sweep); here only the workspace is missing
    longs = [0, 5000, 10000]
    assert _batch(L, prm, longs, offY=longs, nY=2, Y=FAKE, TY=FAKE, pairs=FAKE, nP=1) == WORKSPACE
    need = L.twed_batch_workspace_size(np.array([0, 3, 5], np.int64).ctypes.data_as(binding._i64p), 2,
                                       None, 0, ctypes.byref(prm))
    assert need > 0
    assert _batch(L, prm, [0, 3, 5], ws=FAKE, wsb=need - 1) == WORKSPACE


def test_batch_max_short_length(L):
    assert L.twed_batch_max_short_length(1) == 1024
    assert L.twed_batch_max_short_length(3) == 512
    assert L.twed_batch_max_short_length(8) == 256


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(RuntimeError, match="not built"):
        binding.load_library(str(tmp_path / "nope.so"))


def test_embed_limits_bound_the_workspace(L):
    import ctypes as C
    off = np.arange(0, 1_000_001, 500, dtype=np.int64)  # 2000 series of 500 samples
    po = off.ctypes.data_as(C.POINTER(C.c_int64))
    try:
        full = L.twed_embed_workspace_size(po, 2000, 0)
        L.twed_embed_set_limits(10_000, 0)
        small = L.twed_embed_workspace_size(po, 2000, 0)
        L.twed_embed_set_limits(100, 0)  # below the longest series: one series per chunk
        tiny = L.twed_embed_workspace_size(po, 2000, 0)
        # activations are about 0.3 KB per sample of the chunk
        assert full - small > 250 * (1_000_000 - 10_000)
        assert small - tiny > 250 * (10_000 - 500)
        assert tiny > 0
    finally:
        L.twed_embed_set_limits(0, 0)
    assert L.twed_embed_workspace_size(po, 2000, 0) == full


def test_embed_and_knn_host_checks(L):
    import ctypes as C
    from oracle import cnn as ocnn
    assert L.twed_embed_param_count() == ocnn.n_params()
    assert L.twed_embed_max_length() == 65535
    off = np.array([0, 5, 9], dtype=np.int64)
    po = off.ctypes.data_as(C.POINTER(C.c_int64))
    assert L.twed_embed_workspace_size(po, 2, 0) > 0
    assert L.twed_embed_workspace_size(po, 2, 10) > L.twed_embed_workspace_size(po, 2, 0)
    bad = np.array([1, 5, 9], dtype=np.int64)
    assert L.twed_embed_workspace_size(bad.ctypes.data_as(C.POINTER(C.c_int64)), 2, 0) == 0
    long_ = np.array([0, 70000], dtype=np.int64)
    assert L.twed_embed_workspace_size(long_.ctypes.data_as(C.POINTER(C.c_int64)), 1, 0) == 0
    fake = C.c_void_p(0x100000)
    assert L.twed_embed_forward(None, fake, po, 2, fake, fake, 1 << 30, None) == INVALID
    assert L.twed_embed_loss_grad(fake, fake, po, 2, fake, fake, 0, fake, fake, None, fake, 1 << 30,
                                  None) == INVALID
    assert L.twed_embed_adamw(fake, fake, fake, fake, 0, 1e-3, 0.0, None) == INVALID
    assert L.twed_embed_adamw(fake, fake, fake, fake, 1, -1.0, 0.0, None) == INVALID
    ws = C.c_size_t(L.twed_embed_workspace_size(po, 2, 0))
    assert L.twed_embed_forward(fake, fake, po, 2, fake, None, ws, None) == WORKSPACE
    assert L.twed_embed_forward(fake, fake, po, 2, fake, C.c_void_p(0x100010), ws, None) == WORKSPACE

    prm = binding.make_params(1e-3, 1.0, 1.0, 1, "f32")
    need = L.twed_knn_index_storage_size(po, 2, C.byref(prm))
    assert need > 0
    for bad_prm in (binding.make_params(1e-3, 1.0, 1.0, 2, "f32"), binding.make_params(1e-3, 1.0, 1.0, 1, "f64")):
        assert L.twed_knn_index_storage_size(po, 2, C.byref(bad_prm)) == 0
        h = C.c_void_p()
        assert L.twed_knn_index_create(fake, fake, po, 2, fake, C.byref(bad_prm), fake, need,
                                       C.byref(h)) == UNSUPPORTED
    h = C.c_void_p()
    assert L.twed_knn_index_create(None, fake, po, 2, fake, C.byref(prm), fake, need, C.byref(h)) == INVALID
    assert L.twed_knn_index_create(fake, fake, po, 2, fake, C.byref(prm), fake, need - 1, C.byref(h)) == WORKSPACE
    # host-only creation with placeholder device addresses: nothing touches the device
    assert L.twed_knn_index_create(fake, fake, po, 2, fake, C.byref(prm), fake, need, C.byref(h)) == 0
    assert h.value
    assert L.twed_knn_index_build_workspace_size(h) > 0
    offq = np.array([0, 4], dtype=np.int64)
    pq = offq.ctypes.data_as(C.POINTER(C.c_int64))
    assert L.twed_knn_workspace_size(h, pq, 1, 1, 2) > 0
    assert L.twed_knn_workspace_size(h, pq, 1, 3, 2) == 0  # k > n_cand
    assert L.twed_knn_workspace_size(h, pq, 1, 1, 3) == 0  # n_cand > nDB
    ids = C.c_void_p(0x200000)
    assert L.twed_knn(h, fake, fake, pq, 1, 1, 2, ids, ids, fake, 1 << 30, None) == INVALID  # not built
    assert L.twed_knn(None, fake, fake, pq, 1, 1, 2, ids, ids, fake, 1 << 30, None) == INVALID
    L.twed_knn_index_destroy(h)


def test_tune_host_checks(L):
    import ctypes as C
    prm = binding.make_params(1e-3, 1.0, 1.0, 1, "f64")
    fake = C.c_void_p(0x100000)
    k, g = C.c_int32(0), C.c_int32(0)
    assert L.twed_pair_tune(None, fake, 10, fake, fake, 10, C.byref(prm), fake, 1 << 30, None,
                            C.byref(k), C.byref(g)) == INVALID
    assert L.twed_pair_tune(fake, fake, 0, fake, fake, 10, C.byref(prm), fake, 1 << 30, None,
                            C.byref(k), C.byref(g)) == INVALID
    diag = binding.make_params(1e-3, 1.0, 1.0, 1, "f64", algo="diagonal")
    assert L.twed_pair_tune(fake, fake, 10, fake, fake, 10, C.byref(diag), fake, 1 << 30, None,
                            C.byref(k), C.byref(g)) == INVALID
    assert L.twed_pair_tune(fake, fake, 10, fake, fake, 10, C.byref(prm), None, 0, None,
                            C.byref(k), C.byref(g)) == WORKSPACE
    L.twed_tune_clear()


def test_tile_and_path_host_checks(L):
    c = ctypes
    prm = tw.make_params(dim=2)
    ws_need = L.twed_pair_tile_workspace_size(10, 10, c.byref(prm))
    assert ws_need > 0
    assert L.twed_pair_tile_workspace_size(0, 10, c.byref(prm)) == 0
    assert L.twed_pair_tile_workspace_size(10, 10, c.byref(tw.make_params(precision="f32"))) == 0

    def tile(r0, r1, c0, c1, top=None, left=None, p=prm, ws=None, wsb=0):
        return L.twed_pair_tile(FAKE, FAKE, 20, FAKE, FAKE, 20, c.byref(p), r0, r1, c0, c1, top, left, None, None,
                                None, ws, wsb, None)

    assert tile(5, 5, 0, 10) == INVALID          # empty block
    assert tile(0, 21, 0, 10) == INVALID         # past nA
    assert tile(3, 10, 0, 10) == INVALID         # top row missing
    assert tile(0, 10, 4, 10) == INVALID         # left column missing
    assert tile(0, 10, 0, 10, p=tw.make_params(dim=2, precision="f32")) == UNSUPPORTED
    assert tile(0, 10, 0, 10) == WORKSPACE
    assert L.twed_pair_tile(None, FAKE, 20, FAKE, FAKE, 20, c.byref(prm), 0, 1, 0, 1, None, None, None, None, None,
                            None, 0, None) == INVALID
    need = L.twed_pair_path_workspace_size(100, 90, c.byref(prm), 0)
    assert need > 0
    assert L.twed_pair_path_workspace_size(100, 90, c.byref(prm), -1) == 0
    # blocks of 64: checkpoints every 64 rows and every 64 columns (78 each)
    assert L.twed_pair_path_workspace_size(5000, 5000, c.byref(prm), 64) >= 2 * 78 * 5001 * 16

    def path(block=0, out=FAKE, pth=FAKE, n=FAKE, p=prm, wsb=0):
        return L.twed_pair_path(FAKE, FAKE, 100, FAKE, FAKE, 90, c.byref(p), block, out, pth, n, None, wsb, None)

    assert path(block=-1) == INVALID
    assert path(out=None) == INVALID
    assert path(pth=None) == INVALID
    assert path(p=tw.make_params(dim=2, precision="f32")) == UNSUPPORTED
    assert path() == WORKSPACE


def test_dp_host_checks(L):
    c = ctypes
    prm1 = tw.make_params(dim=1)
    assert L.twed_dp_workspace_size(2, 100, 90, c.byref(prm1)) > 0
    assert L.twed_dp_workspace_size(9, 100, 90, c.byref(prm1)) == 0          # unknown kind
    assert L.twed_dp_workspace_size(2, 100, 90, c.byref(tw.make_params(dim=3))) == 0   # edit needs dim 1
    assert L.twed_dp_workspace_size(1, 100, 90, c.byref(tw.make_params(dim=3))) > 0    # DTW in 3-D

    def dp(kind, p=prm1, A=FAKE, out=FAKE, n=10):
        return L.twed_dp(kind, A, n, FAKE, n, c.byref(p), out, None, 0, None)

    assert dp(0) == INVALID
    assert dp(2, A=None) == INVALID
    assert dp(2, out=None) == INVALID
    assert dp(2, n=0) == INVALID
    assert dp(3, p=tw.make_params(dim=2)) == UNSUPPORTED
    assert dp(1, p=tw.make_params(precision="f32")) == UNSUPPORTED
    assert dp(1, p=tw.make_params(strip_k=4)) == UNSUPPORTED
    assert dp(1) == WORKSPACE
    assert L.twed_dp_path(2, FAKE, 10, FAKE, 10, c.byref(prm1), -1, FAKE, FAKE, FAKE, None, 0, None) == INVALID
    assert L.twed_dp_path(2, FAKE, 10, FAKE, 10, c.byref(prm1), 0, FAKE, None, FAKE, None, 0, None) == INVALID


def test_batch_plan_host_checks(L):
    c = ctypes
    prm = tw.make_params(dim=1)
    off = np.array([0, 5, 9], np.int64)
    bad = np.array([0, 5, 5], np.int64)
    po = off.ctypes.data_as(c.POINTER(c.c_int64))
    pb = bad.ctypes.data_as(c.POINTER(c.c_int64))
    h = c.c_void_p()
    assert L.twed_batch_plan_create(po, 2, None, 0, 0, c.byref(prm), None, 0, None) == INVALID   # no out
    assert L.twed_batch_plan_create(po, 2, None, 0, 0, None, None, 0, c.byref(h)) == INVALID     # no params
    assert L.twed_batch_plan_create(pb, 2, None, 0, 0, c.byref(prm), None, 0, c.byref(h)) == INVALID  # empty series
    assert L.twed_batch_plan_create(po, 2, None, 0, -1, c.byref(prm), None, 0, c.byref(h)) == INVALID
    assert L.twed_batch_plan_create(po, 2, None, 0, 0, c.byref(prm), None, 0, c.byref(h)) == WORKSPACE
    assert not h.value
    assert L.twed_batch_plan_run(None, FAKE, FAKE, None, None, None, FAKE, None) == INVALID
    assert L.twed_batch_plan_stage_y(None, FAKE, FAKE, None) == INVALID
    L.twed_batch_plan_destroy(None)


def test_tune_cache_file_round_trip(L, tmp_path):
    # the tuning cache file: entries written by hand load, save back the
    # same, and a malformed file is refused without changing the cache
    L.twed_tune_clear()
    src = tmp_path / "in.txt"
    lines = ["libtwed-tune 1",
             "pair gfx950-cu256 2 8 1 1000000 8 8 4",
             "batch gfx950-cu256 1 1 0 0 9 9 21 8 16 -1"]
    src.write_text("\n".join(lines) + "\n")
    assert L.twed_tune_load(bytes(str(src), "utf-8")) == 0
    out = tmp_path / "out.txt"
    assert L.twed_tune_save(bytes(str(out), "utf-8")) == 0
    assert out.read_text().splitlines() == lines
    bad = tmp_path / "bad.txt"
    bad.write_text("libtwed-tune 1\npair gfx950-cu256 2 8 1 1000000 3 8 4\n")  # K = 3 is not a strip width
    assert L.twed_tune_load(bytes(str(bad), "utf-8")) == INVALID
    assert L.twed_tune_load(bytes(str(tmp_path / "missing.txt"), "utf-8")) == INVALID
    out2 = tmp_path / "out2.txt"
    assert L.twed_tune_save(bytes(str(out2), "utf-8")) == 0
    assert out2.read_text().splitlines() == lines
    L.twed_tune_clear()
    assert L.twed_tune_save(bytes(str(out2), "utf-8")) == 0
    assert out2.read_text().splitlines() == ["libtwed-tune 1"]

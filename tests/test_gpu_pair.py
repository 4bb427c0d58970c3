"""Single-pair parity: the HIP sweeps against the CPU oracle (GPU only).

Bars (from the arithmetic): FP64 within 1e-12 relative of the oracle (the
sweep re-associates the match cost as (DP + e_prev) + e_cur, and the oracle
uses DP + ((d1 + d2) + nu*(t1 + t2))); integer-valued worked examples
bitwise; FP32 within 1e-5 relative of the FP64 oracle run on the same
FP32-rounded inputs; FP32 costs with FP64 accumulators within 1e-6.
"""
import json
import os
import sys

import numpy as np
import pytest

import oracle
import oracle_pins as pins
from paper_2007_16135_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2007_16135_amd as tw  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
RTOL = {"f64": 1e-12, "f32": 1e-5, "f32_acc64": 1e-6}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(x, dt):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device="cuda")


def dtype_of(precision):
    return torch.float64 if precision == "f64" else torch.float32


class Unavailable(Exception):
    pass


def _call(fn, *a, **kw):
    try:
        return fn(*a, **kw)
    except tw.TwedError as e:
        if e.status == 2 and "switched off" in str(e):
            raise Unavailable(str(e))
        raise


def gpu_twed(A, TA, B, TB, nu, lam, p, precision="f64", **kw):
    dt = dtype_of(precision)
    A = np.asarray(A, dtype=np.float64).reshape(len(TA), -1)
    B = np.asarray(B, dtype=np.float64).reshape(len(TB), -1)
    out = _call(tw.twed_pair, dev(A, dt), dev(TA, dt), dev(B, dt), dev(TB, dt), nu, lam, p, precision, **kw)
    torch.cuda.synchronize()
    return float(out.item())


def gpu_matrix(A, TA, B, TB, nu, lam, p, precision="f64", **kw):
    dt = dtype_of(precision)
    A = np.asarray(A, dtype=np.float64).reshape(len(TA), -1)
    B = np.asarray(B, dtype=np.float64).reshape(len(TB), -1)
    out, dp = _call(tw.twed_pair_matrix, dev(A, dt), dev(TA, dt), dev(B, dt), dev(TB, dt), nu, lam, p,
                    precision, **kw)
    torch.cuda.synchronize()
    return float(out.item()), dp.cpu().numpy().astype(np.float64)


def _switched_off(cfg):
    """True if the library refuses this sweep before any launch (argument-level
    check with a deliberately missing workspace: no device work happens)."""
    import ctypes
    prm = tw.make_params(precision="f64", algo=cfg["algo"], strip_k=cfg.get("strip_k", 0))
    L = tw.load_library()
    fake = ctypes.c_void_p(256)
    st = L.twed_pair(fake, fake, 1, fake, fake, 1, ctypes.byref(prm), fake, None, 0, None)
    return st == 2 and b"switched off" in L.twed_last_error()


def rounded(x, precision):
    x = np.asarray(x, dtype=np.float64)
    return x.astype(np.float32).astype(np.float64) if precision != "f64" else x


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


ALL_ALGOS = [dict(algo="wavefront", strip_k=k) for k in (1, 2, 4, 8)] + [dict(algo="diagonal")]
ALGOS = [c for c in ALL_ALGOS if not _switched_off(c)]
OFF = [c for c in ALL_ALGOS if c not in ALGOS]
FAST = [c for c in ALGOS if c["algo"] != "diagonal"] or ALGOS  # sweep used for the long cases


def test_report_switched_off_sweeps():
    if OFF:
        pytest.skip(f"sweeps switched off in the library: {OFF}")


@pytest.mark.parametrize("cfg", ALL_ALGOS, ids=lambda c: f"{c['algo']}{c.get('strip_k', '')}")
def test_worked_examples_bitwise(cfg):
    if cfg in OFF:
        pytest.skip("sweep switched off in this build")
    for c in pins.load_worked_examples():
        A = np.array(c["A"], float).reshape(-1, c["dim"])
        B = np.array(c["B"], float).reshape(-1, c["dim"])
        say(f"worked example {c['name']} {cfg}")
        if c["exact"] and cfg.get("strip_k", 1) <= 2:
            v, dp = gpu_matrix(A, c["TA"], B, c["TB"], c["nu"], c["lambda"], c["p"], **cfg)
            want = np.array([[np.inf if x == "inf" else x for x in row] for row in c["DP"]], float)
            assert np.array_equal(dp, want), (dp, want)
            assert v == c["twed"]
        elif c["exact"]:
            # cell dumps are for narrow strips; wider ones are checked on the value
            v = gpu_twed(A, c["TA"], B, c["TB"], c["nu"], c["lambda"], c["p"], **cfg)
            assert v == c["twed"]
        else:
            v = gpu_twed(A, c["TA"], B, c["TB"], c["nu"], c["lambda"], c["p"], **cfg)
            assert rel(v, c["twed"]) <= 1e-14


SHAPES = [(1, 1), (1, 7), (7, 1), (2, 3), (5, 9), (9, 5), (63, 64), (64, 63), (65, 65), (1, 700),
          (700, 1), (127, 129), (129, 127), (200, 513), (513, 200), (1023, 1025), (1025, 1023),
          (3000, 40), (40, 3000)]


@pytest.mark.parametrize("precision", ["f64", "f32", "f32_acc64"])
def test_random_shapes_vs_oracle(precision):
    rng = np.random.default_rng(2024)
    orc = oracle.get()
    for k, (nA, nB) in enumerate(SHAPES):
        dim = [1, 2, 3, 5, 8][k % 5]
        p = [1.0, 2.0, 3.0][k % 3] if dim > 1 else 1.0
        nu = [0.0, 1e-3, 0.5][k % 3]
        lam = [0.0, 1.0, 5.0][(k // 3) % 3]
        A, TA = pins.rand_series(rng, nA, dim)
        B, TB = pins.rand_series(rng, nB, dim)
        A, TA, B, TB = (rounded(x, precision) for x in (A, TA, B, TB))
        want = orc.twed(A, TA, B, TB, nu, lam, p)
        for cfg in ALGOS:
            if cfg["algo"] == "diagonal" and nA + nB > 2000:
                continue
            say(f"shape {nA}x{nB} dim{dim} p{p} nu{nu} lam{lam} {precision} {cfg}")
            got = gpu_twed(A, TA, B, TB, nu, lam, p, precision, **cfg)
            assert rel(got, want) <= RTOL[precision], (nA, nB, dim, p, cfg, got, want)


def test_band_dump_matches_oracle_matrix():
    """Every DP cell (row 0, column 0 and the interior), several strips wide."""
    rng = np.random.default_rng(7)
    orc = oracle.get()
    for (nA, nB, dim, p) in [(10, 12, 1, 1.0), (64, 64, 2, 2.0), (33, 200, 3, 2.0), (150, 70, 2, 1.0),
                             (5, 300, 1, 1.0)]:
        A, TA = pins.rand_series(rng, nA, dim)
        B, TB = pins.rand_series(rng, nB, dim)
        _, want = orc.twed(A, TA, B, TB, 0.3, 0.7, p, matrix=True)
        for cfg in [c for c in ALGOS if c.get("strip_k", 1) <= 2]:
            say(f"dump {nA}x{nB} dim{dim} {cfg}")
            _, got = gpu_matrix(A, TA, B, TB, 0.3, 0.7, p, **cfg)
            assert np.array_equal(np.isinf(got), np.isinf(want))
            fin = np.isfinite(want)
            err = np.max(np.abs(got[fin] - want[fin]) / np.maximum(np.abs(want[fin]), 1e-300))
            assert err <= 1e-12, err


def test_schedule_invariance_bitwise():
    """Strip width and algorithm change only the evaluation order across
    cells, never a cell's own arithmetic: FP64 results agree to the bit."""
    for n, prec in ((3000, "f64"), (3000, "f32"), (5000, "f32")):
        c = synth.single_pair_3d(n)
        vals = []
        for cfg in ALGOS:
            say(f"invariance n{n} {prec} {cfg}")
            vals.append(gpu_twed(c.A, c.TA, c.B, c.TB, c.nu, c.lam, c.p, prec, **cfg))
        assert len(set(vals)) == 1, (n, prec, vals)


@pytest.mark.parametrize("nA,nB", [(2500, 1700), (6000, 4500)])
def test_symmetry_bitwise(nA, nB):
    """D(A,B) == D(B,A) to the bit; the second shape is long enough for the
    FP32 cost offset, which is symmetric in (A, B) too."""
    c = synth.random_pair(31, 32, nA, nB, 2, irregular=True, nu=0.05, lam=0.4, p=2.0)
    for prec in ("f64", "f32", "f32_acc64"):
        say(f"symmetry {nA}x{nB} {prec}")
        ab = gpu_twed(c.A, c.TA, c.B, c.TB, c.nu, c.lam, c.p, prec)
        ba = gpu_twed(c.B, c.TB, c.A, c.TA, c.nu, c.lam, c.p, prec)
        assert ab == ba


def test_tiny_values_fp64():
    """FP64 squared distances near 2^-800 take the square root's unscaled
    path: the pair scaled by 2^-400 (values, times and lambda; homogeneity
    keeps the exact result at 2^-400 times the unscaled one) against the
    oracle on the same scaled inputs, and against 2^-400 times the GPU's
    unscaled result."""
    c = synth.random_pair(61, 62, 700, 900, 3, irregular=True, nu=0.02, lam=0.6, p=2.0)
    s = 2.0 ** -400
    want = oracle.twed(c.A * s, c.TA * s, c.B * s, c.TB * s, c.nu, c.lam * s, c.p)
    got = gpu_twed(c.A * s, c.TA * s, c.B * s, c.TB * s, c.nu, c.lam * s, c.p, "f64")
    assert abs(got - want) <= 1e-12 * abs(want), (got, want)
    base = gpu_twed(c.A, c.TA, c.B, c.TB, c.nu, c.lam, c.p, "f64")
    assert abs(got - base * s) <= 1e-12 * abs(base * s), (got, base * s)


def test_identity_is_zero():
    c = synth.single_pair_3d(5000)
    for prec in ("f64", "f32", "f32_acc64"):
        say(f"identity {prec}")
        assert gpu_twed(c.A, c.TA, c.A, c.TA, c.nu, c.lam, c.p, prec) == 0.0


def _golden():
    with open(os.path.join(GOLDEN, "oracle_values.json")) as f:
        return {c["name"]: c for c in json.load(f)["cases"]}


def test_walk1d_n1000():
    g = _golden()
    c = synth.single_pair_1d(1000)
    for prec, key in (("f64", "walk1d_n1000"), ("f32", "walk1d_n1000_f32"), ("f32_acc64", "walk1d_n1000_f32")):
        for cfg in ALGOS:
            say(f"walk1d n1000 {prec} {cfg}")
            got = gpu_twed(c.A, c.TA, c.B, c.TB, c.nu, c.lam, c.p, prec, **cfg)
            assert rel(got, g[key]["value"]) <= RTOL[prec], (prec, cfg, got)


def test_walk3d_n100000_full():
    """3-D walks, n = 100,000, irregular times: the full-size pair."""
    g = _golden()
    c = synth.single_pair_3d(100000)
    say("walk3d n1e5 f64")
    got = gpu_twed(c.A, c.TA, c.B, c.TB, c.nu, c.lam, c.p, "f64")
    assert rel(got, g["walk3d_n100000"]["value"]) <= 1e-12
    want32 = g["walk3d_n100000_f32"]["value"]
    say("walk3d n1e5 f32_acc64")
    got = gpu_twed(c.A, c.TA, c.B, c.TB, c.nu, c.lam, c.p, "f32_acc64")
    assert rel(got, want32) <= 1e-6
    say("walk3d n1e5 f32")
    got32 = gpu_twed(c.A, c.TA, c.B, c.TB, c.nu, c.lam, c.p, "f32")
    say(f"walk3d n1e5 f32 relative error {rel(got32, want32):.3e}")
    assert rel(got32, want32) <= 1e-5


def test_walk3d_prefix():
    g = _golden()
    c = synth.single_pair_3d(100000).prefix(10000)
    for prec, key in (("f64", "walk3d_n100000_prefix10000"), ("f32", "walk3d_n100000_prefix10000_f32"),
                      ("f32_acc64", "walk3d_n100000_prefix10000_f32")):
        say(f"walk3d prefix {prec}")
        got = gpu_twed(c.A, c.TA, c.B, c.TB, c.nu, c.lam, c.p, prec)
        assert rel(got, g[key]["value"]) <= RTOL[prec]


def test_walk8d_prefix():
    g = _golden()
    full = synth.single_pair_8d(1000000)
    for n, key, prec in ((10000, "walk8d_n1000000_prefix10000_f32", "f32_acc64"),
                         (10000, "walk8d_n1000000_prefix10000", "f64"),
                         (20000, "walk8d_n1000000_prefix20000_f32", "f32_acc64")):
        c = full.prefix(n)
        say(f"walk8d prefix {n} {prec}")
        got = gpu_twed(c.A, c.TA, c.B, c.TB, c.nu, c.lam, c.p, prec)
        assert rel(got, g[key]["value"]) <= RTOL[prec]


def test_auto_precision_policy():
    """AUTO: FP32 accumulators up to the threshold, FP64 beyond; f64 result."""
    c = synth.single_pair_3d(4000).astype(np.float32)
    f32 = gpu_twed(c.A, c.TA, c.B, c.TB, c.nu, c.lam, c.p, "f32")
    acc = gpu_twed(c.A, c.TA, c.B, c.TB, c.nu, c.lam, c.p, "f32_acc64")
    lo = gpu_twed(c.A, c.TA, c.B, c.TB, c.nu, c.lam, c.p, "auto", acc64_threshold=4000)
    hi = gpu_twed(c.A, c.TA, c.B, c.TB, c.nu, c.lam, c.p, "auto", acc64_threshold=3999)
    assert lo == f32 and hi == acc


@pytest.mark.parametrize("prec", ["f64", "f32", "f32_acc64"])
def test_strip_groups_bitwise(prec, monkeypatch):
    """Workgroups of 1, 4 or 8 strips hand boundaries over through global
    memory or LDS; the cells and their arithmetic are the same, so results
    agree to the bit with each other and with the per-diagonal sweep.  The
    shape gives 13 strips at K=1 (groups 8+5, or 4+4+4+1), 7 at K=2 and 4 at
    K=4, so full, partial and single-strip groups all occur."""
    c = synth.random_pair(41, 42, 1400, 64 * 13 - 5, 3, irregular=True, nu=0.02, lam=0.6, p=2.0)
    ref = gpu_twed(c.A, c.TA, c.B, c.TB, c.nu, c.lam, c.p, prec, algo="diagonal")
    for k in (1, 2, 4):
        for g in ("1", "4", "8"):
            monkeypatch.setenv("TWED_WAVEFRONT_GROUP", g)
            say(f"groups {prec} K={k} G={g}")
            v = gpu_twed(c.A, c.TA, c.B, c.TB, c.nu, c.lam, c.p, prec, algo="wavefront", strip_k=k)
            assert v == ref, (prec, k, g, v, ref)


@pytest.mark.parametrize("sub", ["8", "32"])
def test_handoff_intervals_bitwise(sub, monkeypatch):
    """In-group hand-over every 8 or 32 rows (TWED_WAVEFRONT_SUB), which also
    moves where groups of several strips fetch the next global window ahead
    (the window's second-to-last and last sub-chunks; with 32-row sub-chunks
    only a tile's given left column is fetched ahead): every strip width and
    group size agrees to the bit with the per-diagonal sweep."""
    c = synth.random_pair(43, 44, 1400, 64 * 13 - 5, 3, irregular=True, nu=0.02, lam=0.6, p=2.0)
    ref = gpu_twed(c.A, c.TA, c.B, c.TB, c.nu, c.lam, c.p, "f64", algo="diagonal")
    monkeypatch.setenv("TWED_WAVEFRONT_SUB", sub)
    for k in (1, 2, 4):
        for g in ("1", "4", "8"):
            monkeypatch.setenv("TWED_WAVEFRONT_GROUP", g)
            say(f"hand-over every {sub} rows K={k} G={g}")
            v = gpu_twed(c.A, c.TA, c.B, c.TB, c.nu, c.lam, c.p, "f64", algo="wavefront", strip_k=k)
            assert v == ref, (sub, k, g, v, ref)


def test_strip_groups_long_pair_vs_oracle(monkeypatch):
    """A pair long enough for many LDS sub-chunks and global windows, in
    groups of 8, against the FP64 oracle (FP32 costs with FP64 accumulators)."""
    c = synth.single_pair_8d(20000).astype(np.float32).astype(np.float64)
    ref = oracle.twed(c.A, c.TA, c.B, c.TB, c.nu, c.lam, c.p, rows=True)
    monkeypatch.setenv("TWED_WAVEFRONT_GROUP", "8")
    for k in (1, 2):
        say(f"groups long K={k}")
        v = gpu_twed(c.A, c.TA, c.B, c.TB, c.nu, c.lam, c.p, "f32_acc64", strip_k=k)
        assert abs(v - ref) <= 1e-6 * abs(ref), (k, v, ref)


@pytest.mark.parametrize("prec", ["f64", "f32", "f32_acc64"])
def test_two_strip_widths_bitwise(prec, monkeypatch):
    """Strips of two widths (8 then 7 columns per lane in groups of eight;
    TWED_WAVEFRONT_MIXED = number of wide strips) cover the same cells with
    the same arithmetic as uniform strips: results agree to the bit for every
    split, including splits inside a group and a last strip holding only a
    few columns; FP64 also against the oracle."""
    monkeypatch.setenv("TWED_WAVEFRONT_GROUP", "8")
    layout, wide = 0, 8
    for nA, nB in ((1500, 64 * wide * 11 - 3), (900, 64 * wide * 17 + 5)):
        c = synth.random_pair(51, 52, nA, nB, 3, irregular=True, nu=0.02, lam=0.6, p=2.0)
        monkeypatch.setenv("TWED_WAVEFRONT_MIXED", "0")
        ref = gpu_twed(c.A, c.TA, c.B, c.TB, c.nu, c.lam, c.p, prec, algo="wavefront", strip_k=8)
        if prec == "f64":
            want = oracle.twed(c.A, c.TA, c.B, c.TB, c.nu, c.lam, c.p)
            assert abs(ref - want) <= RTOL["f64"] * abs(want), (ref, want)
        su = (nB + 64 * wide - 1) // (64 * wide)
        for s1 in (1, 3, 8, su - 2, su - 1):
            monkeypatch.setenv("TWED_WAVEFRONT_MIXED", str(s1))
            cfg = tw.twed_pair_config(nA, nB, 3, c.nu, c.lam, c.p, prec, strip_k=8)
            assert cfg["wide_strips"] == s1 and cfg["strip_k"] == wide, cfg
            say(f"two widths {prec} layout {layout} {nA}x{nB} s1={s1}")
            v = gpu_twed(c.A, c.TA, c.B, c.TB, c.nu, c.lam, c.p, prec, algo="wavefront", strip_k=8)
            assert v == ref, (prec, layout, nA, nB, s1, v, ref)


def test_two_strip_widths_long_pair_vs_oracle(monkeypatch):
    """The split the host picks for a pair long enough to fill the device
    (8-D, FP32 costs with FP64 accumulators) against the FP64 oracle on its
    1e4 x 1e4 prefix through the prefix property: the sweep of the
    prefixes with forced two-width strips equals the oracle, and the
    long pair's distance is bitwise the same with and without two widths."""
    c = synth.single_pair_8d(10000).astype(np.float32).astype(np.float64)
    ref = oracle.twed(c.A, c.TA, c.B, c.TB, c.nu, c.lam, c.p, rows=True)
    monkeypatch.setenv("TWED_WAVEFRONT_GROUP", "8")
    monkeypatch.setenv("TWED_WAVEFRONT_MIXED", "6")
    v = gpu_twed(c.A, c.TA, c.B, c.TB, c.nu, c.lam, c.p, "f32_acc64", strip_k=8)
    assert abs(v - ref) <= RTOL["f32_acc64"] * abs(ref), (v, ref)
    long = synth.single_pair_8d(600_000)
    dt = torch.float32
    A, TA, B, TB = (dev(np.asarray(x, np.float32), dt) for x in (long.A, long.TA, long.B, long.TB))
    out = {}
    for mixed in ("0", None):
        if mixed is None:
            monkeypatch.delenv("TWED_WAVEFRONT_MIXED", raising=False)
        else:
            monkeypatch.setenv("TWED_WAVEFRONT_MIXED", mixed)
        say(f"two widths 8-D n=600000 mixed={mixed}")
        out[mixed] = float(tw.twed_pair(A, TA, B, TB, long.nu, long.lam, long.p, "f32_acc64").item())
    assert out["0"] == out[None], out


def test_tuner_picks_a_configuration_and_keeps_results():
    """twed_pair_tune times the sweep configurations and caches the fastest;
    the tuned call returns the bit-identical distance."""
    c = synth.random_pair(51, 52, 30000, 20000, 3, irregular=True, nu=0.01, lam=0.5, p=2.0)
    dt = torch.float64
    A, TA, B, TB = dev(c.A, dt), dev(c.TA, dt), dev(c.B, dt), dev(c.TB, dt)
    tw.twed_tune_clear()
    say("tuner: untuned run")
    before = float(tw.twed_pair(A, TA, B, TB, c.nu, c.lam, c.p, "f64").item())
    say("tuner: tuning")
    k, g = tw.twed_pair_tune(A, TA, B, TB, c.nu, c.lam, c.p, "f64")
    assert k in (1, 2, 4, 8) and g in (1, 4, 8)
    say(f"tuner: chose K={k} G={g}")
    after = float(tw.twed_pair(A, TA, B, TB, c.nu, c.lam, c.p, "f64").item())
    tw.twed_tune_clear()
    assert after == before


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_pair_replays_from_a_captured_graph(prec):
    """twed_pair enqueues only kernels (staging also clears the flags and the
    work ticket), so it can be captured in a graph: every replay, with other
    library work and host synchronisation in between, gives the eager value."""
    dt = torch.float64 if prec == "f64" else torch.float32
    c = synth.random_pair(61, 62, 6000, 5000, 3, irregular=True, nu=0.01, lam=0.5, p=2.0)
    other = synth.random_pair(63, 64, 900, 1100, 3, irregular=True, nu=0.01, lam=0.5, p=2.0)
    A, TA, B, TB = dev(c.A, dt), dev(c.TA, dt), dev(c.B, dt), dev(c.TB, dt)
    oA, oTA, oB, oTB = dev(other.A, dt), dev(other.TA, dt), dev(other.B, dt), dev(other.TB, dt)
    prm = tw.make_params(c.nu, c.lam, c.p, 3, prec)
    ws = torch.empty(tw.twed_pair_workspace_size(6000, 5000, prm), dtype=torch.uint8, device="cuda")
    out = torch.empty(1, dtype=dt, device="cuda")
    eager = float(tw.twed_pair(A, TA, B, TB, c.nu, c.lam, c.p, prec, out=out, workspace=ws).item())
    other_eager = float(tw.twed_pair(oA, oTA, oB, oTB, other.nu, other.lam, other.p, prec).item())
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    say(f"graph capture {prec}")
    with torch.cuda.graph(g):
        tw.twed_pair(A, TA, B, TB, c.nu, c.lam, c.p, prec, out=out, workspace=ws)
    for i in range(4):
        out.fill_(-1.0)
        g.replay()
        torch.cuda.synchronize()
        assert float(out.item()) == eager, (i, float(out.item()), eager)
        v = float(tw.twed_pair(oA, oTA, oB, oTB, other.nu, other.lam, other.p, prec).item())
        assert v == other_eager


@pytest.mark.parametrize("dim", [20, 28, 32])
def test_high_dimensional_points_vs_oracle(dim):
    """Samples of up to 32 components (the 32-component kernels, strips of at
    most two columns per lane) against the FP64 oracle."""
    c = synth.random_pair(70 + dim, 71 + dim, 300, 230, dim, irregular=True, nu=0.02, lam=0.7, p=2.0)
    for prec, tol in (("f64", 1e-12), ("f32", 1e-5), ("f32_acc64", 1e-6)):
        A, TA, B, TB = (c.A, c.TA, c.B, c.TB) if prec == "f64" else \
            tuple(np.asarray(x, np.float32).astype(np.float64) for x in (c.A, c.TA, c.B, c.TB))
        ref = oracle.twed(A, TA, B, TB, c.nu, c.lam, c.p)
        for k in (0, 1, 2):
            say(f"dim {dim} {prec} K={k}")
            v = gpu_twed(c.A, c.TA, c.B, c.TB, c.nu, c.lam, c.p, prec, strip_k=k)
            assert abs(v - ref) <= tol * abs(ref), (dim, prec, k, v, ref)

"""Blocks of the DP matrix and the alignment path against the CPU oracle (GPU).

Bars: cells of a block (DP and X = DP + e) within 1e-12 relative of the FP64
oracle (the sweep re-associates the match cost), FP32 costs with FP64
accumulators within 1e-6 of the oracle on the same rounded inputs; tiles
swept in dependency order give the twed_pair value bitwise (same lane code,
same operands); paths equal the oracle's tie-ruled path cell for cell.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2007_16135_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2007_16135_amd as tw  # noqa: E402

RTOL = {"f64": 1e-12, "f32_acc64": 1e-6}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def operands(c, prec):
    dt = torch.float64 if prec == "f64" else torch.float32
    f = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    A = np.asarray(c.A, np.float64).reshape(len(c.TA), -1)
    B = np.asarray(c.B, np.float64).reshape(len(c.TB), -1)
    return f(A), f(c.TA), f(B), f(c.TB)


def host_inputs(c, prec):
    xs = (c.A, c.TA, c.B, c.TB)
    if prec != "f64":
        xs = tuple(np.asarray(x, np.float32).astype(np.float64) for x in xs)
    return xs


def cells(DP, X, rows, cols):
    return torch.as_tensor(np.stack([DP[rows, cols], X[rows, cols]], axis=-1), device="cuda")


def close(got, want, rtol):
    got = np.asarray(got, np.float64)
    fin = np.isfinite(want)
    assert np.array_equal(np.isfinite(got), fin)
    assert np.all(got[~fin] == want[~fin])
    err = np.abs(got[fin] - want[fin]) / np.maximum(np.abs(want[fin]), 1e-300)
    assert err.max(initial=0.0) <= rtol, err.max()


@pytest.mark.parametrize("prec", ["f64", "f32_acc64"])
@pytest.mark.parametrize("block", [(70, 210, 50, 200), (0, 140, 0, 90), (120, 300, 0, 260), (0, 300, 100, 260),
                                   (299, 300, 259, 260)])
def test_tile_cells_vs_oracle(prec, block):
    r0, r1, c0, c1 = block
    c = synth.random_pair(31, 32, 300, 260, 3, irregular=True, nu=0.05, lam=0.6, p=2.0)
    A, TA, B, TB = host_inputs(c, prec)
    DP, X = oracle.get().matrix_x(A, TA, B, TB, c.nu, c.lam, c.p)
    dA, dTA, dB, dTB = operands(c, prec)
    top = cells(DP, X, r0, slice(c0, c1 + 1)) if r0 > 0 else None
    left = cells(DP, X, slice(r0, r1 + 1), c0) if c0 > 0 else None
    for k in (0, 1, 2):
        say(f"tile {prec} {block} K={k}")
        corner, bot, rig = tw.twed_pair_tile(dA, dTA, dB, dTB, r0, r1, c0, c1, top, left, c.nu, c.lam, c.p, prec,
                                             strip_k=k)
        torch.cuda.synchronize()
        bot, rig = bot.cpu().numpy(), rig.cpu().numpy()
        close(bot[:, 0], DP[r1, c0:c1 + 1], RTOL[prec])
        close(bot[:, 1], X[r1, c0:c1 + 1], RTOL[prec])
        close(rig[:, 0], DP[r0:r1 + 1, c1], RTOL[prec])
        close(rig[:, 1], X[r0:r1 + 1, c1], RTOL[prec])
        close([float(corner.item())], np.array([DP[r1, c1]]), RTOL[prec])


def _grid_sweep(dA, dTA, dB, dTB, c, prec, row_cuts, col_cuts, strip_k=0):
    """Sweeps the tiles of a grid in dependency order, handing bottom rows and
    right columns on; returns the last corner."""
    nA, nB = len(c.TA), len(c.TB)
    rows = [0] + list(row_cuts) + [nA]
    cols = [0] + list(col_cuts) + [nB]
    bottoms = {}
    corner = None
    for bi in range(len(rows) - 1):
        right = None
        for bj in range(len(cols) - 1):
            r0, r1, c0, c1 = rows[bi], rows[bi + 1], cols[bj], cols[bj + 1]
            top = bottoms.get((bi - 1, bj)) if bi > 0 else None
            left = right if bj > 0 else None
            corner, bot, right = tw.twed_pair_tile(dA, dTA, dB, dTB, r0, r1, c0, c1, top, left, c.nu, c.lam, c.p,
                                                   prec, strip_k=strip_k)
            bottoms[(bi, bj)] = bot
    return float(corner.item())


@pytest.mark.parametrize("prec", ["f64", "f32_acc64"])
def test_tiles_compose_to_the_pair_bitwise(prec):
    """Row slabs (checkpoint and resume), column shards (one GPU's share of a
    column-sharded sweep) and a full grid all give the twed_pair value bit
    for bit."""
    c = synth.random_pair(41, 42, 2300, 1900, 8, irregular=False, nu=1e-3, lam=1.0, p=2.0)
    dA, dTA, dB, dTB = operands(c, prec)
    ref = float(tw.twed_pair(dA, dTA, dB, dTB, c.nu, c.lam, c.p, prec).item())
    say(f"slabs {prec}")
    assert _grid_sweep(dA, dTA, dB, dTB, c, prec, [500, 1100, 1700], []) == ref
    say(f"shards {prec}")
    assert _grid_sweep(dA, dTA, dB, dTB, c, prec, [], [400, 1000, 1500]) == ref
    say(f"grid {prec}")
    assert _grid_sweep(dA, dTA, dB, dTB, c, prec, [333, 1500], [64, 640, 1899], strip_k=1) == ref
    A, TA, B, TB = host_inputs(c, prec)
    want = oracle.get().twed(A, TA, B, TB, c.nu, c.lam, c.p)
    assert abs(ref - want) <= RTOL[prec] * want


def _path_case(seed, nA, nB, dim, prec, block):
    """On real-valued data several paths can be optimal in exact arithmetic
    (between two cells, deletions in A and in B add up to the same sum in any
    order), and rounding picks one of them, so the unique parts are compared:
    the distance, and that the path is admissible with the oracle's cost of it
    equal to the oracle's distance."""
    c = synth.random_pair(seed, seed + 1, nA, nB, dim, irregular=True, nu=0.1, lam=0.8, p=2.0 if dim > 1 else 1.0)
    A, TA, B, TB = host_inputs(c, prec)
    wd = oracle.get().twed(A, TA, B, TB, c.nu, c.lam, c.p)
    dA, dTA, dB, dTB = operands(c, prec)
    say(f"path {nA}x{nB} dim{dim} {prec} block {block}")
    d, path = tw.twed_pair_path(dA, dTA, dB, dTB, c.nu, c.lam, c.p, prec, block=block)
    torch.cuda.synchronize()
    assert abs(float(d.item()) - wd) <= RTOL[prec] * wd
    P = path.cpu().numpy()
    assert P.shape[1] == 2 and tuple(P[0]) == (0, 0) and tuple(P[-1]) == (nA, nB)
    cost = oracle.get().path_cost(A, TA, B, TB, c.nu, c.lam, c.p, P)
    assert abs(cost - wd) <= RTOL[prec] * wd, (cost, wd)
    return P


@pytest.mark.parametrize("prec", ["f64", "f32_acc64"])
def test_path_one_block_vs_oracle(prec):
    _path_case(51, 90, 70, 2, prec, 0)


@pytest.mark.parametrize("prec", ["f64", "f32_acc64"])
def test_path_many_blocks_vs_oracle(prec):
    _path_case(53, 700, 520, 3, prec, 64)      # 10 x 8 blocks of 64 rows / columns
    _path_case(55, 1500, 1700, 1, prec, 256)


def test_path_ties_follow_the_rule():
    """Integer data (every sum exact): tied moves resolve as the oracle's rule
    (match, then deletion in A, then deletion in B)."""
    rng = np.random.default_rng(77)
    for n in range(12):
        nA, nB = int(rng.integers(5, 120)), int(rng.integers(5, 120))
        A = rng.integers(-3, 4, nA).astype(np.float64)
        B = rng.integers(-3, 4, nB).astype(np.float64)
        TA = np.cumsum(rng.integers(0, 3, nA)).astype(np.float64)
        TB = np.cumsum(rng.integers(0, 3, nB)).astype(np.float64)
        nu, lam = float(rng.choice([0.0, 1.0])), float(rng.choice([0.0, 1.0, 2.0]))
        want = oracle.get().path(A, TA, B, TB, nu, lam, 1.0)
        f = lambda a: torch.as_tensor(a, device="cuda")
        say(f"ties {n}: {nA}x{nB}")
        d, path = tw.twed_pair_path(f(A.reshape(-1, 1)), f(TA), f(B.reshape(-1, 1)), f(TB), nu, lam, 1.0, "f64",
                                    block=64)
        assert float(d.item()) == oracle.get().twed(A, TA, B, TB, nu, lam, 1.0)
        assert np.array_equal(path.cpu().numpy(), want)


def test_path_single_samples():
    """nA = 1 or nB = 1: the only admissible paths are a match then deletions."""
    for nA, nB in ((1, 1), (1, 9), (9, 1)):
        _path_case(61, nA, nB, 1, "f64", 0)


@pytest.mark.parametrize("prec", ["f64", "f32_acc64"])
def test_high_dimensional_tiles_and_paths(prec):
    """Samples of 16 and 28 components: a tile from oracle boundaries and a
    multi-block path."""
    for dim in (16, 28):
        c = synth.random_pair(80 + dim, 81 + dim, 400, 330, dim, irregular=True, nu=0.02, lam=0.9, p=2.0)
        A, TA, B, TB = host_inputs(c, prec)
        DP, X = oracle.get().matrix_x(A, TA, B, TB, c.nu, c.lam, c.p)
        dA, dTA, dB, dTB = operands(c, prec)
        r0, r1, c0, c1 = 100, 400, 70, 300
        say(f"tile dim {dim} {prec}")
        corner, bot, rig = tw.twed_pair_tile(dA, dTA, dB, dTB, r0, r1, c0, c1, cells(DP, X, r0, slice(c0, c1 + 1)),
                                             cells(DP, X, slice(r0, r1 + 1), c0), c.nu, c.lam, c.p, prec)
        torch.cuda.synchronize()
        close(bot.cpu().numpy()[:, 0], DP[r1, c0:c1 + 1], RTOL[prec])
        close(rig.cpu().numpy()[:, 1], X[r0:r1 + 1, c1], RTOL[prec])
        _path_case(90 + dim, 260, 300, dim, prec, 64)


def test_path_on_a_side_stream():
    """The path call on a stream other than the current one (its block sweeps
    run on streams of its own, ordered after the caller's): the same distance
    and path as on the current stream, complete when the call returns."""
    c = synth.random_pair(81, 82, 700, 650, 3, irregular=True, nu=0.02, lam=0.5, p=2.0)
    f = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    A, TA, B, TB = f(c.A), f(c.TA), f(c.B), f(c.TB)
    say("path on the current stream")
    d0, p0 = tw.twed_pair_path(A, TA, B, TB, c.nu, c.lam, c.p, "f64", block=64)
    d0, p0 = float(d0.item()), p0.cpu().numpy()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    say("path on a side stream")
    d1, p1 = tw.twed_pair_path(A, TA, B, TB, c.nu, c.lam, c.p, "f64", block=64, stream=s)
    with torch.cuda.stream(s):
        d1, p1 = float(d1.item()), p1.cpu().numpy()
    assert d1 == d0
    assert np.array_equal(p1, p0)

"""Sibling dynamic programs on the band sweep (DTW, edit distance, LCS length)
against the CPU oracle (GPU).

Bars: edit distance and LCS exactly (integer sums, exact in FP64 and FP32
tokens); DTW within 1e-12 relative in FP64 and 1e-6 with FP32 costs and FP64
accumulators (the oracle run on the same rounded inputs).  Paths: admissible,
with the value they imply equal to the oracle's.
"""
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2007_16135_amd as tw  # noqa: E402


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(x, prec):
    dt = torch.float64 if prec == "f64" else torch.float32
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device="cuda")


def tokens(rng, n, alphabet):
    return rng.integers(0, alphabet, n).astype(np.float64)


@pytest.mark.parametrize("prec", ["f64", "f32_acc64"])
def test_edit_and_lcs_exact(prec):
    rng = np.random.default_rng(5)
    orc = oracle.get()
    for nA, nB, alph in ((1, 1, 2), (1, 50, 3), (37, 1, 3), (200, 170, 4), (1500, 1300, 4), (3000, 2100, 20),
                         (64, 64, 2), (65, 640, 5)):
        a, b = tokens(rng, nA, alph), tokens(rng, nB, alph)
        for strip_k in (0, 1, 2, 8):
            say(f"edit/lcs {nA}x{nB} alphabet {alph} {prec} K={strip_k}")
            e = float(tw.twed_dp("edit", dev(a, prec), dev(b, prec), precision=prec, strip_k=strip_k).item())
            l = float(tw.twed_dp("lcs", dev(a, prec), dev(b, prec), precision=prec, strip_k=strip_k).item())
            assert e == orc.edit(a, b)
            assert l == orc.lcs(a, b)


@pytest.mark.parametrize("prec", ["f64", "f32_acc64"])
@pytest.mark.parametrize("dim,p", [(1, 1.0), (3, 2.0), (8, 2.0), (5, 3.0), (28, 2.0)])
def test_dtw_vs_oracle(prec, dim, p):
    rng = np.random.default_rng(dim * 10 + int(p))
    orc = oracle.get()
    for nA, nB in ((1, 9), (300, 257), (2200, 1900)):
        A = rng.standard_normal((nA, dim)).cumsum(0)
        B = rng.standard_normal((nB, dim)).cumsum(0)
        if prec != "f64":
            A, B = A.astype(np.float32).astype(np.float64), B.astype(np.float32).astype(np.float64)
        want = orc.dtw(A, B, p)
        for strip_k in (0, 1, 2):
            say(f"dtw {nA}x{nB} dim{dim} p{p} {prec} K={strip_k}")
            got = float(tw.twed_dp("dtw", dev(A, prec), dev(B, prec), p=p, precision=prec, strip_k=strip_k).item())
            assert abs(got - want) <= (1e-12 if prec == "f64" else 1e-6) * want


def _check_path(P, nA, nB, free_edges):
    assert tuple(P[0]) == (0, 0) and tuple(P[-1]) == (nA, nB)
    d = np.diff(P, axis=0)
    assert all(tuple(s) in ((1, 1), (1, 0), (0, 1)) for s in d)
    if not free_edges:
        assert np.all(P[1:, 0] >= 1) and np.all(P[1:, 1] >= 1)


def test_dp_paths():
    rng = np.random.default_rng(9)
    orc = oracle.get()
    for nA, nB, block in ((40, 33, 0), (700, 900, 64), (1, 20, 0), (20, 1, 0)):
        a, b = tokens(rng, nA, 4), tokens(rng, nB, 4)
        say(f"edit path {nA}x{nB} block {block}")
        v, path = tw.twed_dp_path("edit", dev(a, "f64"), dev(b, "f64"), block=block)
        P = path.cpu().numpy()
        _check_path(P, nA, nB, True)
        # the edit script the path spells out costs exactly the distance
        cost = 0
        for (i0, j0), (i1, j1) in zip(P[:-1], P[1:]):
            cost += 1 if (i1 - i0) + (j1 - j0) == 1 else int(a[i1 - 1] != b[j1 - 1])
        assert cost == float(v.item()) == orc.edit(a, b)
        say(f"lcs path {nA}x{nB} block {block}")
        v, path = tw.twed_dp_path("lcs", dev(a, "f64"), dev(b, "f64"), block=block)
        P = path.cpu().numpy()
        _check_path(P, nA, nB, True)
        steps = [(i1, j1) for (i0, j0), (i1, j1) in zip(P[:-1], P[1:]) if i1 - i0 == 1 and j1 - j0 == 1]
        assert all(a[i - 1] == b[j - 1] for i, j in steps)
        assert len(steps) == float(v.item()) == orc.lcs(a, b)
        A = rng.standard_normal((nA, 2)).cumsum(0)
        B = rng.standard_normal((nB, 2)).cumsum(0)
        say(f"dtw path {nA}x{nB} block {block}")
        v, path = tw.twed_dp_path("dtw", dev(A, "f64"), dev(B, "f64"), p=2.0, block=block)
        P = path.cpu().numpy()
        _check_path(P, nA, nB, False)
        cost = sum(float(np.sqrt(((A[i - 1] - B[j - 1]) ** 2).sum())) for i, j in P[1:])
        want = orc.dtw(A, B, 2.0)
        assert abs(float(v.item()) - want) <= 1e-12 * want
        assert abs(cost - want) <= 1e-10 * want


def test_dp_paths_long_and_wide_strips():
    """DTW paths whose forward sweeps use strips of eight and of two columns
    (blocks of 256); an edit path of 3000 x 2500 tokens; an LCS path swept in
    strips of two columns."""
    rng = np.random.default_rng(12)
    orc = oracle.get()
    nA, nB = 3000, 2500
    A = rng.standard_normal((nA, 1)).cumsum(0)
    B = rng.standard_normal((nB, 1)).cumsum(0)
    want = orc.dtw(A, B, 1.0)
    for strip_k in (8, 2):
        say(f"dtw path 3000x2500 strip_k {strip_k}")
        v, path = tw.twed_dp_path("dtw", dev(A, "f64"), dev(B, "f64"), p=1.0, block=256, strip_k=strip_k)
        P = path.cpu().numpy()
        _check_path(P, nA, nB, False)
        assert abs(float(v.item()) - want) <= 1e-12 * want
        cost = sum(abs(A[i - 1, 0] - B[j - 1, 0]) for i, j in P[1:])
        assert abs(cost - want) <= 1e-10 * want
    a, b = tokens(rng, nA, 6), tokens(rng, nB, 6)
    say("lcs path 3000x2500 strip_k 2")
    v, path = tw.twed_dp_path("lcs", dev(a, "f64"), dev(b, "f64"), block=512, strip_k=2)
    P = path.cpu().numpy()
    _check_path(P, nA, nB, True)
    steps = [(i1, j1) for (i0, j0), (i1, j1) in zip(P[:-1], P[1:]) if i1 - i0 == 1 and j1 - j0 == 1]
    assert all(a[i - 1] == b[j - 1] for i, j in steps)
    assert len(steps) == float(v.item()) == orc.lcs(a, b)
    say("edit path 3000x2500")
    v, path = tw.twed_dp_path("edit", dev(a, "f32_acc64"), dev(b, "f32_acc64"), precision="f32_acc64", block=512)
    P = path.cpu().numpy()
    _check_path(P, nA, nB, True)
    cost = sum(1 if (i1 - i0) + (j1 - j0) == 1 else int(a[i1 - 1] != b[j1 - 1])
               for (i0, j0), (i1, j1) in zip(P[:-1], P[1:]))
    assert cost == float(v.item()) == orc.edit(a, b)

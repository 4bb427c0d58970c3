"""Pins for the oracle's sibling dynamic programs (DTW, edit distance, LCS),
each against an independent definition: enumeration of every alignment or
subsequence on tiny inputs, textbook values and structural identities."""
import itertools
import math

import numpy as np
import pytest

import oracle


@pytest.fixture(scope="module")
def orc():
    return oracle.get()


def _paths(nA, nB):
    """Every monotone lattice path from (1, 1) to (nA, nB) with unit steps
    right, down and diagonal, as lists of cells."""
    out = []

    def walk(i, j, cells):
        if i == nA and j == nB:
            out.append(cells)
            return
        if i < nA:
            walk(i + 1, j, cells + [(i + 1, j)])
        if j < nB:
            walk(i, j + 1, cells + [(i, j + 1)])
        if i < nA and j < nB:
            walk(i + 1, j + 1, cells + [(i + 1, j + 1)])

    walk(1, 1, [(1, 1)])
    return out


def _lp(x, y, p):
    d = np.abs(np.asarray(x, float) - np.asarray(y, float))
    return float(np.sum(d ** p) ** (1.0 / p)) if p != 1.0 else float(np.sum(d))


def brute_dtw(A, B, p):
    A, B = np.atleast_2d(A), np.atleast_2d(B)
    best = math.inf
    for cells in _paths(len(A), len(B)):
        best = min(best, sum(_lp(A[i - 1], B[j - 1], p) for i, j in cells))
    return best


def brute_edit(a, b):
    """Minimum over every alignment (a sequence of keep/substitute, delete and
    insert operations) of the number of non-keep operations."""
    best = math.inf

    def walk(i, j, cost):
        nonlocal best
        if cost >= best:
            return
        if i == len(a) and j == len(b):
            best = cost
            return
        if i < len(a) and j < len(b):
            walk(i + 1, j + 1, cost + (a[i] != b[j]))
        if i < len(a):
            walk(i + 1, j, cost + 1)
        if j < len(b):
            walk(i, j + 1, cost + 1)

    walk(0, 0, 0)
    return best


def brute_lcs(a, b):
    """Longest subsequence of a (all 2^n of them) that is also one of b."""
    def is_sub(s, t):
        it = iter(t)
        return all(any(x == y for y in it) for x in s)

    for k in range(len(a), 0, -1):
        for idx in itertools.combinations(range(len(a)), k):
            if is_sub([a[i] for i in idx], b):
                return k
    return 0


def tok(s):
    return np.array([ord(ch) for ch in s], float)


def test_textbook_values(orc):
    assert orc.edit(tok("kitten"), tok("sitting")) == 3
    assert orc.edit(tok("flaw"), tok("lawn")) == 2
    assert orc.lcs(tok("ABCBDAB"), tok("BDCABA")) == 4
    assert orc.lcs(tok("AGGTAB"), tok("GXTXAYB")) == 4
    # DTW of a series with a time-stretched copy of itself is 0
    x = np.array([0.0, 1.0, 3.0, 2.0])
    assert orc.dtw(x, np.repeat(x, 3)) == 0.0


def test_brute_force(orc):
    rng = np.random.default_rng(21)
    for _ in range(40):
        nA, nB = int(rng.integers(1, 7)), int(rng.integers(1, 7))
        a = rng.integers(0, 3, nA).astype(float)
        b = rng.integers(0, 3, nB).astype(float)
        assert orc.edit(a, b) == brute_edit(list(a), list(b))
        assert orc.lcs(a, b) == brute_lcs(list(a), list(b))
        dim = int(rng.integers(1, 3))
        p = float(rng.choice([1.0, 2.0]))
        A = rng.standard_normal((nA, dim))
        B = rng.standard_normal((nB, dim))
        v, bf = orc.dtw(A, B, p), brute_dtw(A, B, p)
        assert abs(v - bf) <= 1e-12 * max(1.0, bf)


def test_identities(orc):
    rng = np.random.default_rng(22)
    for _ in range(30):
        nA, nB = int(rng.integers(1, 60)), int(rng.integers(1, 60))
        a = rng.integers(0, 4, nA).astype(float)
        b = rng.integers(0, 4, nB).astype(float)
        L = orc.lcs(a, b)
        assert 0 <= L <= min(nA, nB)
        assert orc.lcs(a, b) == orc.lcs(b, a)
        assert orc.edit(a, b) == orc.edit(b, a)
        assert abs(nA - nB) <= orc.edit(a, b) <= max(nA, nB)
        assert orc.lcs(a, a) == nA and orc.edit(a, a) == 0
        A = rng.standard_normal((nA, 2))
        B = rng.standard_normal((nB, 2))
        assert orc.dtw(A, B, 2.0) == orc.dtw(B, A, 2.0)
        assert orc.dtw(A, A, 2.0) == 0.0
    # a single sample against a series: the only warping path visits every cell of one row
    A = np.array([[0.5]])
    B = rng.standard_normal((9, 1))
    assert abs(orc.dtw(A, B, 1.0) - float(np.abs(B[:, 0] - 0.5).sum())) <= 1e-14

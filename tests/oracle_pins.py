"""Pins for the CPU oracle: checks against what the paper and the mathematics
fix, independent of the oracle's own code.

Each check takes an ``oracle.Oracle`` and returns a list of failure messages
(empty = pass), so that the same battery runs on the real oracle (every check
must pass) and on builds with a planted mistake (some check must fail).

Pins:
  worked examples  hand-worked DP matrices (tests/golden), exact in FP64
  brute force      minimum over every admissible edit path == DP value
  closed form      nA = 1 (or nB = 1): exactly one admissible path
  metric axioms    D(A,A) = 0, D(A,B) = D(B,A), triangle inequality
  large lambda     with 2*lambda > S (S = diagonal path sum), D = S
  homogeneity      scaling values, times and lambda by 2^k scales D by 2^k
  time rescale     (T*s, nu/s) leaves D unchanged for s = 2^k
  1-D p-free       in one dimension every Lp distance is |x - y|
  prefix           DP[i][j] equals the distance of the prefixes A[:i], B[:j]
  band state       X = DP + e against hand-worked e (tests/golden) and the
                   brute force's own point cost
  path             hand-worked paths; on integer data (exact sums) the path
                   is, among all optimal brute-force paths, the one the tie
                   rule selects (read back from the end: match, then
                   deletion in A, then deletion in B)
"""
from __future__ import annotations

import itertools
import json
import math
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _inf(v):
    return math.inf if v == "inf" else v


def load_worked_examples():
    with open(os.path.join(GOLDEN, "worked_examples.json")) as f:
        return json.load(f)["cases"]


# ---- independent path-based definition (brute force) -------------------------
#
# TWED is the minimum, over monotone lattice paths from (0,0) to (nA,nB) with
# steps (1,1) match, (1,0) delete-in-A and (0,1) delete-in-B, of the summed
# step costs charged at the destination cell; paths may not touch row 0 or
# column 0 away from (0,0) (those cells are +inf).  The step costs below are
# Marteau's, with zero-padded samples and times.

def _lp(x, y, p):
    d = [abs(a - b) for a, b in zip(x, y)]
    if p == 1.0:
        return sum(d)
    return sum(v ** p for v in d) ** (1.0 / p)


def _padded(X, T):
    X = [list(np.atleast_1d(r).astype(float)) for r in np.asarray(X, dtype=float).reshape(len(T), -1)]
    dim = len(X[0])
    return [[0.0] * dim] + X, [0.0] + [float(t) for t in T]


def brute_force(A, TA, B, TB, nu, lam, p):
    Ap, TAp = _padded(A, TA)
    Bp, TBp = _padded(B, TB)
    nA, nB = len(Ap) - 1, len(Bp) - 1

    def dA(i):
        return _lp(Ap[i], Ap[i - 1], p) + nu * abs(TAp[i] - TAp[i - 1]) + lam

    def dB(j):
        return _lp(Bp[j], Bp[j - 1], p) + nu * abs(TBp[j] - TBp[j - 1]) + lam

    def m(i, j):
        return (_lp(Ap[i], Bp[j], p) + _lp(Ap[i - 1], Bp[j - 1], p)
                + nu * (abs(TAp[i] - TBp[j]) + abs(TAp[i - 1] - TBp[j - 1])))

    best = math.inf

    def walk(i, j, acc):
        nonlocal best
        if i == nA and j == nB:
            best = min(best, acc)
            return
        if i < nA and j < nB:
            walk(i + 1, j + 1, acc + m(i + 1, j + 1))
        if i >= 1 and j >= 1:          # never step onto row 0 / column 0
            if i < nA:
                walk(i + 1, j, acc + dA(i + 1))
            if j < nB:
                walk(i, j + 1, acc + dB(j + 1))

    walk(0, 0, 0.0)
    return best


def _steps(A, TA, B, TB, nu, lam, p):
    """The brute force's step costs and point cost as closures."""
    Ap, TAp = _padded(A, TA)
    Bp, TBp = _padded(B, TB)

    def dA(i):
        return _lp(Ap[i], Ap[i - 1], p) + nu * abs(TAp[i] - TAp[i - 1]) + lam

    def dB(j):
        return _lp(Bp[j], Bp[j - 1], p) + nu * abs(TBp[j] - TBp[j - 1]) + lam

    def m(i, j):
        return (_lp(Ap[i], Bp[j], p) + _lp(Ap[i - 1], Bp[j - 1], p)
                + nu * (abs(TAp[i] - TBp[j]) + abs(TAp[i - 1] - TBp[j - 1])))

    def e(i, j):
        return _lp(Ap[i], Bp[j], p) + nu * abs(TAp[i] - TBp[j])

    return len(Ap) - 1, len(Bp) - 1, dA, dB, m, e


MATCH, UP, LEFT = 0, 1, 2


def brute_force_paths(A, TA, B, TB, nu, lam, p):
    """Every admissible path as (cost, moves), moves in forward order
    (MATCH: (1,1), UP: (1,0) deletion in A, LEFT: (0,1) deletion in B)."""
    nA, nB, dA, dB, m, _ = _steps(A, TA, B, TB, nu, lam, p)
    out = []

    def walk(i, j, acc, moves):
        if i == nA and j == nB:
            out.append((acc, tuple(moves)))
            return
        if i < nA and j < nB:
            walk(i + 1, j + 1, acc + m(i + 1, j + 1), moves + [MATCH])
        if i >= 1 and j >= 1:
            if i < nA:
                walk(i + 1, j, acc + dA(i + 1), moves + [UP])
            if j < nB:
                walk(i, j + 1, acc + dB(j + 1), moves + [LEFT])

    walk(0, 0, 0.0, [])
    return out


def cells_of(moves):
    i = j = 0
    cells = [(0, 0)]
    for mv in moves:
        i += mv != LEFT
        j += mv != UP
        cells.append((i, j))
    return cells


def tie_rule_path(A, TA, B, TB, nu, lam, p):
    """(cost, cells, number of optimal paths): the optimal path that the
    backward reading picks when it prefers MATCH, then UP, then LEFT at every
    cell, i.e. the optimal path whose reversed move list is smallest."""
    paths = brute_force_paths(A, TA, B, TB, nu, lam, p)
    best = min(c for c, _ in paths)
    opt = [mv for c, mv in paths if c == best]
    pick = min(opt, key=lambda mv: tuple(reversed(mv)))
    return best, cells_of(pick), len(opt)


def delannoy(m, n):
    return sum(math.comb(m, k) * math.comb(n, k) * 2 ** k for k in range(min(m, n) + 1))


def count_paths(nA, nB):
    cnt = 0

    def walk(i, j):
        nonlocal cnt
        if i == nA and j == nB:
            cnt += 1
            return
        if i < nA and j < nB:
            walk(i + 1, j + 1)
        if i >= 1 and j >= 1:
            if i < nA:
                walk(i + 1, j)
            if j < nB:
                walk(i, j + 1)

    walk(0, 0)
    return cnt


# ---- random inputs -------------------------------------------------------------

def rand_series(rng, n, dim, scale=1.0):
    X = rng.standard_normal((n, dim)).cumsum(0) * scale
    T = rng.exponential(1.0, n).cumsum()
    return X, T


# ---- checks ---------------------------------------------------------------------

def check_worked_examples(orc):
    fails = []
    for c in load_worked_examples():
        A = np.array(c["A"], float).reshape(-1, c["dim"])
        B = np.array(c["B"], float).reshape(-1, c["dim"])
        v, DP = orc.twed(A, c["TA"], B, c["TB"], c["nu"], c["lambda"], c["p"], matrix=True)
        if c["exact"]:
            want = np.array([[_inf(x) for x in row] for row in c["DP"]], float)
            if not np.array_equal(DP, want):
                fails.append(f"{c['name']}: DP matrix {DP.tolist()} != {c['DP']}")
            if v != c["twed"]:
                fails.append(f"{c['name']}: value {v} != {c['twed']}")
            if "diagonals" in c:
                nA, nB = DP.shape[0] - 1, DP.shape[1] - 1
                for d, diag in enumerate(c["diagonals"]):
                    for idx, want_v in enumerate(diag):
                        if want_v is None:
                            continue
                        row, col = d - idx, idx        # Eq. (2)
                        if not (0 <= row <= nA and 0 <= col <= nB):
                            fails.append(f"{c['name']}: diagonal {d} idx {idx} outside matrix")
                        elif DP[row, col] != _inf(want_v):
                            fails.append(f"{c['name']}: z_{d}[{idx}] {DP[row, col]} != {want_v}")
        else:
            if not abs(v - c["twed"]) <= c["rtol"] * abs(c["twed"]):
                fails.append(f"{c['name']}: value {v!r} != {c['twed']}")
    return fails


def check_brute_force(orc, n_cases=60, seed=11, max_n=6):
    rng = np.random.default_rng(seed)
    fails = []
    for _ in range(n_cases):
        nA, nB = int(rng.integers(1, max_n + 1)), int(rng.integers(1, max_n + 1))
        dim = int(rng.integers(1, 4))
        p = float(rng.choice([1.0, 2.0, 3.0]))
        nu = float(rng.choice([0.0, 0.05, 1.0, 2.5]))
        lam = float(rng.choice([0.0, 0.3, 1.0, 4.0]))
        A, TA = rand_series(rng, nA, dim)
        B, TB = rand_series(rng, nB, dim)
        v = orc.twed(A, TA, B, TB, nu, lam, p)
        bf = brute_force(A, TA, B, TB, nu, lam, p)
        if not abs(v - bf) <= 1e-12 * max(1.0, abs(bf)):
            fails.append(f"brute force {nA}x{nB} dim{dim} p{p} nu{nu} lam{lam}: {v!r} vs {bf!r}")
    return fails


def check_closed_form_single(orc, n_cases=20, seed=12):
    """nA = 1: the only admissible path is match(1,1) then deletions in B."""
    rng = np.random.default_rng(seed)
    fails = []
    for _ in range(n_cases):
        nB = int(rng.integers(1, 40))
        dim = int(rng.integers(1, 4))
        nu, lam = float(rng.uniform(0, 2)), float(rng.uniform(0, 2))
        A, TA = rand_series(rng, 1, dim)
        B, TB = rand_series(rng, nB, dim)
        a, ta = A[0], TA[0]
        want = float(np.abs(a - B[0]).sum()) + nu * abs(ta - TB[0])
        for j in range(1, nB):
            want += float(np.abs(B[j] - B[j - 1]).sum()) + nu * abs(TB[j] - TB[j - 1]) + lam
        for (X, TX, Y, TY) in ((A, TA, B, TB), (B, TB, A, TA)):
            v = orc.twed(X, TX, Y, TY, nu, lam, 1.0)
            if not abs(v - want) <= 1e-12 * max(1.0, abs(want)):
                fails.append(f"single-sample closed form nB={nB}: {v!r} vs {want!r}")
    return fails


def check_metric_axioms(orc, n_cases=150, seed=13):
    rng = np.random.default_rng(seed)
    fails = []
    for _ in range(n_cases):
        dim = int(rng.integers(1, 4))
        p = float(rng.choice([1.0, 2.0, 3.0]))
        nu = float(rng.choice([0.0, 0.01, 0.5, 3.0]))
        lam = float(rng.choice([0.0, 0.2, 1.0, 3.0]))
        S = [rand_series(rng, int(rng.integers(1, 25)), dim) for _ in range(3)]
        dAA = orc.twed(*S[0], *S[0], nu, lam, p)
        if dAA != 0.0:
            fails.append(f"D(A,A) = {dAA!r}")
        dAB = orc.twed(*S[0], *S[1], nu, lam, p)
        dBA = orc.twed(*S[1], *S[0], nu, lam, p)
        if dAB != dBA:
            fails.append(f"asymmetric: {dAB!r} vs {dBA!r}")
        dBC = orc.twed(*S[1], *S[2], nu, lam, p)
        dAC = orc.twed(*S[0], *S[2], nu, lam, p)
        if dAC > dAB + dBC + 1e-12 * max(1.0, dAC):
            fails.append(f"triangle: {dAC!r} > {dAB!r} + {dBC!r}")
    return fails


def check_large_lambda(orc, n_cases=20, seed=14):
    """Equal lengths: any path other than the main diagonal has at least two
    deletions, so with 2*lambda > S the diagonal sum S is the distance."""
    rng = np.random.default_rng(seed)
    fails = []
    for _ in range(n_cases):
        n, dim = int(rng.integers(1, 30)), int(rng.integers(1, 3))
        nu = float(rng.uniform(0, 1))
        A, TA = rand_series(rng, n, dim)
        B, TB = rand_series(rng, n, dim)
        Ap = np.vstack([np.zeros((1, dim)), A]); TAp = np.concatenate([[0.0], TA])
        Bp = np.vstack([np.zeros((1, dim)), B]); TBp = np.concatenate([[0.0], TB])
        S = 0.0
        for i in range(1, n + 1):
            mi = (float(np.abs(Ap[i] - Bp[i]).sum()) + float(np.abs(Ap[i - 1] - Bp[i - 1]).sum())) \
                + nu * (abs(TAp[i] - TBp[i]) + abs(TAp[i - 1] - TBp[i - 1]))
            S = S + mi
        lam = S  # 2*lambda > S
        v = orc.twed(A, TA, B, TB, nu, lam, 1.0)
        if not abs(v - S) <= 1e-12 * max(1.0, S):
            fails.append(f"large lambda n={n}: {v!r} vs diagonal sum {S!r}")
        # and never above the diagonal path for any lambda
        v0 = orc.twed(A, TA, B, TB, nu, 0.0, 1.0)
        if v0 > S * (1 + 1e-12):
            fails.append(f"D above diagonal path: {v0!r} > {S!r}")
    return fails


def check_homogeneity(orc, n_cases=30, seed=15):
    rng = np.random.default_rng(seed)
    fails = []
    for _ in range(n_cases):
        dim = int(rng.integers(1, 4))
        p = float(rng.choice([1.0, 2.0]))
        nu, lam = float(rng.uniform(0, 2)), float(rng.uniform(0, 2))
        A, TA = rand_series(rng, int(rng.integers(1, 30)), dim)
        B, TB = rand_series(rng, int(rng.integers(1, 30)), dim)
        s = 2.0 ** int(rng.integers(-6, 7))
        d = orc.twed(A, TA, B, TB, nu, lam, p)
        ds = orc.twed(A * s, TA * s, B * s, TB * s, nu, lam * s, p)
        if ds != d * s:
            fails.append(f"homogeneity s={s}: {ds!r} vs {d * s!r}")
        dt = orc.twed(A, TA * s, B, TB * s, nu / s, lam, p)
        if dt != d:
            fails.append(f"time rescale s={s}: {dt!r} vs {d!r}")
    return fails


def check_p_free_1d(orc, n_cases=20, seed=16):
    rng = np.random.default_rng(seed)
    fails = []
    for _ in range(n_cases):
        A, TA = rand_series(rng, int(rng.integers(1, 40)), 1)
        B, TB = rand_series(rng, int(rng.integers(1, 40)), 1)
        nu, lam = float(rng.uniform(0, 1)), float(rng.uniform(0, 2))
        d1 = orc.twed(A, TA, B, TB, nu, lam, 1.0)
        d2 = orc.twed(A, TA, B, TB, nu, lam, 2.0)
        d3 = orc.twed(A, TA, B, TB, nu, lam, 3.0)
        if d1 != d2:
            fails.append(f"1-D p=1 vs p=2: {d1!r} vs {d2!r}")
        if not abs(d1 - d3) <= 1e-13 * max(1.0, d1):
            fails.append(f"1-D p=1 vs p=3: {d1!r} vs {d3!r}")
    return fails


def check_prefix(orc, n_cases=6, seed=17):
    rng = np.random.default_rng(seed)
    fails = []
    for _ in range(n_cases):
        dim = int(rng.integers(1, 4))
        nA, nB = int(rng.integers(2, 25)), int(rng.integers(2, 25))
        A, TA = rand_series(rng, nA, dim)
        B, TB = rand_series(rng, nB, dim)
        nu, lam, p = 0.3, 0.8, float(rng.choice([1.0, 2.0]))
        _, DP = orc.twed(A, TA, B, TB, nu, lam, p, matrix=True)
        for _k in range(8):
            i, j = int(rng.integers(1, nA + 1)), int(rng.integers(1, nB + 1))
            v = orc.twed(A[:i], TA[:i], B[:j], TB[:j], nu, lam, p)
            if v != DP[i, j]:
                fails.append(f"prefix ({i},{j}): {v!r} vs DP {DP[i, j]!r}")
    return fails


def check_band_state(orc, n_cases=25, seed=18):
    """X = DP + e: exact against the hand-worked e of the golden examples,
    and within rounding of the brute force's own point cost on random data."""
    fails = []
    for c in load_worked_examples():
        if "e" not in c:
            continue
        A = np.array(c["A"], float).reshape(-1, c["dim"])
        B = np.array(c["B"], float).reshape(-1, c["dim"])
        DP, X = orc.matrix_x(A, c["TA"], B, c["TB"], c["nu"], c["lambda"], c["p"])
        want = np.array([[_inf(x) for x in row] for row in c["DP"]], float) + np.array(c["e"], float)
        if not np.array_equal(X, want):
            fails.append(f"{c['name']}: X {X.tolist()} != DP + e {want.tolist()}")
    rng = np.random.default_rng(seed)
    for _ in range(n_cases):
        nA, nB = int(rng.integers(1, 9)), int(rng.integers(1, 9))
        dim = int(rng.integers(1, 4))
        p = float(rng.choice([1.0, 2.0, 3.0]))
        nu = float(rng.choice([0.0, 0.05, 1.0]))
        A, TA = rand_series(rng, nA, dim)
        B, TB = rand_series(rng, nB, dim)
        DP, X = orc.matrix_x(A, TA, B, TB, nu, 0.5, p)
        _, _, _, _, _, e = _steps(A, TA, B, TB, nu, 0.5, p)
        for i in range(nA + 1):
            for j in range(nB + 1):
                w = DP[i, j] + e(i, j)
                if not (X[i, j] == w or abs(X[i, j] - w) <= 1e-13 * abs(w)):
                    fails.append(f"X[{i},{j}] {X[i, j]!r} vs DP + e {w!r}")
    return fails


def check_paths(orc, n_cases=80, seed=19, max_n=6):
    """Hand-worked paths, then the tie rule on integer data against the
    brute force (every path sum is exact, so ties are real ties)."""
    fails = []
    for c in load_worked_examples():
        if "path" not in c:
            continue
        A = np.array(c["A"], float).reshape(-1, c["dim"])
        B = np.array(c["B"], float).reshape(-1, c["dim"])
        P = orc.path(A, c["TA"], B, c["TB"], c["nu"], c["lambda"], c["p"])
        if P.tolist() != c["path"]:
            fails.append(f"{c['name']}: path {P.tolist()} != {c['path']}")
    rng = np.random.default_rng(seed)
    ties = 0
    for _ in range(n_cases):
        nA, nB = int(rng.integers(1, max_n + 1)), int(rng.integers(1, max_n + 1))
        A = rng.integers(-3, 4, (nA, 1)).astype(float)
        B = rng.integers(-3, 4, (nB, 1)).astype(float)
        TA = np.cumsum(rng.integers(0, 3, nA)).astype(float)
        TB = np.cumsum(rng.integers(0, 3, nB)).astype(float)
        nu = float(rng.choice([0.0, 1.0, 2.0]))
        lam = float(rng.choice([0.0, 1.0, 3.0]))
        cost, cells, n_opt = tie_rule_path(A, TA, B, TB, nu, lam, 1.0)
        ties += n_opt > 1
        # the cost of every admissible path against the brute force's sum
        for c_bf, mv in brute_force_paths(A, TA, B, TB, nu, lam, 1.0)[:40]:
            pc = orc.path_cost(A, TA, B, TB, nu, lam, 1.0, cells_of(mv))
            if pc != c_bf:
                fails.append(f"path cost {pc!r} vs brute force {c_bf!r}")
                break
        try:
            P = orc.path(A, TA, B, TB, nu, lam, 1.0)
        except ValueError:
            fails.append(f"path {nA}x{nB}: no path")
            continue
        if [tuple(r) for r in P.tolist()] != cells:
            fails.append(f"path {nA}x{nB} nu{nu} lam{lam}: {P.tolist()} vs tie rule {cells}")
        if orc.twed(A, TA, B, TB, nu, lam, 1.0) != cost:
            fails.append(f"path {nA}x{nB}: value vs brute force {cost}")
    # real-valued data: the optimal path's cost is the distance, bit for bit
    # (the DP sums the same steps in the same order); a non-path is rejected
    for _ in range(15):
        nA, nB = int(rng.integers(1, 30)), int(rng.integers(1, 30))
        A, TA = rand_series(rng, nA, 2)
        B, TB = rand_series(rng, nB, 2)
        P = orc.path(A, TA, B, TB, 0.3, 0.7, 2.0)
        if orc.path_cost(A, TA, B, TB, 0.3, 0.7, 2.0, P) != orc.twed(A, TA, B, TB, 0.3, 0.7, 2.0):
            fails.append(f"path cost of the optimal path differs from the distance ({nA}x{nB})")
        bad = P.copy()
        bad[-1] = (nA + 1, nB)
        if not math.isnan(orc.path_cost(A, TA, B, TB, 0.3, 0.7, 2.0, bad)):
            fails.append("an inadmissible path was given a cost")
    if ties < 10:
        fails.append(f"only {ties} cases with tied optimal paths: the tie rule is not exercised")
    return fails


ALL_CHECKS = [check_worked_examples, check_brute_force, check_closed_form_single,
              check_metric_axioms, check_large_lambda, check_homogeneity,
              check_p_free_1d, check_prefix, check_band_state, check_paths]

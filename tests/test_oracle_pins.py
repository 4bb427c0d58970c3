"""The CPU oracle against its pins (no GPU).  See oracle_pins.py for the list."""
import os

import numpy as np
import pytest

import oracle
import oracle_pins as pins


@pytest.fixture(scope="module")
def orc():
    return oracle.get()


@pytest.mark.parametrize("check", pins.ALL_CHECKS, ids=lambda f: f.__name__)
def test_pin(orc, check):
    fails = check(orc)
    assert not fails, "\n".join(fails[:10])


def test_path_count_is_delannoy():
    # the admissible paths of the brute force are exactly the Delannoy paths
    # between (1,1) and (nA,nB)
    for nA in range(1, 6):
        for nB in range(1, 6):
            assert pins.count_paths(nA, nB) == pins.delannoy(nA - 1, nB - 1)
    assert pins.count_paths(3, 3) == 13
    assert pins.count_paths(7, 7) == 8989


def test_brute_force_7x7(orc):
    rng = np.random.default_rng(99)
    A, TA = pins.rand_series(rng, 7, 2)
    B, TB = pins.rand_series(rng, 7, 2)
    v = orc.twed(A, TA, B, TB, 0.4, 0.6, 2.0)
    bf = pins.brute_force(A, TA, B, TB, 0.4, 0.6, 2.0)
    assert abs(v - bf) <= 1e-12 * bf


def test_rows_equal_matrix(orc):
    rng = np.random.default_rng(5)
    for _ in range(10):
        dim = int(rng.integers(1, 5))
        A, TA = pins.rand_series(rng, int(rng.integers(1, 80)), dim)
        B, TB = pins.rand_series(rng, int(rng.integers(1, 80)), dim)
        for p in (1.0, 2.0, 2.5):
            assert orc.twed(A, TA, B, TB, 0.1, 1.0, p) == orc.twed(A, TA, B, TB, 0.1, 1.0, p, rows=True)


def test_pairs_equal_single_calls(orc):
    from paper_2007_16135_amd import synth
    col = synth.batch_collection(12, 5, 40, seed=7)
    prs = np.array([(i, j) for i in range(12) for j in range(12)], dtype=np.int64)
    D = orc.pairs(col.X, col.T, col.off, col.X, col.T, col.off, prs, 1e-3, 1.0, 1.0, threads=3)
    for k, (i, j) in enumerate(prs):
        xa, ta = col.series(i)
        xb, tb = col.series(j)
        assert D[k] == orc.twed(xa, ta, xb, tb, 1e-3, 1.0, 1.0)
    M = orc.all_pairs(col.X, col.T, col.off, 1e-3, 1.0, 1.0, threads=2)
    assert np.array_equal(M, M.T) and np.all(np.diag(M) == 0)
    assert np.array_equal(M.reshape(-1), np.where(prs[:, 0] == prs[:, 1], 0.0, D))


def test_reference_walk_value(orc):
    # 1-D walks n=1000 (seeds 0/1), nu=1e-3, lambda=1, L1.  The value is not
    # printed anywhere in the paper; this only guards the generator+oracle
    # pairing against silent drift.
    from paper_2007_16135_amd import synth
    c = synth.single_pair_1d(1000)
    v = orc.twed(c.A, c.TA, c.B, c.TB, c.nu, c.lam, c.p)
    assert v == 2826.5990263257186


@pytest.mark.parametrize("mutant", range(1, 9))
def test_planted_mistake_is_caught(tmp_path, mutant):
    """Each planted mistake in the oracle (dropped term, wrong index, missing
    root, misplaced penalty, missing stiffness, wrong pad, swapped costs,
    wrong boundary) fails at least one pin."""
    path = oracle.build(str(tmp_path / f"liboracle_m{mutant}.so"), mutant=mutant)
    bad = oracle.Oracle(path)
    assert bad.mutant == mutant
    caught = []
    for check in pins.ALL_CHECKS:
        try:
            fails = check(bad)
        except Exception as e:  # a crash also counts as detection
            fails = [repr(e)]
        if fails:
            caught.append(check.__name__)
    assert caught, f"mutant {mutant} passed every pin"

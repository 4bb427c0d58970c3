"""Plain FP64 CPU oracle for Time Warp Edit Distance.

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and
by the CPU-baseline leg of the benchmark, never by the product path.  It shares
no code with the HIP library and imports nothing from it.

The TWED oracle is ``twed_oracle.c`` (see its header for the definition it
writes out, section "Time Warp Edit Distance" of the paper with Marteau's cost
terms); this module builds it with gcc and exposes numpy-friendly wrappers.
The CNN oracle used by the learned k-NN part lives in ``oracle/cnn.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "twed_oracle.c")
_LIB = os.path.join(_HERE, "libtwed_oracle.so")

_dbl_p = ctypes.POINTER(ctypes.c_double)
_i64_p = ctypes.POINTER(ctypes.c_int64)


def build(out_path: str = _LIB, mutant: int = 0) -> str:
    """Compile the oracle with gcc (-O2, no FP contraction). Returns the path."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-std=c11",
           f"-DORACLE_MUTANT={int(mutant)}", "-o", out_path, _SRC, "-lm", "-lpthread"]
    subprocess.run(cmd, check=True)
    return out_path


def _needs_build(path: str) -> bool:
    return (not os.path.exists(path)) or os.path.getmtime(path) < os.path.getmtime(_SRC)


class Oracle:
    """ctypes view of one build of the oracle library."""

    def __init__(self, path: str):
        lib = ctypes.CDLL(path)
        lib.twed_oracle_matrix.restype = ctypes.c_double
        lib.twed_oracle_matrix.argtypes = [_dbl_p, _dbl_p, ctypes.c_int64, _dbl_p, _dbl_p,
                                           ctypes.c_int64, ctypes.c_int32, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_double, _dbl_p]
        lib.twed_oracle_rows.restype = ctypes.c_double
        lib.twed_oracle_rows.argtypes = lib.twed_oracle_matrix.argtypes[:-1]
        lib.twed_oracle_pairs.restype = None
        lib.twed_oracle_pairs.argtypes = [_dbl_p, _dbl_p, _i64_p, _dbl_p, _dbl_p, _i64_p,
                                          _i64_p, ctypes.c_int64, ctypes.c_int32,
                                          ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                          _dbl_p, ctypes.c_int32]
        lib.twed_oracle_matrix_x.restype = ctypes.c_double
        lib.twed_oracle_matrix_x.argtypes = lib.twed_oracle_matrix.argtypes + [_dbl_p]
        lib.twed_oracle_path.restype = ctypes.c_int64
        lib.twed_oracle_path.argtypes = lib.twed_oracle_matrix.argtypes[:-1] + [_i64_p]
        lib.twed_oracle_path_cost.restype = ctypes.c_double
        lib.twed_oracle_path_cost.argtypes = lib.twed_oracle_matrix.argtypes[:-1] + [_i64_p, ctypes.c_int64]
        lib.twed_oracle_dtw.restype = ctypes.c_double
        lib.twed_oracle_dtw.argtypes = [_dbl_p, ctypes.c_int64, _dbl_p, ctypes.c_int64, ctypes.c_int32,
                                        ctypes.c_double]
        for f in (lib.twed_oracle_edit, lib.twed_oracle_lcs):
            f.restype = ctypes.c_int64
            f.argtypes = [_dbl_p, ctypes.c_int64, _dbl_p, ctypes.c_int64]
        lib.twed_oracle_mutant.restype = ctypes.c_int32
        self.lib = lib
        self.mutant = lib.twed_oracle_mutant()

    @staticmethod
    def _pts(x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        if x.ndim == 1:
            x = x[:, None]
        return np.ascontiguousarray(x)

    @staticmethod
    def _vec(t):
        return np.ascontiguousarray(t, dtype=np.float64).reshape(-1)

    def twed(self, A, TA, B, TB, nu, lam, p=1.0, matrix=False, rows=False):
        """TWED of one pair.  A: (nA, dim) or (nA,), TA: (nA,).  FP64.

        matrix=True returns (value, DP) with DP of shape (nA+1, nB+1).
        rows=True uses the two-row form (same cells, same arithmetic).
        """
        A, B = self._pts(A), self._pts(B)
        TA, TB = self._vec(TA), self._vec(TB)
        nA, dim = A.shape
        nB = B.shape[0]
        if B.shape[1] != dim or TA.shape[0] != nA or TB.shape[0] != nB:
            raise ValueError("shape mismatch")
        args = (A.ctypes.data_as(_dbl_p), TA.ctypes.data_as(_dbl_p), nA,
                B.ctypes.data_as(_dbl_p), TB.ctypes.data_as(_dbl_p), nB, dim,
                float(nu), float(lam), float(p))
        if rows:
            return self.lib.twed_oracle_rows(*args)
        if matrix:
            DP = np.empty((nA + 1, nB + 1), dtype=np.float64)
            v = self.lib.twed_oracle_matrix(*args, DP.ctypes.data_as(_dbl_p))
            return v, DP
        return self.lib.twed_oracle_matrix(*args, None)

    def _args(self, A, TA, B, TB, nu, lam, p):
        A, B = self._pts(A), self._pts(B)
        TA, TB = self._vec(TA), self._vec(TB)
        nA, dim = A.shape
        nB = B.shape[0]
        if B.shape[1] != dim or TA.shape[0] != nA or TB.shape[0] != nB:
            raise ValueError("shape mismatch")
        keep = (A, TA, B, TB)
        return keep, (A.ctypes.data_as(_dbl_p), TA.ctypes.data_as(_dbl_p), nA,
                      B.ctypes.data_as(_dbl_p), TB.ctypes.data_as(_dbl_p), nB, dim,
                      float(nu), float(lam), float(p))

    def matrix_x(self, A, TA, B, TB, nu, lam, p=1.0):
        """(DP, X): the full DP matrix and X = DP + e, both (nA+1, nB+1)."""
        keep, args = self._args(A, TA, B, TB, nu, lam, p)
        nA, nB = args[2], args[5]
        DP = np.empty((nA + 1, nB + 1), dtype=np.float64)
        X = np.empty_like(DP)
        self.lib.twed_oracle_matrix_x(*args, DP.ctypes.data_as(_dbl_p), X.ctypes.data_as(_dbl_p))
        return DP, X

    def path(self, A, TA, B, TB, nu, lam, p=1.0):
        """One optimal alignment path as an (L, 2) int64 array of cells (i, j)
        from (0, 0) to (nA, nB); ties prefer the match, then the deletion in
        A, then the deletion in B."""
        keep, args = self._args(A, TA, B, TB, nu, lam, p)
        nA, nB = args[2], args[5]
        P = np.empty((nA + nB + 1, 2), dtype=np.int64)
        n = self.lib.twed_oracle_path(*args, P.ctypes.data_as(_i64_p))
        if n < 0:
            raise ValueError("no finite path")
        return P[:n].copy()

    def path_cost(self, A, TA, B, TB, nu, lam, p, path):
        """Summed step costs of a path ((L, 2) cells from (0, 0) to (nA, nB));
        NaN if it is not an admissible path."""
        keep, args = self._args(A, TA, B, TB, nu, lam, p)
        P = np.ascontiguousarray(np.asarray(path, dtype=np.int64).reshape(-1, 2))
        return self.lib.twed_oracle_path_cost(*args, P.ctypes.data_as(_i64_p), P.shape[0])

    def dtw(self, A, B, p=1.0):
        """Dynamic time warping distance with the Lp point distance."""
        A, B = self._pts(A), self._pts(B)
        if A.shape[1] != B.shape[1]:
            raise ValueError("shape mismatch")
        return self.lib.twed_oracle_dtw(A.ctypes.data_as(_dbl_p), A.shape[0], B.ctypes.data_as(_dbl_p),
                                        B.shape[0], A.shape[1], float(p))

    def edit(self, A, B):
        """Levenshtein distance between two 1-D sequences of tokens."""
        A, B = self._vec(A), self._vec(B)
        return int(self.lib.twed_oracle_edit(A.ctypes.data_as(_dbl_p), len(A), B.ctypes.data_as(_dbl_p), len(B)))

    def lcs(self, A, B):
        """Length of a longest common subsequence of two 1-D token sequences."""
        A, B = self._vec(A), self._vec(B)
        return int(self.lib.twed_oracle_lcs(A.ctypes.data_as(_dbl_p), len(A), B.ctypes.data_as(_dbl_p), len(B)))

    def pairs(self, X, TX, offX, Y, TY, offY, pairs, nu, lam, p=1.0, threads=None):
        """TWED for explicit (i, j) pairs of two packed collections (CSR offsets)."""
        X, Y = self._pts(X), self._pts(Y)
        TX, TY = self._vec(TX), self._vec(TY)
        offX = np.ascontiguousarray(offX, dtype=np.int64)
        offY = np.ascontiguousarray(offY, dtype=np.int64)
        pairs = np.ascontiguousarray(pairs, dtype=np.int64).reshape(-1, 2)
        D = np.empty(pairs.shape[0], dtype=np.float64)
        if threads is None:
            threads = os.cpu_count() or 1
        self.lib.twed_oracle_pairs(X.ctypes.data_as(_dbl_p), TX.ctypes.data_as(_dbl_p),
                                   offX.ctypes.data_as(_i64_p), Y.ctypes.data_as(_dbl_p),
                                   TY.ctypes.data_as(_dbl_p), offY.ctypes.data_as(_i64_p),
                                   pairs.ctypes.data_as(_i64_p), pairs.shape[0], X.shape[1],
                                   float(nu), float(lam), float(p),
                                   D.ctypes.data_as(_dbl_p), int(threads))
        return D

    def all_pairs(self, X, TX, offX, nu, lam, p=1.0, threads=None):
        """Symmetric all-pairs matrix of one packed collection (upper triangle
        computed, mirrored, zero diagonal)."""
        n = len(offX) - 1
        iu = np.triu_indices(n, 1)
        prs = np.stack(iu, axis=1)
        d = self.pairs(X, TX, offX, X, TX, offX, prs, nu, lam, p, threads)
        D = np.zeros((n, n), dtype=np.float64)
        D[iu] = d
        D[(iu[1], iu[0])] = d
        return D


_default = None


def get() -> Oracle:
    """The normal (unmutated) oracle, built on first use if needed."""
    global _default
    if _default is None:
        if _needs_build(_LIB):
            build(_LIB)
        _default = Oracle(_LIB)
    return _default


def twed(*a, **k):
    return get().twed(*a, **k)

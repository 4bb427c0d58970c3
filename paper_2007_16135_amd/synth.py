"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds only input generation (NumPy PCG64 streams): no part of the
distance computation.  Both the HIP path and the CPU oracle consume what it
produces.

Series follow the shape of the paper's workloads (section "Performance":
random single pairs of growing length, all-pairs batches of short series, a
long-series batch, and one query against a large collection), with synthetic
values in place of the public datasets the paper used:

* ``walk(rng, n, dim)``   Gaussian random walk, x_0 is the first N(0,1) step.
* irregular timestamps    cumulative Exp(1) gaps, drawn after the values from
                          the same generator (so t_0 > 0).
* regular timestamps      0, 1, ..., n-1.
* FP32 inputs             generated in FP64 and rounded once.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np


def walk(rng: np.random.Generator, n: int, dim: int) -> np.ndarray:
    return rng.standard_normal((n, dim)).cumsum(axis=0)


def irregular_times(rng: np.random.Generator, n: int) -> np.ndarray:
    return rng.exponential(1.0, n).cumsum()


def regular_times(n: int) -> np.ndarray:
    return np.arange(n, dtype=np.float64)


@dataclass
class PairCase:
    """One pair of series with its parameters (values (n, dim), times (n,))."""
    name: str
    A: np.ndarray
    TA: np.ndarray
    B: np.ndarray
    TB: np.ndarray
    nu: float
    lam: float
    p: float

    @property
    def dim(self) -> int:
        return self.A.shape[1]

    def astype(self, dtype) -> "PairCase":
        return PairCase(self.name, self.A.astype(dtype), self.TA.astype(dtype),
                        self.B.astype(dtype), self.TB.astype(dtype), self.nu, self.lam, self.p)

    def prefix(self, n: int) -> "PairCase":
        return PairCase(f"{self.name}[:{n}]", self.A[:n], self.TA[:n], self.B[:n], self.TB[:n],
                        self.nu, self.lam, self.p)


def random_pair(seed_a: int, seed_b: int, nA: int, nB: int, dim: int, *, irregular: bool,
                nu: float, lam: float, p: float, name: str = "pair") -> PairCase:
    ra, rb = np.random.default_rng(seed_a), np.random.default_rng(seed_b)
    A, B = walk(ra, nA, dim), walk(rb, nB, dim)
    if irregular:
        TA, TB = irregular_times(ra, nA), irregular_times(rb, nB)
    else:
        TA, TB = regular_times(nA), regular_times(nB)
    return PairCase(name, A, TA, B, TB, nu, lam, p)


def single_pair_1d(n: int = 1000) -> PairCase:
    """1-D Gaussian walks, seeds 0/1, timestamps 0..n-1, nu=1e-3, lambda=1, L1."""
    return random_pair(0, 1, n, n, 1, irregular=False, nu=1e-3, lam=1.0, p=1.0,
                       name=f"walk1d_n{n}")


def single_pair_3d(n: int = 100_000) -> PairCase:
    """3-D walks, seeds 2/3, irregular Exp(1) timestamps, nu=0.01, lambda=0.5, L2."""
    return random_pair(2, 3, n, n, 3, irregular=True, nu=0.01, lam=0.5, p=2.0,
                       name=f"walk3d_n{n}")


def single_pair_8d(n: int = 1_000_000) -> PairCase:
    """8-D walks, seeds 4/5, regular timestamps, nu=1e-3, lambda=1, L2."""
    return random_pair(4, 5, n, n, 8, irregular=False, nu=1e-3, lam=1.0, p=2.0,
                       name=f"walk8d_n{n}")


@dataclass
class Collection:
    """Packed ragged collection: values (sum n, dim), times (sum n,), CSR offsets."""
    X: np.ndarray
    T: np.ndarray
    off: np.ndarray
    labels: np.ndarray = field(default=None)

    @property
    def count(self) -> int:
        return len(self.off) - 1

    @property
    def lengths(self) -> np.ndarray:
        return np.diff(self.off)

    def series(self, k: int):
        a, b = self.off[k], self.off[k + 1]
        return self.X[a:b], self.T[a:b]

    def astype(self, dtype) -> "Collection":
        return Collection(self.X.astype(dtype), self.T.astype(dtype), self.off.copy(), self.labels)

    def subset(self, idx) -> "Collection":
        parts_x, parts_t, off = [], [], [0]
        for k in idx:
            x, t = self.series(int(k))
            parts_x.append(x)
            parts_t.append(t)
            off.append(off[-1] + len(t))
        lab = None if self.labels is None else self.labels[np.asarray(idx)]
        return Collection(np.concatenate(parts_x), np.concatenate(parts_t),
                          np.asarray(off, dtype=np.int64), lab)


def pack(series_x, series_t, labels=None) -> Collection:
    off = np.zeros(len(series_x) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(t) for t in series_t])
    X = np.concatenate([np.asarray(x).reshape(len(x), -1) for x in series_x])
    T = np.concatenate(series_t)
    return Collection(X, T, off, None if labels is None else np.asarray(labels))


def batch_collection(count: int = 2048, lo: int = 64, hi: int = 1024, seed: int = 2048) -> Collection:
    """1-D walks with irregular Exp(1) timestamps, lengths uniform in [lo, hi].

    Lengths come from default_rng(seed); series k from default_rng([seed, k]).
    Used with nu=1e-3, lambda=1, L1.
    """
    lengths = np.random.default_rng(seed).integers(lo, hi + 1, count)
    xs, ts = [], []
    for k, L in enumerate(lengths):
        r = np.random.default_rng([seed, k])
        xs.append(walk(r, int(L), 1))
        ts.append(irregular_times(r, int(L)))
    return pack(xs, ts)


def paper_shaped_collection(count: int, length: int, seed: int = 600) -> Collection:
    """Equal-length 1-D walks with regular timestamps (all-pairs shapes of the
    paper's validation table: 600 x 60 and 10 x 100k)."""
    xs, ts = [], []
    for k in range(count):
        r = np.random.default_rng([seed, k])
        xs.append(walk(r, length, 1))
        ts.append(regular_times(length))
    return pack(xs, ts)


def paper_shaped_rn(count: int = 60000, length: int = 28, dim: int = 28, seed: int = 28) -> Collection:
    """Series of `length` samples in R^dim with regular timestamps -- the
    shape of the paper's R^N timing (one query against 60,000 series of 28
    steps in R^28), with seeded Gaussian random walks standing in for the
    images (series k from default_rng([seed, k]))."""
    xs, ts = [], []
    for k in range(count):
        r = np.random.default_rng([seed, k])
        xs.append(walk(r, length, dim))
        ts.append(regular_times(length))
    return pack(xs, ts)


# ---- learned k-NN workload ---------------------------------------------------

N_CLASSES = 8


def sinusoid_classes(seed: int = 8):
    """Per-class (amplitude, angular frequency, phase, offset), drawn once."""
    r = np.random.default_rng(seed)
    a = r.uniform(0.5, 3.0, N_CLASSES)
    w = r.uniform(0.02, 0.3, N_CLASSES)
    ph = r.uniform(0.0, 2 * np.pi, N_CLASSES)
    b = r.uniform(-2.0, 2.0, N_CLASSES)
    return a, w, ph, b


def knn_series(seed_base: int, k: int, classes, lo: int = 128, hi: int = 512, sigma: float = 0.3):
    """Series k of a k-NN collection: even k a 1-D random walk, odd k a noisy
    sinusoid of class (k // 2) % 8.  Returns (values (L,1), times (L,), label);
    label -1 marks a walk."""
    r = np.random.default_rng([seed_base, k])
    L = int(r.integers(lo, hi + 1))
    t = regular_times(L)
    if k % 2 == 0:
        return walk(r, L, 1), t, -1
    c = (k // 2) % N_CLASSES
    a, w, ph, b = classes
    x = b[c] + a[c] * np.sin(w[c] * t + ph[c]) + r.normal(0.0, sigma, L)
    return x.reshape(L, 1), t, c


def knn_collection(count: int, seed_base: int, class_seed: int = 8) -> Collection:
    """Database (seed_base=3) or queries (seed_base=4) for the k-NN workload:
    lengths uniform in [128, 512], half random walks, half noisy sinusoids of
    8 seeded classes; regular timestamps.  Used with nu=1e-3, lambda=1, L1."""
    classes = sinusoid_classes(class_seed)
    xs, ts, ls = [], [], []
    for k in range(count):
        x, t, lab = knn_series(seed_base, k, classes)
        xs.append(x)
        ts.append(t)
        ls.append(lab)
    return pack(xs, ts, ls)

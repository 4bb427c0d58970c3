"""Training loop of the k-NN embedding network (host orchestration only).

Every numeric step runs in libtwed: the TWED labels come from the batched
sweep in pair-list mode (twed_batch), the loss and gradients from
twed_embed_loss_grad, the update from twed_embed_adamw, and mined
neighbours from the exhaustive search of the index (twed_knn).  This module only chooses
which series and pairs go into each step; PyTorch gathers the chosen series
into one packed device buffer.

Pair sampling (two kinds per step, both labelled with their exact TWED):
  random  pairs of series drawn uniformly from the database;
  mined   an anchor and some of its exact nearest database series, found
          once before training by the exhaustive k-NN of the index -- these
          teach the fine ordering that a k-NN query depends on.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import binding as B
from .binding import EMBED_DIM

CHANNELS = (2, 64, 64, 64, 4)
KSIZE = 5


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights, zero biases, as the flat float32 parameter vector
    (per layer W (5, C_in, C_out) row-major, then b)."""
    rng = np.random.default_rng(seed)
    parts = []
    for l in range(4):
        cin, cout = CHANNELS[l], CHANNELS[l + 1]
        parts.append(rng.standard_normal(KSIZE * cin * cout) * np.sqrt(2.0 / (KSIZE * cin)))
        parts.append(np.zeros(cout))
    return np.concatenate(parts).astype(np.float32)


class Collection:
    """A packed 1-D FP32 collection resident on the device."""

    def __init__(self, X, T, off):
        self.X, self.T = X, T
        self.off = np.ascontiguousarray(np.asarray(off, dtype=np.int64))
        self.n = len(self.off) - 1
        self.lengths = np.diff(self.off)

    def gather(self, idx):
        """The series `idx` packed into a new device collection."""
        import torch
        idx = np.asarray(idx, dtype=np.int64)
        lens = self.lengths[idx]
        off = np.zeros(len(idx) + 1, dtype=np.int64)
        off[1:] = np.cumsum(lens)
        starts = np.repeat(self.off[idx] - off[:-1], lens)
        rows = torch.as_tensor(starts + np.arange(off[-1], dtype=np.int64), device=self.X.device)
        return Collection(self.X.index_select(0, rows), self.T.index_select(0, rows), off)


class Trainer:
    def __init__(self, db: Collection, nu=1e-3, lam=1.0, seed=0, lr=2e-3, weight_decay=1e-4,
                 batch_series=256, pairs_per_step=2048, mined_fraction=0.5, n_anchors=1024, pool=20,
                 per_anchor=10, params=None):
        import torch
        self.torch = torch
        self.db, self.nu, self.lam = db, nu, lam
        self.rng = np.random.default_rng(seed)
        dev = db.X.device
        p = init_params(seed) if params is None else np.asarray(params, dtype=np.float32)
        self.params = torch.as_tensor(p, device=dev)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.empty_like(self.params)
        self.loss = torch.empty(1, dtype=torch.float32, device=dev)
        self.lr, self.wd = lr, weight_decay
        self.S, self.P = batch_series, pairs_per_step
        self.mined_fraction, self.per_anchor = mined_fraction, per_anchor
        self.step_count = 0
        self.pairs_seen = 0
        self.history = []
        self.mine_s = 0.0
        self.neigh = self._mine(min(db.n, n_anchors), min(pool, db.n - 1)) if mined_fraction > 0 else None

    # -- pair sampling --------------------------------------------------------------

    def _mine(self, n_anchors, pool):
        """Exact nearest database series of random anchors: the exhaustive
        k-NN of the index (every database series re-ranked, n_cand = n)."""
        torch = self.torch
        t0 = time.perf_counter()
        n = self.db.n
        anchors = self.rng.choice(n, size=n_anchors, replace=False)
        q = self.db.gather(anchors)
        index = B.KnnIndex(self.db.X, self.db.T, self.db.off, self.params, self.nu, self.lam)
        ids, _ = index.query(q.X, q.T, q.off, k=pool + 1, n_cand=n)
        ids = ids.cpu().numpy()
        index.close()
        nb = np.array([[j for j in row if j != a][:pool] for a, row in zip(anchors, ids)], dtype=np.int64)
        self.mine_s = time.perf_counter() - t0
        self.pairs_seen += n_anchors * n
        return anchors, nb

    def _sample(self):
        """Series of this step and (local) pairs among them: groups of an
        anchor and some of its exact neighbours (anchor-neighbour pairs),
        then random series and random pairs."""
        n, S, P = self.db.n, self.S, self.P
        series, pairs = [], []
        if self.neigh is not None:
            anchors, nb = self.neigh
            per = min(self.per_anchor, nb.shape[1])
            groups = min(len(anchors), int(S * self.mined_fraction) // (per + 1))
            for r in self.rng.choice(len(anchors), size=groups, replace=False):
                base = len(series)
                series.append(int(anchors[r]))
                series += [int(j) for j in nb[r][self.rng.choice(nb.shape[1], per, replace=False)]]
                pairs += [(base, base + j) for j in range(1, per + 1)]
        rest = S - len(series)
        if rest > 0:
            series += [int(i) for i in self.rng.choice(n, size=rest, replace=False)]
        m = P - len(pairs)
        a = self.rng.integers(0, len(series), m)
        b = self.rng.integers(0, len(series) - 1, m)
        b = b + (b >= a)
        pairs += list(zip(a.tolist(), b.tolist()))
        return np.array(series, dtype=np.int64), np.asarray(pairs, dtype=np.int64)

    # -- one optimisation step ----------------------------------------------------

    def step(self, lr=None):
        torch = self.torch
        series, pairs = self._sample()
        batch = self.db.gather(series)
        dev = batch.X.device
        p64 = torch.as_tensor(pairs, device=dev)
        target = B.twed_batch(batch.X, batch.T, batch.off, batch.X, batch.T, batch.off, pairs=p64,
                              nu=self.nu, lam=self.lam, p=1.0, precision="f32")
        p32 = p64.to(torch.int32).contiguous()
        B.twed_embed_loss_grad(self.params, batch.X, batch.off, p32, target, grad=self.grad, loss=self.loss)
        self.step_count += 1
        B.twed_embed_adamw(self.params, self.m, self.v, self.grad, self.step_count, self.lr if lr is None else lr,
                           self.wd)
        self.pairs_seen += len(pairs)
        return self.loss

    def train(self, steps, log_every=0, log=None, schedule="cosine", lr_floor=0.02):
        """`steps` optimisation steps.  schedule "cosine": the learning rate
        falls from lr to lr * lr_floor along a half cosine over the steps;
        "constant": lr throughout."""
        t0 = time.perf_counter()
        for i in range(steps):
            lr = self.lr
            if schedule == "cosine" and steps > 1:
                lr = self.lr * (lr_floor + (1.0 - lr_floor) * 0.5 * (1.0 + math.cos(math.pi * i / (steps - 1))))
            loss = self.step(lr)
            if log_every and (i + 1) % log_every == 0:
                v = float(loss.item())
                self.history.append((self.step_count, v))
                if log:
                    log(f"train step {self.step_count}: loss {v:.4f} ({time.perf_counter() - t0:.1f} s)")
        self.torch.cuda.synchronize()
        return time.perf_counter() - t0


def recall_at(ids, truth):
    """Mean |ids_q intersect truth_q| / k over the queries."""
    ids = np.asarray(ids)
    truth = np.asarray(truth)
    k = truth.shape[1]
    return float(np.mean([len(set(a[:k].tolist()) & set(b.tolist())) / k for a, b in zip(ids, truth)]))


def exact_knn_from_matrix(D, k):
    """Top-k ids per row of a distance matrix by (distance, id)."""
    D = np.asarray(D)
    idx = np.argsort(D, axis=1, kind="stable")[:, :k]
    return idx

"""Training loop of the k-NN embedding network (host orchestration only).

Every numeric step runs in libtwed: the TWED labels come from the batched
sweep in pair-list mode (twed_batch), the loss and gradients from
twed_embed_loss_grad, the update from twed_embed_adamw, and mined
neighbours from the index itself (twed_knn).  This module only chooses
which series and pairs go into each step; PyTorch gathers the chosen series
into one packed device buffer.

Pair sampling (two kinds per step, both labelled with their exact TWED):
  random  pairs of series drawn uniformly from the database;
  mined   an anchor and its nearest database series under the current
          index (exact TWED among the network's candidates), refreshed
          every `refresh` steps -- these teach the fine ordering that a
          k-NN query depends on.
"""
from __future__ import annotations

import time

import numpy as np

from . import binding as B
from .binding import EMBED_DIM

CHANNELS = (2, 64, 64, 64, 32)
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
                 batch_series=256, pairs_per_step=2048, mined_fraction=0.5, mined_k=8, refresh=100,
                 params=None):
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
        self.mined_fraction, self.mined_k, self.refresh = mined_fraction, mined_k, refresh
        self.step_count = 0
        self.pairs_seen = 0
        self.neigh = None  # (anchors, neighbour ids) mined from the current index
        self.history = []

    # -- pair sampling --------------------------------------------------------------

    def _mine(self):
        """Nearest database series of a random anchor set under the current
        network (exact TWED among its candidates)."""
        torch = self.torch
        n = self.db.n
        anchors = self.rng.choice(n, size=min(n, 4096), replace=False)
        q = self.db.gather(anchors)
        index = B.KnnIndex(self.db.X, self.db.T, self.db.off, self.params, self.nu, self.lam)
        k = min(self.mined_k + 1, n)
        ids, _ = index.query(q.X, q.T, q.off, k=k, n_cand=min(n, max(4 * k, 64)))
        torch.cuda.synchronize()
        index.close()
        self.neigh = (anchors, ids.cpu().numpy())

    def _sample(self):
        """Series of this step and (local) pairs among them."""
        n, S, P = self.db.n, self.S, self.P
        n_mined = int(P * self.mined_fraction) if self.neigh is not None else 0
        chosen, pairs = [], []
        if n_mined:
            anchors, ids = self.neigh
            per = max(1, ids.shape[1] - 1)
            n_groups = max(1, min(S // (per + 1), n_mined // per))
            rows = self.rng.choice(len(anchors), size=n_groups, replace=False)
            for r in rows:
                group = [int(anchors[r])] + [int(i) for i in ids[r] if int(i) != int(anchors[r])][:per]
                chosen.append(group)
        flat = [i for g in chosen for i in g]
        rest = S - len(flat)
        if rest > 0:
            flat += [int(i) for i in self.rng.choice(n, size=rest, replace=False)]
        series = np.array(flat, dtype=np.int64)
        # mined pairs: anchor with each of its neighbours, and neighbours among themselves
        pos = 0
        for g in chosen:
            idx = list(range(pos, pos + len(g)))
            for a in range(len(idx)):
                for b in range(a + 1, len(idx)):
                    pairs.append((idx[a], idx[b]))
            pos += len(g)
        pairs = pairs[:n_mined] if n_mined else []
        m = P - len(pairs)
        a = self.rng.integers(0, len(series), m)
        b = self.rng.integers(0, len(series) - 1, m)
        b = b + (b >= a)
        pairs += list(zip(a.tolist(), b.tolist()))
        return series, np.asarray(pairs, dtype=np.int64)

    # -- one optimisation step ----------------------------------------------------

    def step(self):
        torch = self.torch
        if self.mined_fraction > 0 and self.step_count % self.refresh == 0 and self.step_count > 0:
            self._mine()
        series, pairs = self._sample()
        batch = self.db.gather(series)
        dev = batch.X.device
        p64 = torch.as_tensor(pairs, device=dev)
        target = B.twed_batch(batch.X, batch.T, batch.off, batch.X, batch.T, batch.off, pairs=p64,
                              nu=self.nu, lam=self.lam, p=1.0, precision="f32")
        p32 = p64.to(torch.int32).contiguous()
        B.twed_embed_loss_grad(self.params, batch.X, batch.off, p32, target, grad=self.grad, loss=self.loss)
        self.step_count += 1
        B.twed_embed_adamw(self.params, self.m, self.v, self.grad, self.step_count, self.lr, self.wd)
        self.pairs_seen += len(pairs)
        return self.loss

    def train(self, steps, log_every=0, log=None):
        t0 = time.perf_counter()
        for i in range(steps):
            loss = self.step()
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

"""Plain FP64 CPU reference of the k-NN embedding network.

TEST INFRASTRUCTURE ONLY: used by the test suite to check the HIP training and
inference kernels; it shares no code with them.

The network maps one series (values x_0..x_{L-1}, L <= T_MAX) to a 128-d
embedding whose Euclidean distances are trained to follow TWED:

  input features    f_t = (x_t / 8, L / 256)                        (2 channels)
  layer l = 1..4    y_t = b + sum_{k=0..4} W[k]^T h_{t+k-2}          (kernel 5,
                    h outside [0, L) is zero; y_t = 0 for t >= L      same padding)
                    ReLU after layers 1-3, none after layer 4
  channels          2 -> 64 -> 64 -> 64 -> 4
  pooling           segment s = 0..31 covers t in [floor(s L/32), floor((s+1) L/32));
                    e[4 s + c] = mean over the segment of layer-4 channel c
                    (0 for an empty segment, which happens when L < 32)
  pair loss         p = sqrt(|e_a - e_b|^2 + eps);
                    loss = (log(1 + p) - log(1 + d))^2, d the TWED of the pair

Everything below is written directly from these definitions with NumPy, in
FP64, one series at a time.
"""
from __future__ import annotations

import numpy as np

CHANNELS = (2, 64, 64, 64, 4)
KSIZE = 5
SEGMENTS = 32
EMB = SEGMENTS * CHANNELS[-1]
T_MAX = 512
X_SCALE = 1.0 / 8.0
L_SCALE = 1.0 / 256.0
EPS = 1e-6


def init_params(seed: int = 0):
    """He-normal weights and zero biases, NumPy PCG64.  Shapes: W[l] is
    (KSIZE, C_in, C_out), b[l] is (C_out,)."""
    rng = np.random.default_rng(seed)
    W, b = [], []
    for l in range(4):
        cin, cout = CHANNELS[l], CHANNELS[l + 1]
        std = np.sqrt(2.0 / (KSIZE * cin))
        W.append(rng.standard_normal((KSIZE, cin, cout)) * std)
        b.append(np.zeros(cout))
    return {"W": W, "b": b}


def features(x):
    x = np.asarray(x, dtype=np.float64).reshape(-1)
    L = len(x)
    return np.stack([x * X_SCALE, np.full(L, L * L_SCALE)], axis=1)


def conv(h, W, b):
    """Same-padded 1-D convolution over the series' own length."""
    L = h.shape[0]
    out = np.tile(b, (L, 1)).astype(np.float64)
    for k in range(KSIZE):
        shift = k - KSIZE // 2
        src = np.zeros_like(h)
        lo, hi = max(0, -shift), min(L, L - shift)
        if hi > lo:
            src[lo:hi] = h[lo + shift:hi + shift]
        out += src @ W[k]
    return out


def segments(L):
    return [((s * L) // SEGMENTS, ((s + 1) * L) // SEGMENTS) for s in range(SEGMENTS)]


def forward(params, x):
    """Embedding of one series; returns (e, cache)."""
    h = features(x)
    cache = {"inputs": [], "pre": []}
    for l in range(4):
        cache["inputs"].append(h)
        y = conv(h, params["W"][l], params["b"][l])
        cache["pre"].append(y)
        h = np.maximum(y, 0.0) if l < 3 else y
    L = h.shape[0]
    e = np.concatenate([h[a:c].mean(axis=0) if c > a else np.zeros(h.shape[1]) for (a, c) in segments(L)])
    cache["last"] = h
    return e, cache


def backward(params, cache, de):
    """Gradients of a scalar with d(scalar)/de = de, for one series."""
    h = cache["last"]
    L = h.shape[0]
    C = h.shape[1]
    dh = np.zeros_like(h)
    for s, (a, c) in enumerate(segments(L)):
        if c > a:
            dh[a:c] += de[s * C:(s + 1) * C] / (c - a)
    gW = [None] * 4
    gb = [None] * 4
    for l in reversed(range(4)):
        dy = dh if l == 3 else dh * (cache["pre"][l] > 0)
        hin = cache["inputs"][l]
        gb[l] = dy.sum(axis=0)
        gW[l] = np.zeros_like(params["W"][l])
        dhin = np.zeros_like(hin)
        for k in range(KSIZE):
            shift = k - KSIZE // 2
            lo, hi = max(0, -shift), min(L, L - shift)
            if hi > lo:
                # y[t] += h[t + shift] @ W[k] for t in [lo, hi)
                gW[l][k] += hin[lo + shift:hi + shift].T @ dy[lo:hi]
                dhin[lo + shift:hi + shift] += dy[lo:hi] @ params["W"][l][k].T
        dh = dhin
    return {"W": gW, "b": gb}


def pair_loss(ea, eb, d):
    """Loss of one pair and its gradients with respect to ea and eb."""
    diff = ea - eb
    p = np.sqrt(diff @ diff + EPS)
    r = np.log1p(p) - np.log1p(d)
    loss = r * r
    g = 2.0 * r / (1.0 + p) / p * diff
    return loss, g, -g


def batch_loss_and_grads(params, series, pairs, targets):
    """Mean pair loss over a batch and its parameter gradients (FP64)."""
    embs, caches = [], []
    for x in series:
        e, c = forward(params, x)
        embs.append(e)
        caches.append(c)
    de = [np.zeros(EMB) for _ in series]
    total = 0.0
    P = len(pairs)
    for (i, j), d in zip(pairs, targets):
        loss, ga, gb_ = pair_loss(embs[i], embs[j], d)
        total += loss
        de[i] += ga / P
        de[j] += gb_ / P
    gW = [np.zeros_like(w) for w in params["W"]]
    gbias = [np.zeros_like(b) for b in params["b"]]
    for c, g in zip(caches, de):
        if np.any(g):
            gr = backward(params, c, g)
            for l in range(4):
                gW[l] += gr["W"][l]
                gbias[l] += gr["b"][l]
    return total / P, {"W": gW, "b": gbias}, np.array(embs)


def embed(params, series):
    return np.array([forward(params, x)[0] for x in series])


def flatten(params):
    """Parameters as one vector in the order W1, b1, W2, b2, ... (W as
    (KSIZE, C_in, C_out) row-major)."""
    return np.concatenate([np.concatenate([params["W"][l].reshape(-1), params["b"][l]]) for l in range(4)])


def unflatten(vec):
    out = {"W": [], "b": []}
    pos = 0
    for l in range(4):
        cin, cout = CHANNELS[l], CHANNELS[l + 1]
        n = KSIZE * cin * cout
        out["W"].append(np.asarray(vec[pos:pos + n], dtype=np.float64).reshape(KSIZE, cin, cout))
        pos += n
        out["b"].append(np.asarray(vec[pos:pos + cout], dtype=np.float64))
        pos += cout
    return out


def n_params():
    return sum(KSIZE * CHANNELS[l] * CHANNELS[l + 1] + CHANNELS[l + 1] for l in range(4))


def adamw_step(w, m, v, g, step, lr, weight_decay, beta1=0.9, beta2=0.999, eps=1e-8):
    """One AdamW update (Adam with decoupled weight decay, Loshchilov and
    Hutter), FP64: moments m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2, bias
    corrections 1 - b^step, then w <- w - lr (m_hat / (sqrt(v_hat) + eps) + wd w).
    Returns new (w, m, v)."""
    w = np.asarray(w, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** step)
    v_hat = v / (1.0 - beta2 ** step)
    w = w - lr * (m_hat / (np.sqrt(v_hat) + eps) + weight_decay * w)
    return w, m, v

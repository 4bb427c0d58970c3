"""Pins for the CPU reference of the embedding network (no GPU).

The backward pass is pinned by central finite differences of the forward
pass; the convolution by delta kernels (a pure shift) and linearity; the
pooling by its segment definition; the loss by its minimum."""
import numpy as np
import pytest

from oracle import cnn


def rand_series(rng, L):
    return rng.standard_normal(L).cumsum()


def test_delta_kernel_is_a_shift():
    rng = np.random.default_rng(0)
    L, C = 37, 3
    h = rng.standard_normal((L, C))
    for k in range(cnn.KSIZE):
        W = np.zeros((cnn.KSIZE, C, C))
        W[k] = np.eye(C)
        y = cnn.conv(h, W, np.zeros(C))
        shift = k - cnn.KSIZE // 2
        want = np.zeros_like(h)
        for t in range(L):
            if 0 <= t + shift < L:
                want[t] = h[t + shift]
        assert np.array_equal(y, want)


def test_conv_is_linear_with_bias():
    rng = np.random.default_rng(1)
    h1, h2 = rng.standard_normal((20, 4)), rng.standard_normal((20, 4))
    W, b = rng.standard_normal((5, 4, 6)), rng.standard_normal(6)
    lhs = cnn.conv(2.0 * h1 + h2, W, b)
    rhs = 2.0 * cnn.conv(h1, W, b) + cnn.conv(h2, W, b) - 2.0 * b
    assert np.allclose(lhs, rhs, rtol=1e-12, atol=1e-12)


def test_pooling_segments():
    assert cnn.SEGMENTS == 32
    assert cnn.segments(64) == [(2 * s, 2 * s + 2) for s in range(32)]
    assert cnn.segments(65)[-1] == (62, 65) and cnn.segments(65)[0] == (0, 2)
    for L in (1, 5, 31, 32, 33, 100, 512):
        seg = cnn.segments(L)
        assert seg[0][0] == 0 and seg[-1][1] == L
        assert all(a[1] == b[0] for a, b in zip(seg, seg[1:]))         # contiguous, in order
        assert all(c - a in (L // 32, -(-L // 32)) for a, c in seg)    # floor or ceil of L/32
    # constant last layer -> every segment mean equals the constant
    p = cnn.init_params(3)
    for l in range(4):
        p["W"][l][:] = 0.0
    p["b"][3][:] = np.arange(cnn.CHANNELS[-1])
    e, _ = cnn.forward(p, np.ones(77))
    assert np.array_equal(e, np.tile(np.arange(cnn.CHANNELS[-1], dtype=float), cnn.SEGMENTS))


def test_loss_minimum():
    e = np.arange(cnn.EMB, dtype=float)
    d = 0.0
    loss, ga, gb = cnn.pair_loss(e, e, d)
    assert loss < 1e-6 and np.all(ga == 0) and np.all(gb == 0)


@pytest.mark.parametrize("seed", [0, 1])
def test_gradients_match_finite_differences(seed):
    rng = np.random.default_rng(seed)
    params = cnn.init_params(seed)
    series = [rand_series(rng, L) for L in (9, 13, 16)]
    pairs = [(0, 1), (1, 2), (2, 0)]
    targets = [5.0, 12.0, 30.0]
    loss, grads, _ = cnn.batch_loss_and_grads(params, series, pairs, targets)
    flat = cnn.flatten(params)
    gflat = cnn.flatten(grads)
    assert flat.size == cnn.n_params()
    idx = rng.choice(flat.size, 60, replace=False)
    # include every bias of the last layer and a tap at each edge of layer 1
    idx = np.concatenate([idx, np.arange(cnn.n_params() - cnn.CHANNELS[-1], cnn.n_params()), [0, 4 * 2 * 64]])
    h = 1e-6
    for i in idx:
        fp, fm = flat.copy(), flat.copy()
        fp[i] += h
        fm[i] -= h
        lp, _, _ = cnn.batch_loss_and_grads(cnn.unflatten(fp), series, pairs, targets)
        lm, _, _ = cnn.batch_loss_and_grads(cnn.unflatten(fm), series, pairs, targets)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - gflat[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (i, fd, gflat[i])


def test_flatten_roundtrip():
    p = cnn.init_params(5)
    q = cnn.unflatten(cnn.flatten(p))
    for l in range(4):
        assert np.array_equal(p["W"][l], q["W"][l]) and np.array_equal(p["b"][l], q["b"][l])


def test_adamw_first_step_is_signed_lr():
    # at step 1 the bias-corrected ratio m_hat / sqrt(v_hat) is g / |g| exactly
    # (up to eps), so each weight moves by lr against the gradient's sign
    rng = np.random.default_rng(5)
    w = rng.standard_normal(50)
    g = rng.standard_normal(50)
    w1, m1, v1 = cnn.adamw_step(w, np.zeros(50), np.zeros(50), g, 1, 1e-2, 0.0, eps=0.0)
    np.testing.assert_allclose(w1, w - 1e-2 * np.sign(g), rtol=0, atol=1e-15)
    np.testing.assert_allclose(m1, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v1, 0.001 * g * g, rtol=1e-12)


def test_adamw_decay_only():
    # zero gradient and zero moments: only the decoupled decay acts
    w = np.linspace(-1, 1, 9)
    w1, _, _ = cnn.adamw_step(w, np.zeros(9), np.zeros(9), np.zeros(9), 3, 0.1, 0.5)
    np.testing.assert_allclose(w1, w * (1 - 0.05), rtol=1e-15)

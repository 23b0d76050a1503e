"""Pins for the float64 selector reference (oracle/mlp_ref.py): central finite
differences, the closed-form softmax cross-entropy gradient, Adam's first
step, and block features of a hand-built parse."""
import numpy as np

import oracle
from oracle import mlp_ref


def _rand(seed, B=7):
    rng = np.random.default_rng(seed)
    theta = rng.normal(0, 0.3, mlp_ref.N_PARAMS)
    x = rng.normal(0, 1, (B, 64))
    y = rng.integers(0, 16, B)
    return theta, x, y


def test_param_count():
    assert mlp_ref.N_PARAMS == 64 * 128 + 128 + 128 * 128 + 128 + 128 * 16 + 16 == 26896


def test_gradient_matches_central_differences():
    theta, x, y = _rand(1)
    g = mlp_ref.grad(theta, x, y)
    rng = np.random.default_rng(2)
    idx = rng.choice(theta.size, 60, replace=False)
    # include every block of parameters
    idx = np.concatenate([idx, [0, 64 * 128 + 3, 64 * 128 + 128 + 5, 26896 - 16 - 1, 26896 - 1]])
    h = 1e-6
    for i in idx:
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        fd = (mlp_ref.loss(tp, x, y) - mlp_ref.loss(tm, x, y)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd), (i, fd, g[i])


def test_softmax_ce_closed_form():
    """With a zero last layer the logits vanish: loss = ln 16 and the output
    bias gradient is (1/16 - onehot) averaged over the batch."""
    theta, x, y = _rand(3, B=5)
    o3 = mlp_ref.N_PARAMS - 16 - 128 * 16
    theta[o3:] = 0.0
    assert abs(mlp_ref.loss(theta, x, y) - np.log(16.0)) < 1e-12
    g = mlp_ref.grad(theta, x, y)
    gb3 = g[-16:]
    want = np.full(16, 1.0 / 16) - np.bincount(y, minlength=16) / len(y)
    assert np.allclose(gb3, want, atol=1e-15)


def test_adam_first_step_is_sign_step():
    rng = np.random.default_rng(4)
    th = rng.normal(size=100)
    g = rng.normal(size=100)
    t2, m, v = mlp_ref.adam(th, g, np.zeros(100), np.zeros(100), 1, lr=1e-3, eps=1e-12)
    assert np.allclose(th - t2, 1e-3 * np.sign(g), rtol=1e-9, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_block_features_hand_built():
    """Two blocks of 64 bytes laid out by hand (distance bounds 20/40/80)."""
    n = 128
    ll = np.array([16, 16, 0, 8], np.uint32)
    ml = np.array([32, 0, 40, 16], np.uint32)
    src = np.array([0, 0, 0, 88], np.uint64)
    lit = np.arange(40, dtype=np.uint8) + 1
    arc = oracle.write_archive(n, 6, ll, ml, src, lit)
    T = oracle.tokens(arc)
    F = mlp_ref.block_features(T, n, 6, (20, 40, 80))
    assert F.shape == (2, 64)
    f0 = F[0].reshape(4, 16)
    f1 = F[1].reshape(4, 16)
    # block 0: match at dst 16, src 0 -> d 16 -> class 0, len 32 -> bin 8 ([32,48))
    assert f0[0, 8] == 32 / 64 and f0.sum() == 32 / 64
    # block 1: match at dst 64 from 0 -> d 64 -> class 2, len 40 -> bin 8;
    # match at dst 112 from 88 -> d 24 -> class 1, len 16 -> bin 5 ([16,20))
    assert f1[2, 8] == 40 / 64 and f1[1, 5] == 16 / 64 and abs(f1.sum() - 56 / 64) < 1e-15

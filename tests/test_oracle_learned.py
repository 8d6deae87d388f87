"""Pins of the selector-network oracle and of the learned (q, p) oracle.

* Backward pass: central finite differences of the forward loss (h = 1e-6,
  FP64) on every parameter of a small random network.
* Forward pass: a hand-computed two-sample example; the loss of the zero
  network is log(15) exactly.
* Adam: the first step moves each parameter by -lr g / (|g| + eps) exactly
  (bias correction makes m^ = g and v^ = g^2).
* Features: the sketch spectrum is scale invariant, starts at 1, is
  descending, equals the spectrum of the sketch's QR factor, and a rank-r
  matrix has no more than r non-negligible values.
* Labels: a matrix with a huge spectral gap after k needs the cheapest pair;
  a slowly decaying one needs power iterations.
"""
import math

import numpy as np
import pytest

from oracle import learned as lrn
from oracle import philox
from oracle import mlp
from oracle import rsvd as orc
from synth import matrices as syn


def _rand_theta(seed, scale=0.3):
    return np.random.default_rng(seed).standard_normal(mlp.N_PARAMS) * scale


def test_param_count():
    assert mlp.N_PARAMS == 131 * 64 + 64 + 64 * 64 + 64 + 64 * 15 + 15 == 13583


def test_backward_matches_central_differences():
    rng = np.random.default_rng(3)
    theta = _rand_theta(4)
    X = rng.standard_normal((7, mlp.N_IN))
    y = rng.integers(0, mlp.N_OUT, size=7)
    _, g = mlp.loss_and_grad(theta, X, y)
    h = 1e-6
    idx = np.concatenate([rng.choice(mlp.N_PARAMS, 300, replace=False),
                          np.arange(mlp.N_PARAMS - 15 - 64 * 15, mlp.N_PARAMS)])   # all of layer 3
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss(tp, X, y) - mlp.loss(tm, X, y)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_forward_hand_example():
    theta = np.zeros(mlp.N_PARAMS)
    P = mlp.unpack(theta)
    P["W1"][0, 0] = 2.0          # h1[0] = relu(2 x0)
    P["W1"][1, 1] = -1.0         # h1[1] = relu(-x1)
    P["b1"][2] = -0.5            # h1[2] = relu(-0.5) = 0
    P["W2"][0, 0] = 1.0          # h2[0] = h1[0]
    P["W2"][1, 0] = 3.0          #       + 3 h1[1]
    P["b2"][1] = 0.25            # h2[1] = 0.25
    P["W3"][0, 4] = 1.0          # z[4] = h2[0]
    P["W3"][1, 7] = -2.0         # z[7] = -2 h2[1] = -0.5
    P["b3"][0] = 0.1
    X = np.zeros((2, mlp.N_IN))
    X[0, 0], X[0, 1] = 1.5, -2.0     # h1 = (3, 2, 0) -> h2[0] = 9
    X[1, 0], X[1, 1] = -1.0, 4.0     # h1 = (0, 0, 0) -> h2[0] = 0
    f = mlp.forward(theta, X)
    z0 = np.zeros(15); z0[0] = 0.1; z0[4] = 9.0; z0[7] = -0.5
    z1 = np.zeros(15); z1[0] = 0.1; z1[7] = -0.5
    np.testing.assert_allclose(f["z"], np.stack([z0, z1]), rtol=0, atol=1e-15)
    e0 = np.exp(z0 - z0.max())
    np.testing.assert_allclose(f["prob"][0], e0 / e0.sum(), rtol=1e-15)


def test_zero_network_loss_is_log_classes():
    X = np.random.default_rng(0).standard_normal((5, mlp.N_IN))
    assert mlp.loss(np.zeros(mlp.N_PARAMS), X, np.arange(5)) == pytest.approx(math.log(15), abs=1e-15)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(1)
    theta = rng.standard_normal(mlp.N_PARAMS)
    g = rng.standard_normal(mlp.N_PARAMS) * 1e-2
    z = np.zeros(mlp.N_PARAMS)
    t1, m1, v1 = mlp.adam_step(theta, g, z, z, 1, lr=1e-3)
    np.testing.assert_allclose(t1, theta - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-18)
    np.testing.assert_allclose(m1, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v1, 0.001 * g * g, rtol=1e-14)   # 1 - 0.999 is 0.001 + 9e-19


def test_classes_and_costs():
    assert lrn.N_CLASSES == 15
    assert [lrn.class_pair(c) for c in (0, 2, 3, 14)] == [(0, 5), (0, 20), (1, 5), (4, 20)]
    order = lrn.classes_by_cost(10)
    assert order[0] == lrn.pair_class(0, 5)
    costs = [lrn.pair_cost(10, *lrn.class_pair(c)) for c in order]
    assert costs == sorted(costs)
    # (q=0, p=20) and (q=1, p=5) both cost 60 at k = 10: the lower class first
    assert order.index(lrn.pair_class(0, 20)) < order.index(lrn.pair_class(1, 5))


def test_features_properties():
    A = syn.planted(300, 120, syn.spectrum("poly", 120, alpha=1.0), 5)
    f = lrn.features(A, 12, seed=9, stream_id=3)
    l0 = lrn.sketch_width0(300, 120, 12)
    assert l0 == 32 and f.shape == (131,)
    assert f[0] == 1.0 and np.all(np.diff(f[:l0]) <= 0) and np.all(f[l0:128] == 0)
    np.testing.assert_allclose(f[128:], [math.log2(300) / 12, math.log2(120) / 12, math.log2(12) / 12])
    np.testing.assert_allclose(lrn.features(A * 1024.0, 12, seed=9, stream_id=3), f, rtol=1e-13, atol=0)
    # same spectrum through the QR factor of the sketch
    _, R0 = orc.hqr(lrn.sketch(A, 12, seed=9, stream_id=3))
    s = np.linalg.svd(R0, compute_uv=False)
    np.testing.assert_allclose(f[:l0], s / s[0], rtol=1e-12, atol=1e-15)


def test_features_of_low_rank_matrix():
    A = syn.planted(200, 100, np.array([3.0, 2.0, 1.0]), 6)
    f = lrn.features(A, 5, seed=1)
    assert np.all(f[3:lrn.sketch_width0(200, 100, 5)] < 1e-12)
    assert f[1] > 0.1 and f[2] > 0.05


def test_label_gap_needs_cheapest_pair():
    k = 6
    sig = np.concatenate([np.linspace(10, 5, k), 1e-6 * 0.5 ** np.arange(94)])
    A = syn.planted(240, 100, sig, 7)
    c, ok = lrn.label(A, k, seed=2, sigma_next=sig[k])
    assert ok and c == lrn.classes_by_cost(k)[0]


def test_label_slow_decay_needs_power_iterations():
    k = 10
    sig = syn.spectrum("poly", 150, alpha=0.5)
    A = syn.planted(400, 150, sig, 8)
    c, ok = lrn.label(A, k, seed=2, sigma_next=sig[k])
    q, p = lrn.class_pair(c)
    assert ok and q >= 1
    assert lrn.excess_error(A, k, 0, 20, seed=2, sigma_next=sig[k]) > 0.01


def test_posterior_estimate_bounds_the_error():
    A = syn.planted(300, 200, syn.spectrum("poly", 200, alpha=1.0), 9)
    U, s, V = orc.rsvd(A, 10, p=5, q=0, seed=1)
    true = np.linalg.norm(A - (U * s[None, :]) @ V.T, 2)
    hits = sum(lrn.posterior_estimate(A, U, s, V, r=10, seed=100 + t) >= true for t in range(20))
    assert hits == 20


def test_posterior_estimate_rank_one_residual_closed_form():
    """R = A - U S V^T = sigma a b^T gives ||R w_i|| = sigma ||a|| |b^T w_i|
    exactly, so the estimate is 10 sqrt(2/pi) sigma ||a|| max_i |b^T w_i|."""
    rng = np.random.default_rng(4)
    m, n, k, r = 60, 40, 5, 7
    U = np.linalg.qr(rng.standard_normal((m, k)))[0]
    V = np.linalg.qr(rng.standard_normal((n, k)))[0]
    s = np.sort(rng.uniform(1, 3, k))[::-1]
    a, b, sig = rng.standard_normal(m), rng.standard_normal(n), 0.37
    A = (U * s) @ V.T + sig * np.outer(a, b)
    W = philox.test_matrix(n, r, 12, 34)
    want = 10.0 * np.sqrt(2.0 / np.pi) * sig * np.linalg.norm(a) * np.max(np.abs(b @ W))
    assert lrn.posterior_estimate(A, U, s, V, r=r, seed=12, stream_id=34) == pytest.approx(want, rel=1e-12)

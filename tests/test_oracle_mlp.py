"""Pins of the rank-predictor oracle: chain rule against central differences,
closed-form networks, the first Adam step, invariances of the features and
their tie to eq. (bounds)."""
import math

import numpy as np
import pytest

from oracle import hss as ohss, mlp, secular as osec


def rand_theta(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, mlp.NPARAM)


def test_param_count():
    assert mlp.NPARAM == 16 * 64 + 64 + 64 * 64 + 64 + 64 + 1 == 5313


def test_gradient_vs_central_differences():
    rng = np.random.default_rng(1)
    th = rand_theta(2)
    X = rng.normal(0, 1, (7, 16))
    y = rng.normal(0, 1, 7)
    loss, g = mlp.loss_grad(th, X, y)
    assert abs(loss - np.mean((mlp.forward(th, X) - y) ** 2)) <= 1e-14 * max(loss, 1)
    # every bias and a sample of weights of every layer
    idx = list(range(1024, 1088)) + list(range(5184, 5248)) + [5312]
    idx += list(rng.choice(1024, 40, replace=False)) + list(1088 + rng.choice(4096, 60, replace=False))
    idx += list(range(5248, 5312))
    h = 1e-6
    for i in idx:
        tp = th.copy()
        tp[i] += h
        tm = th.copy()
        tm[i] -= h
        fd = (mlp.loss_grad(tp, X, y)[0] - mlp.loss_grad(tm, X, y)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_forward_closed_form():
    """W1 = [I; 0], W2 = I, W3 = 1, b3 = 0.5: y = sum_k relu(x_k) + 0.5."""
    th = np.zeros(mlp.NPARAM)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(th)
    W1[:16, :16] = np.eye(16)
    W2[:, :] = np.eye(64)
    W3[:] = 1.0
    b3[:] = 0.5
    X = np.random.default_rng(3).normal(0, 1, (9, 16))
    y = mlp.forward(th, X)
    assert np.allclose(y, np.maximum(X, 0).sum(axis=1) + 0.5, rtol=0, atol=1e-14)
    # a negative bias switches a unit off and its gradient with it
    b2[0] = -1e3
    _, g = mlp.loss_grad(th, X, np.zeros(9))
    W2g = mlp.unpack(g)[2]
    assert np.all(W2g[0] == 0.0)


def test_first_adam_step_closed_form():
    """With m = v = 0 the first bias-corrected step is lr g / (|g| + eps)."""
    rng = np.random.default_rng(4)
    th = rand_theta(5)
    X = rng.normal(0, 1, (5, 16))
    y = rng.normal(0, 1, 5)
    _, g = mlp.loss_grad(th, X, y)
    th1, st, _ = mlp.adam_train(th, X, y, epochs=1, batch=5, lr=1e-2)
    assert np.allclose(th1, th - 1e-2 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert st["t"] == 1


def test_adam_learns_a_linear_target():
    rng = np.random.default_rng(6)
    X = rng.uniform(-1, 1, (512, 16))
    y = X @ rng.normal(0, 1, 16) + 0.3
    th = rand_theta(7, 0.2)
    l0 = mlp.loss_grad(th, X, y)[0]
    th, _, last = mlp.adam_train(th, X, y, epochs=40, batch=64, lr=3e-3)
    assert mlp.loss_grad(th, X, y)[0] < 0.02 * l0
    assert last < 0.05 * l0


def merge_generators(K, seed, spread="uniform"):
    rng = np.random.default_rng(seed)
    if spread == "uniform":
        d = np.sort(rng.uniform(0, 1, K))
    else:
        d = np.sort(np.concatenate([rng.uniform(0, 1e-3, K // 2), rng.uniform(0.5, 1, K - K // 2)]))
    z = rng.normal(0, 1, K)
    z /= np.linalg.norm(z)
    rho = 1.3
    _, gam, mu, _ = osec.secular_roots(d, z, rho)
    return d, gam, mu


@pytest.mark.parametrize("spread", ["uniform", "clustered"])
def test_features_invariant_under_affine_maps(spread):
    """Every feature is a ratio of differences: d -> a d + c with gam, mu -> a
    gam, a mu (a > 0) leaves them unchanged."""
    d, gam, mu = merge_generators(300, 8, spread)
    bounds = [0, 37, 75, 150, 225, 300]
    F = mlp.features(d, gam, mu, bounds)
    a, c = 2.0 ** 7, -3.25
    F2 = mlp.features(a * d + c, a * gam, a * mu, bounds)
    assert F.shape == (4, 16)
    assert np.all(np.isfinite(F)) and np.max(np.abs(F)) <= 2.0
    assert np.max(np.abs(F - F2)) <= 1e-9


def test_feature_3_is_the_ratio_of_eq_bounds():
    d, gam, mu = merge_generators(400, 9)
    bounds = [0, 100, 200, 300, 400]
    F = mlp.features(d, gam, mu, bounds)
    r, _, ranks = ohss.estimate_rank(d, gam, mu, bounds, shift_thresh=0.0)
    for b in range(3):
        R = 2.0 ** (32 * F[b, 3])
        assert ohss.rank_bound(R, 1e-16) == ranks[b]
    # feature 4 (the worst split of the window) is at least feature 3
    assert np.all(F[:, 4] >= F[:, 3] - 1e-15)


def test_feature_layout_values():
    d, gam, mu = merge_generators(64, 10)
    bounds = [0, 16, 32, 48, 64]
    F = mlp.features(d, gam, mu, bounds)
    assert np.allclose(F[:, 0], 6 / 16)
    assert np.allclose(F[:, 1], 4 / 8) and np.allclose(F[:, 2], 4 / 8)
    assert np.allclose(F[:, 12], [0.25, 0.5, 0.75])
    assert np.allclose(F[:, 13], 2 / 8)
    assert np.all(F[:, 5] <= F[:, 6]) and np.all(F[:, 6] <= F[:, 7])
    assert np.all(F[:, 15] <= 0.0)  # dist(p) <= the pole gap at p
    assert np.all(F[:, 11] == 0.0)


def test_boundary_targets_and_predicted_rank():
    # root [0,8), children [0,4) [4,8), leaves [0,2) [2,4) [4,6) [6,8)
    lo = [0, 0, 4, 0, 2, 4, 6]
    hi = [8, 4, 8, 2, 4, 6, 8]
    kr = [0, 5, 6, 3, 2, 7, 1]
    kc = [0, 4, 9, 1, 3, 2, 2]
    t = mlp.boundary_targets(lo, hi, kr, kc, [0, 2, 4, 6, 8])
    assert np.allclose(t, np.log2([3, 9, 7]))
    assert mlp.predicted_rank(np.log2([3.0, 9.0, 7.0])) == 16  # ceil(1.25 * 9) + 4
    assert mlp.predicted_rank(np.array([0.0])) == 8
    assert mlp.predicted_rank(np.array([9.0])) == 100


def test_features_by_hand():
    """All 16 features of a tiny merge, worked out by hand from the feature
    definitions (module docstring of oracle/mlp.py).  K = 8 poles, leaves
    [0,2) [2,4) [4,6) [6,8), boundaries p = 2, 4, 6.  Pole gaps g = 1 1 2 1 1 2 2,
    gam = 1/4 1/2 1 1/4 1/2 1 1 6, mu = g - gam (mu_7 = inf), so
    lam = 0.25 1.5 3 4.25 5.5 7 9 16 and span = lam_7 - d_0 = 16.  By
    interlacing, dist(q) = mu_{q-1}: dist(1..7) = 3/4 1/2 1 3/4 1/2 1 1."""
    d = np.array([0.0, 1, 2, 4, 5, 6, 8, 10])
    gam = np.array([0.25, 0.5, 1.0, 0.25, 0.5, 1.0, 1.0, 6.0])
    mu = np.array([0.75, 0.5, 1.0, 0.75, 0.5, 1.0, 1.0, np.inf])
    F = mlp.features(d, gam, mu, [0, 2, 4, 6, 8])
    l2 = math.log2
    s2 = math.sqrt(2.0) / 3.0  # std of log2 gaps {-4,-4,-3} and {-4,-3,-3}
    want = [
        # p = 2: window [0,4); gaps 1 1 2 -> log2(g/16) = -4 -4 -3;
        # min(gam, mu) = 1/4 1/2 1 1/4 -> log2(./16) = -6 -5 -4 -6
        [3 / 16, 1 / 8, 1 / 8, l2(16 / 0.5) / 32, l2(16 / 0.5) / 32,
         -4 / 32, (-11 / 3) / 32, -3 / 32, s2 / 8, (-21 / 4) / 32, -6 / 32,
         0.0, 2 / 8, l2(4) / 8, l2(4 / 16) / 32, l2(0.5 / 1) / 32],
        # p = 4: window [2,6); gaps 2 1 1; min(gam, mu) = 1 1/4 1/2 1;
        # dist(4) = 3/4, min dist over q = 3, 4, 5 is 1/2
        [3 / 16, 1 / 8, 1 / 8, l2(16 / 0.75) / 32, l2(16 / 0.5) / 32,
         -4 / 32, (-11 / 3) / 32, -3 / 32, s2 / 8, (-19 / 4) / 32, -6 / 32,
         0.0, 4 / 8, l2(4) / 8, l2(4 / 16) / 32, l2(0.75 / 1) / 32],
        # p = 6: window [4,8); gaps 1 2 2; min(gam, mu) = 1/2 1 1 6;
        # dist(6) = 1, min dist over q = 5, 6, 7 is 1/2
        [3 / 16, 1 / 8, 1 / 8, l2(16 / 1.0) / 32, l2(16 / 0.5) / 32,
         -4 / 32, (-10 / 3) / 32, -3 / 32, s2 / 8, ((-13 + l2(6 / 16)) / 4) / 32, -5 / 32,
         0.0, 6 / 8, l2(4) / 8, l2(5 / 16) / 32, l2(1 / 2) / 32],
    ]
    assert np.max(np.abs(F - np.array(want))) <= 1e-15


def test_feature_11_counts_tiny_gaps():
    """Feature 11 by hand: K = 6, one window [0, 6) (two leaves); pole gaps
    1 1e-12 1 1 2 over span 16 -> one of five gaps is below 1e-10 span."""
    d = np.array([0.0, 1.0, 1.0 + 1e-12, 2.0 + 1e-12, 3.0 + 1e-12, 5.0 + 1e-12])
    gap = np.diff(d)
    gam = np.concatenate([gap / 2, [16.0 - d[-1]]])
    mu = np.concatenate([gap - gap / 2, [np.inf]])
    F = mlp.features(d, gam, mu, [0, 3, 6])
    assert F.shape == (1, 16)
    assert F[0, 11] == 1 / 5
    assert F[0, 13] == 1 / 8  # log2(2 leaves) / 8

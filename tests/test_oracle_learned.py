"""Pins for the oracle side of the power-iteration predictor (CPU only)."""
import numpy as np
import pytest

import workloads as W
from oracle import randqlp, rel_error
from oracle import mlp
from oracle.learned import (features_from_sigma, label_q, optimal_error, qlp_errors,
                            qlp_errors_diag, sketch_features, sketch_features_diag)


def _diag(m, n, sigma):
    A = np.zeros((m, n))
    A[np.arange(sigma.size), np.arange(sigma.size)] = sigma
    return A


def test_one_run_errors_equal_separate_runs():
    """e(j) and e_k(j) from one power loop equal those of separate q = j runs,
    with the rank-k error formed explicitly from the returned factors."""
    A, U, s, V = W.poly_decay(260, 180, 0.7, seed=3)
    k, p, qmax, seed = 15, 5, 3, 11
    e, ek = qlp_errors(A, k, p, qmax, seed)
    for j in range(qmax + 1):
        Q, L, P = randqlp(A, k, p, j, seed)
        assert abs(e[j] - rel_error(A, Q, L, P)) < 1e-12
        trunc = np.linalg.norm(A - Q @ L[:, :k] @ P[:, :k].T) / np.linalg.norm(A)
        assert abs(ek[j] - trunc) < 1e-12
    assert np.all(np.diff(ek) <= 1e-12)        # power rounds do not hurt here


def test_diagonal_products_equal_dense_diagonal():
    sigma = np.arange(1, 151, dtype=np.float64) ** -1.2
    for (m, n) in [(300, 150), (150, 220)]:
        A = _diag(m, n, sigma)
        e1, k1 = qlp_errors(A, 20, 6, 3, 5)
        e2, k2 = qlp_errors_diag(sigma, m, n, 20, 6, 3, 5)
        assert np.abs(e1 - e2).max() < 1e-12 and np.abs(k1 - k2).max() < 1e-12
        f1 = sketch_features(A, 20, 5)
        f2 = sketch_features_diag(sigma, m, n, 20, 5)
        assert np.abs(f1 - f2).max() < 1e-12


def test_rotation_invariance_in_distribution():
    """The error of U diag(s) V^T and of diag(s) have the same distribution
    over the sketch: the means over 24 seeds agree within their spread."""
    m, n, k, p = 200, 160, 10, 4
    A, U, s, V = W.poly_decay(m, n, 1.0, seed=2)
    rot = np.array([qlp_errors(A, k, p, 0, sd)[0][0] for sd in range(24)])
    dia = np.array([qlp_errors_diag(s, m, n, k, p, 0, sd)[0][0] for sd in range(24)])
    se = np.sqrt((rot.var() + dia.var()) / 24)
    assert abs(rot.mean() - dia.mean()) < 4 * se + 1e-12


def test_exact_rank_gives_zero_error_and_label_zero():
    sigma = np.array([5.0, 3.0, 1.0, 0.5])
    e, ek = qlp_errors_diag(sigma, 50, 40, 4, 3, 2, 1)
    assert np.all(e < 3e-8) and np.all(ek < 3e-8)   # sqrt(u) floor of the identity
    assert label_q(ek, sigma, 4) == 0


def test_features_closed_forms():
    f = features_from_sigma(np.array([2.0, 0.2, 0.02, 0.0]), 64)
    assert np.allclose(f[:3], [0.0, -1 / 6, -2 / 6])
    assert np.all(f[3:64] == -1.0) and f[64] == 0.25
    # a rank-1 A: one nonzero sketch singular value
    u = np.linspace(1, 2, 90)[:, None]
    v = np.linspace(-1, 1, 70)[None, :]
    g = sketch_features(u @ v, 8, 0)
    assert g[0] == 0.0 and np.all(g[1:64] == -1.0)


def test_label_and_optimal_error():
    s = np.array([1.0, 0.5, 0.1, 0.1])
    assert abs(optimal_error(s, 2) - np.sqrt(0.02 / 1.27)) < 1e-15
    t = 1.05 * np.sqrt(0.02 / 1.27)
    assert label_q([t * 1.2, t * 1.01, t * 0.99], s, 2) == 2
    assert label_q([t * 1.2, t * 1.1], s, 2) == 2       # unreachable -> len
    assert label_q([0.0], s, 2) == 0


# ------------------------------------------------------------------ the MLP
def _toy(seed, B=64):
    r = np.random.default_rng(seed)
    X = r.standard_normal((B, 65)) * 0.5
    y = r.integers(0, 6, B)
    return X, y


def test_mlp_gradient_matches_central_differences():
    X, y = _toy(0, 12)
    theta = mlp.init_params(3)
    theta += 0.01 * np.random.default_rng(1).standard_normal(theta.size)   # nonzero biases
    loss, g = mlp.loss_and_grad(theta, X, y)
    idx = np.random.default_rng(2).choice(theta.size, 60, replace=False)
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        num = (mlp.loss_and_grad(tp, X, y)[0] - mlp.loss_and_grad(tm, X, y)[0]) / (2 * h)
        assert abs(num - g[i]) <= 1e-7 * max(1.0, abs(num))


def test_mlp_softmax_cross_entropy_closed_form():
    theta = np.zeros(mlp.param_count())
    X, y = _toy(4, 5)
    loss, g = mlp.loss_and_grad(theta, X, y)
    assert abs(loss - np.log(6.0)) < 1e-15       # uniform logits
    (W1, b1), (W2, b2), (W3, b3) = mlp.unpack(g)
    cnt = np.bincount(y, minlength=6)
    assert np.allclose(b3, (5 / 6 - cnt) / 5)    # d/db3 = mean(softmax - onehot)


def test_adam_first_step_is_signed_lr():
    theta = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 0.0])
    t1, m1, v1 = mlp.adam_step(theta, g, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(t1[:2], theta[:2] - 0.01 * np.sign(g[:2]), atol=1e-9)
    assert t1[2] == theta[2]


def test_mlp_learns_a_separable_rule():
    r = np.random.default_rng(5)
    X = r.standard_normal((600, 65))
    y = (X[:, 0] > 0).astype(int) + 2 * (X[:, 1] > 0)
    theta = mlp.init_params(0)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    for t in range(1, 301):
        loss, g = mlp.loss_and_grad(theta, X, y)
        theta, m, v = mlp.adam_step(theta, g, m, v, t, 3e-3)
    assert np.mean(mlp.predict(theta, X) == y) > 0.97


def test_label_rank_on_a_step_spectrum():
    """sigma = 1 on the first r values, 0 after: the rank-k optimum is
    sqrt((r - k) / r) for k < r (closed form), so for r = 40 and tol = 0.5
    the first class with sqrt((40 - k) / 40) <= 0.5 / 1.05 is k = 32."""
    from oracle.learned import RANK_CLASSES, label_rank
    s = np.concatenate([np.ones(40), np.zeros(60)])
    for k in (8, 16, 32, 39):
        assert abs(optimal_error(s, k) - np.sqrt((40 - k) / 40)) < 1e-15
    assert RANK_CLASSES[label_rank(s, 0.5)] == 32
    assert RANK_CLASSES[label_rank(s, 0.9)] == 16     # sqrt(32/40) = 0.894 > 0.9 / 1.05
    assert RANK_CLASSES[label_rank(s, 0.95)] == 8     # 0.894 <= 0.95 / 1.05 = 0.905
    assert label_rank(s, 1e-9) == 3                   # k = 64 >= r: error 0
    assert label_rank(np.arange(1, 2001) ** -0.3, 1e-3) == len(RANK_CLASSES) - 1


def test_label_rank_matches_brute_force_truncation():
    """On small matrices: the truncation error of the SVD (numpy's, an
    independent routine) at each class k decides the label the same way."""
    from oracle.learned import RANK_CLASSES, RANK_SLACK, label_rank
    for alpha, tol in [(0.8, 0.2), (1.5, 0.05), (2.5, 0.01), (0.5, 0.3)]:
        A, U, s, V = W.poly_decay(300, 280, alpha, seed=17)
        u, sv, vt = np.linalg.svd(A)
        errs = [np.linalg.norm(A - (u[:, :k] * sv[:k]) @ vt[:k]) / np.linalg.norm(A)
                for k in RANK_CLASSES]
        want = next((c for c, e in enumerate(errs) if e <= tol / RANK_SLACK),
                    len(RANK_CLASSES) - 1)
        assert label_rank(s, tol) == want


def test_rank_errors_and_smallest_rank():
    """Dense rank-k errors of the oracle's factors against the orthogonal
    split e_k^2 = e^2 + ||L[k:, k:]||^2 / ||A||^2, and the first k under a
    tolerance."""
    from oracle.learned import rank_errors, smallest_rank
    A, U, s, V = W.poly_decay(220, 160, 1.3, seed=5)
    Q, L, P = randqlp(A, 20, 5, 1, 3)
    ek = rank_errors(A, Q, L, P)
    nrm2 = np.sum(A * A)
    e2 = rel_error(A, Q, L, P) ** 2
    for k in (1, 7, 25):
        assert abs(ek[k - 1] - np.sqrt(e2 + np.sum(L[k:, k:] ** 2) / nrm2)) < 1e-12
    assert np.all(np.diff(ek) <= 1e-15)
    tol = float(ek[9])
    assert smallest_rank(ek, tol) == 10
    assert smallest_rank(ek, 0.0) == 25

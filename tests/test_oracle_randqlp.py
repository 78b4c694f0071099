"""Pins for the oracle's Rand-QLP against what the paper and algebra fix.

None of these re-types the oracle's own formulas: each checks a consequence
that an error in the oracle (a transposed operand, a dropped power
iteration, a missing sign fix, L = R instead of R^T, a wrong Omega) breaks.
"""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import (jacobi_singular_values, orth_error, qr_pos, randqlp,
                    randqlp_flops, rel_error, sketch_width, subspace_sine,
                    paper_flops_full)
from oracle import bounds as B
from oracle.philox import gaussian_matrix

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- Jacobi SVD
def test_jacobi_diag_and_permuted():
    s = np.array([3.0, 1e-3, 2.0, 0.5])
    A = np.diag(s)[:, [2, 0, 3, 1]]
    assert np.allclose(jacobi_singular_values(A), np.sort(s)[::-1], rtol=1e-14, atol=0)


def test_jacobi_known_spectrum_and_rank_one():
    A, U, s, V = W.svd_matrix(30, 20, np.linspace(5.0, 0.1, 20), seed=3)
    assert np.allclose(jacobi_singular_values(A), s, rtol=1e-12)
    x = np.arange(1.0, 8.0)
    y = np.array([2.0, -1.0, 0.5])
    sv = jacobi_singular_values(np.outer(x, y))
    assert sv[0] == pytest.approx(np.sqrt(x @ x) * np.sqrt(y @ y), rel=1e-14)
    assert np.all(np.abs(sv[1:]) < 1e-13)


# ------------------------------------------------------------------ qr_pos
def test_qr_pos_hand_examples():
    Q, R = qr_pos(np.array([[3.0], [4.0]]))
    assert np.allclose(Q, [[0.6], [0.8]]) and np.allclose(R, [[5.0]])
    Q, R = qr_pos(np.array([[-1.0, 1.0], [0.0, 2.0], [0.0, 0.0]]))
    assert np.allclose(Q, [[-1, 0], [0, 1], [0, 0]]) and np.allclose(R, [[1, -1], [0, 2]])


def _gram_schmidt(X):
    Q = np.zeros_like(X)
    R = np.zeros((X.shape[1], X.shape[1]))
    for j in range(X.shape[1]):
        v = X[:, j].copy()
        for _ in range(2):
            for i in range(j):
                c = Q[:, i] @ v
                R[i, j] += c
                v -= c * Q[:, i]
        R[j, j] = np.linalg.norm(v)
        Q[:, j] = v / R[j, j]
    return Q, R


def test_qr_pos_matches_gram_schmidt():
    X = np.random.default_rng(0).standard_normal((40, 9))
    Q, R = qr_pos(X)
    Qg, Rg = _gram_schmidt(X)
    assert np.allclose(Q, Qg, atol=1e-13) and np.allclose(R, Rg, atol=1e-12)
    assert np.all(np.diag(R) >= 0) and np.allclose(np.tril(R, -1), 0)


# ----------------------------------------------------- algebraic identities
@pytest.mark.parametrize("shape,k,p,q", [((120, 80), 10, 5, 0), ((120, 80), 10, 5, 2),
                                         ((60, 90), 7, 3, 1), ((50, 50), 45, 10, 1)])
def test_identities(shape, k, p, q):
    m, n = shape
    A, U, s, V = W.fast_decay(m, n, seed=1)
    Q, L, P = randqlp(A, k, p, q, seed=5)
    d = sketch_width(m, n, k, p)
    assert Q.shape == (m, d) and L.shape == (d, d) and P.shape == (n, d)
    assert orth_error(Q) < 1e-13 and orth_error(P) < 1e-13
    assert np.all(np.triu(L, 1) == 0) and np.all(np.diag(L) >= 0)
    assert np.allclose(L, Q.T @ A @ P, atol=1e-14)                      # L = Q^T A P
    assert np.allclose(Q @ L @ P.T, Q @ (Q.T @ A), atol=1e-14)          # Q L P^T = Q Q^T A
    lhs = np.linalg.norm(A - Q @ L @ P.T) ** 2
    rhs = np.linalg.norm(A) ** 2 - np.linalg.norm(L) ** 2
    assert abs(lhs - rhs) < 1e-13 * np.linalg.norm(A) ** 2


def test_full_width_reconstructs_exactly():
    # d = min(m, n): Q spans range(A) for full-rank A, so A = Q L P^T exactly.
    for (m, n) in [(40, 40), (60, 30), (30, 45)]:
        A = np.asfortranarray(np.random.default_rng(m + n).random((m, n)))
        Q, L, P = randqlp(A, min(m, n), 0, 0, seed=2)
        assert rel_error(A, Q, L, P) < 1e-12
        if m == n:
            assert np.allclose(jacobi_singular_values(L), jacobi_singular_values(A), rtol=1e-10)


def test_scaled_orthonormal_gives_scaled_identity():
    U = W.haar(70, 25, seed=4, stream=9)
    Q, L, P = randqlp(3.5 * U, 20, 5, 1, seed=8)
    assert np.allclose(L, 3.5 * np.eye(25), atol=1e-13)


def test_exact_low_rank_reconstructs_and_reveals():
    sig = np.array([4.0, 2.0, 1.0, 0.5, 0.25, 0.1])
    A, U, s, V = W.svd_matrix(80, 60, sig, seed=6)
    Q, L, P = randqlp(A, 8, 4, 0, seed=3)
    assert rel_error(A, Q, L, P) < 1e-13
    assert np.allclose(jacobi_singular_values(L[:6, :6]), sig, rtol=1e-10)
    assert np.abs(L[6:, 6:]).max() < 1e-13


def test_range_equals_explicit_power_sketch():
    # R(Q) = R((A A^T)^(q+1) Omega) and R(P) = R(A^T (A A^T)^(q+1) Omega),
    # nested by prefix (the proofs of Theorems 1 and 2).  Built here without
    # any QR between the products, on a well-conditioned spectrum.
    sig = np.linspace(2.0, 1.0, 30)
    A, U, s, V = W.svd_matrix(50, 30, sig, seed=11)
    for q in (0, 1, 2):
        Q, L, P = randqlp(A, 6, 2, q, seed=4)
        om = gaussian_matrix(50, 8, seed=4)
        Y = om
        for _ in range(q + 1):
            Y = A @ (A.T @ Y)
        Z = A.T @ Y
        for j in (3, 8):
            Qy, _ = np.linalg.qr(Y[:, :j])
            Qz, _ = np.linalg.qr(Z[:, :j])
            assert subspace_sine(Qy, Q[:, :j]) < 1e-11
            assert subspace_sine(Qz, P[:, :j]) < 1e-11
        Y2 = A @ (A.T @ Y)          # one power too many must not match
        Qw, _ = np.linalg.qr(Y2)
        assert subspace_sine(Qw, Q) > 1e-6


def test_prefix_property_across_oversampling():
    A, U, s, V = W.fast_decay(90, 70, seed=2)
    Q1, L1, P1 = randqlp(A, 10, 0, 1, seed=7)
    Q2, L2, P2 = randqlp(A, 10, 12, 1, seed=7)
    assert np.allclose(Q1, Q2[:, :10], atol=1e-13)
    assert np.allclose(P1, P2[:, :10], atol=1e-13)
    assert np.allclose(L1, L2[:10, :10], atol=1e-14)


def test_deterministic_inequalities():
    A, U, s, V = W.fast_decay(60, 40, seed=5)
    Q, L, P = randqlp(A, 12, 4, 1, seed=9)
    d = L.shape[0]
    sv_a = jacobi_singular_values(A)
    assert L[0, 0] <= sv_a[0] * (1 + 1e-14)
    for j in (4, 9, d):
        sv_l = jacobi_singular_values(L[:j, :j])
        assert np.all(sv_l <= sv_a[:j] * (1 + 1e-12))                     # interlacing
        assert np.prod(np.diag(L)[:j]) <= np.prod(sv_a[:j]) * (1 + 1e-10)
    ey = np.sqrt(np.sum(s[d:] ** 2)) / np.linalg.norm(A)                # Eckart-Young
    assert rel_error(A, Q, L, P) >= ey * (1 - 1e-12)


def test_more_power_iterations_approach_optimum():
    sig = np.concatenate([np.ones(10), 0.3 * np.ones(50)])
    A, U, s, V = W.svd_matrix(80, 60, sig, seed=12)
    errs = [rel_error(A, *randqlp(A, 10, 0, q, seed=3)) for q in range(4)]
    opt = np.sqrt(np.sum(s[10:] ** 2)) / np.linalg.norm(A)
    assert errs[3] < errs[0]
    assert errs[3] / opt < 1.01


# ------------------------------------------------------ Theorems 1, 2, 3
@pytest.mark.parametrize("q", [0, 1, 2])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_paper_bounds_hold(q, seed):
    m, n, k, p = 90, 60, 8, 4
    sig = np.concatenate([np.linspace(1.0, 0.5, k), 0.3 * 0.9 ** np.arange(n - k)])
    A, U, s, V = W.svd_matrix(m, n, sig, seed=seed + 20)
    Q, L, P, st = randqlp(A, k, p, q, seed=seed, return_steps=True)
    t = B.theorem_quantities(U, s, st["omega"], k, q)
    lo, up, l22 = B.theorem1_bounds(t)
    sv = jacobi_singular_values(L[:k, :k])
    assert np.all(sv <= up * (1 + 1e-12)) and np.all(sv >= lo * (1 - 1e-12))
    assert np.linalg.norm(L[k:, k:], 2) <= l22 * (1 + 1e-12)
    b2 = B.theorem2_bounds(t)
    assert subspace_sine(U[:, :k], Q[:, :k]) <= b2["theta_Q"] * (1 + 1e-9) + 1e-14
    assert subspace_sine(V[:, :k], P[:, :k]) <= b2["theta_P"] * (1 + 1e-9) + 1e-14
    for rho in ("fro", 2):
        bq, bp = B.theorem3_bounds(t, A, rho)
        Qk, Pk = Q[:, :k], P[:, :k]
        eq = np.linalg.norm(A - Qk @ (Qk.T @ A), rho)
        ep = np.linalg.norm(A - (A @ Pk) @ Pk.T, rho)
        assert eq <= bq * (1 + 1e-12) and ep <= bp * (1 + 1e-12)


def test_paper_trailing_subspace_bounds_full_width():
    # phi bounds need Q2, P2 to span the trailing subspaces: d = n.
    n, k = 40, 6
    sig = np.concatenate([np.ones(k), 0.2 * 0.8 ** np.arange(n - k)])
    for seed in range(4):
        A, U, s, V = W.svd_matrix(n, n, sig, seed=seed + 40)
        Q, L, P, st = randqlp(A, n, 0, 0, seed=seed, return_steps=True)
        b2 = B.theorem2_bounds(B.theorem_quantities(U, s, st["omega"], k, 0))
        assert subspace_sine(U[:, k:], Q[:, k:]) <= b2["phi_Q"] * (1 + 1e-9) + 1e-14
        assert subspace_sine(V[:, k:], P[:, k:]) <= b2["phi_P"] * (1 + 1e-9) + 1e-14


# -------------------------------------------------------------- flop model
def test_flop_model_reduces_to_paper_count():
    g = json.load(open(os.path.join(GOLDEN, "flop_count.json")))
    assert g["total"] == "8*m*n^2 + 3*n^3 - 2*n^2"
    for (m, n) in [(1856, 1856), (7320, 7320), (5000, 3000)]:
        ours = randqlp_flops(m, n, n, 0)
        paper = paper_flops_full(m, n)
        items = (m * n + (2 * m * n * n - n * n) + 5 * n ** 3 / 3 + (2 * m * n * n - m * n)
                 + (2 * m * n * n - n ** 3 / 3) + (2 * m * n * n - n * n) + 5 * n ** 3 / 3)
        assert items == pytest.approx(paper, rel=1e-12)      # the itemisation sums to the total
        assert ours == pytest.approx(paper, rel=5.0 / n)     # equal up to lower-order terms
    # passes over A: 2q + 3 GEMMs read A; q = 0 gives the paper's three.
    assert g["passes_over_A"]["value"] == 3
    assert randqlp_flops(100, 100, 10, 2) > randqlp_flops(100, 100, 10, 1)


# ---------------------------------------------------- planted mistakes
def _mutant(kind):
    def run(A, k, p, q, seed):
        m, n = A.shape
        d = sketch_width(m, n, k, p)
        om = gaussian_matrix(m, d, seed)
        qb, _ = qr_pos(A.T @ om)
        for _ in range(q + (1 if kind == "extra_power" else 0)):
            qq, _ = qr_pos(A @ qb)
            qb, _ = qr_pos(A.T @ qq)
        Q, _ = qr_pos(A @ qb)
        if kind == "no_sign_fix":
            P, R = np.linalg.qr(A.T @ Q)      # final QR without the diag(R) >= 0 normalisation
        else:
            P, R = qr_pos(A.T @ Q)
        L = R if kind == "L_is_R" else R.T
        if kind == "transposed_sketch":
            Q2, _ = qr_pos(A @ gaussian_matrix(n, d, seed))
            P2, R2 = qr_pos(A.T @ Q2)
            return Q2, R2.T, P2
        return Q, L, P
    return run


@pytest.mark.parametrize("kind", ["extra_power", "L_is_R", "no_sign_fix", "transposed_sketch"])
def test_planted_mistakes_are_caught(kind):
    # Each mutant must fail one of the independent pins above: triangularity
    # and sign of L, L = Q^T A P, or the explicit power-sketch range.
    sig = np.concatenate([np.linspace(2.0, 1.0, 8), 0.6 * 0.97 ** np.arange(52)])
    A, U, s, V = W.svd_matrix(90, 60, sig, seed=21)
    k, p, q = 8, 4, 1
    Q, L, P = _mutant(kind)(A, k, p, q, 0)
    om = gaussian_matrix(90, k + p, seed=0)
    Y = om
    for _ in range(q + 1):
        Y = A @ (A.T @ Y)
    Qy, _ = np.linalg.qr(Y)
    caught = (np.any(np.triu(L, 1) != 0) or np.any(np.diag(L) < 0)
              or not np.allclose(L, Q.T @ A @ P, atol=1e-12)
              or subspace_sine(Qy, Q) > 1e-8)
    assert caught
    # and the unmutated oracle passes the same checks
    Q, L, P = randqlp(A, k, p, q, 0)
    assert not (np.any(np.triu(L, 1) != 0) or np.any(np.diag(L) < 0)
                or not np.allclose(L, Q.T @ A @ P, atol=1e-12)
                or subspace_sine(Qy, Q) > 1e-8)


@pytest.mark.parametrize("q", [0, 1, 2, 3])
def test_bound_exponents_are_attained_in_two_dimensions(q):
    """A = diag(s1, s2), k = 1, p = 0: the sketch direction after q power
    rounds is (AA^T)^(q+1) Omega = (s1^e w1, s2^e w2) with e = 2(q+1), so
    tan theta_Q = psi^(2(q+1)) |M| with M = w2 / w1 exactly, and the
    projection gives tan theta_P = psi^(2q+3) |M|.  Theorem 2's bounds t
    (for R13's exponents) are then attained as sin theta = t / sqrt(1 + t^2):
    a looser exponent gives a larger t and fails the equality as surely as
    a tighter one fails the bound.  Theorem 1's lower bound s1 / sqrt(1 +
    psi^(4(q+1)) |M|^2) = s1 cos theta_Q is attained to O(psi^2 t^2), and
    Theorem 3's bounds are the tail plus ||A|| times Theorem 2's."""
    s = np.array([1.0, 0.5])
    A = np.diag(s)
    for seed in range(3):
        Q, L, P, st = randqlp(A, 1, 0, q, seed=seed, return_steps=True)
        t = B.theorem_quantities(np.eye(2), s, st["omega"], 1, q)
        w = st["omega"][:, 0]
        assert t["M"] == pytest.approx(abs(w[1] / w[0]), rel=1e-14)
        b2 = B.theorem2_bounds(t)
        tq, tp = b2["theta_Q"], b2["theta_P"]
        assert tq == pytest.approx(0.5 ** (2 * (q + 1)) * t["M"], rel=1e-14)
        assert tp == pytest.approx(0.5 ** (2 * q + 3) * t["M"], rel=1e-14)
        sin_q, sin_p = abs(Q[1, 0]), abs(P[1, 0])
        assert sin_q == pytest.approx(tq / np.sqrt(1 + tq * tq), rel=1e-10)
        assert sin_p == pytest.approx(tp / np.sqrt(1 + tp * tp), rel=1e-10)
        lo, up, l22 = B.theorem1_bounds(t)
        assert lo[0] == pytest.approx(s[0] / np.sqrt(1 + tq * tq), rel=1e-14)
        assert lo[0] <= L[0, 0] <= lo[0] * (1 + 0.25 * tq * tq + 1e-14)
        for rho in ("fro", 2):
            bq, bp = B.theorem3_bounds(t, A, rho)
            a = np.linalg.norm(A, rho)
            assert bq == pytest.approx(s[1] + a * tq, rel=1e-14)
            assert bp == pytest.approx(s[1] + a * tp, rel=1e-14)

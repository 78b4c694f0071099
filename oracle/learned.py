"""Oracle side of the learned power-iteration predictor (test infrastructure).

The predictor reads the spectrum of a cheap first sketch and guesses how
many power rounds q the generalised Algorithm 1 needs.  This module gives
the plain fp64 definitions that its training data and tests rest on.

* ``sketch_features`` -- the predictor's input: the singular values of the
  64-column sketch A^T Omega[:, :64] (the same Philox columns that start the
  full sketch), as log10(sigma_i / sigma_1) clamped to [-6, 0] and divided by
  6, followed by k / 256.  The clamp sits where an fp32 sketch still resolves
  the ratio.
* ``qlp_errors`` -- for j = 0..qmax, the error of the method run with q = j:
  e(j) = ||A - Q L P^T||_F / ||A||_F and the error of its rank-k truncation
  e_k(j) = ||A - Q L[:, :k] P[:, :k]^T||_F / ||A||_F (the rank-k
  approximation the QLP factors give).  One run gives all of them: the power
  loop's Q after j rounds *is* the q = j range basis and its product A^T Q
  is the q = j projection, whose QR gives that run's P and L.  Since
  Q L P^T = Q Q^T A, e(j)^2 = 1 - ||A^T Q_j||_F^2 / ||A||_F^2, and because
  the two residuals are orthogonal, e_k(j)^2 = e(j)^2 + ||L[k:, k:]||_F^2 /
  ||A||_F^2 (L lower-triangular: L[:, k:] is its trailing block).  The
  subtraction in e(j)^2 limits both to about sqrt(u) ~ 1.5e-8 absolute.
* ``qlp_errors_diag`` -- the same for A = diag(sigma) (m x n), with the
  products written for the diagonal (O((m + n) d) each).  A Gaussian sketch
  is rotation invariant (the paper's error analysis uses the same fact), so
  for A = U diag(sigma) V^T with orthonormal U, V the error e(j) has the same
  distribution as for diag(sigma): labels for a spectrum can be drawn on the
  diagonal matrix.
* ``label_q`` -- the smallest q in 0..qmax whose rank-k error meets
  e_k(q) <= 1.05 ||sigma_{>k}||_2 / ||sigma||_2 (1.05 x the Eckart-Young
  optimum; errors below the 4e-8 floor of the identity count as met), else
  qmax + 1 ("unreachable").
* ``label_rank`` -- the rank half of the predictor: for a tolerance tol on
  the relative Frobenius error of the rank-k approximation, the smallest k
  of the classes 8, 16, ..., 256 whose Eckart-Young error
  ||sigma_{>k}|| / ||sigma|| is at most tol / 1.05 (else the last class).
  A rank-k QLP approximation run with the q that label_q asks for is within
  1.05 x that optimum, so the pair (k, q) meets tol.  The rank network
  reads the same 64 sketch features with rank_feature(tol) in place of
  k / 256.
* ``rank_errors`` -- e_k = ||A - Q L[:, :k] P[:, :k]^T||_F / ||A||_F for
  k = 1..d, written out with the dense residual (the plain definition), and
  ``smallest_rank`` -- the first k with e_k <= tol.
"""
import numpy as np

from .philox import gaussian_matrix
from .randqlp import qr_pos, sketch_width

NFEAT_SIGMA = 64
FEAT_CLAMP = 6.0
RANK_CLASSES = (8, 16, 32, 64, 128, 256)
RANK_SLACK = 1.05
ERR_FLOOR = 4e-8   # ~2 sqrt(u): resolution of 1 - ||A^T Q||^2 / ||A||^2


def features_from_sigma(s, k):
    """Normalised log-spectrum features (65 values) from singular values s."""
    s = np.sort(np.asarray(s, dtype=np.float64))[::-1]
    f = np.full(NFEAT_SIGMA, -1.0)
    if s.size and s[0] > 0:
        r = s[:NFEAT_SIGMA] / s[0]
        with np.errstate(divide="ignore"):
            lg = np.log10(np.maximum(r, 0.0))
        f[:r.size] = np.clip(lg, -FEAT_CLAMP, 0.0) / FEAT_CLAMP
    return np.concatenate([f, [k / 256.0]])


def sketch_features(A, k, seed):
    """Features of the dense matrix A: spectrum of A^T Omega[:, :64]."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    omega = gaussian_matrix(m, NFEAT_SIGMA, seed, stream=0)
    s = np.linalg.svd(A.T @ omega, compute_uv=False)
    return features_from_sigma(s, k)


def sketch_features_diag(sigma, m, n, k, seed):
    """sketch_features for A = diag(sigma) (m x n, len(sigma) <= min(m, n))."""
    sigma = np.asarray(sigma, dtype=np.float64)
    r = sigma.size
    omega = gaussian_matrix(m, NFEAT_SIGMA, seed, stream=0)
    Y = sigma[:, None] * omega[:r, :]          # nonzero rows of A^T Omega
    s = np.linalg.svd(Y, compute_uv=False)
    return features_from_sigma(s, k)


def _errors_from_projection(W, nrm2, k):
    """(e, e_k) from the projection W = A^T Q of one run (see the header)."""
    e2 = max(0.0, 1.0 - float(np.sum(W * W)) / nrm2)
    _, R = qr_pos(W)                            # P R = W, L = R^T
    L = R.T
    ek2 = e2 + float(np.sum(L[k:, k:] ** 2)) / nrm2
    return np.sqrt(e2), np.sqrt(ek2)


def qlp_errors(A, k, p, qmax, seed):
    """(e, e_k), arrays over q = 0..qmax, of the method on the dense A."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    d = sketch_width(m, n, k, p)
    nrm2 = float(np.sum(A * A))
    omega = gaussian_matrix(m, d, seed, stream=0)
    qbar, _ = qr_pos(A.T @ omega)
    e, ek = [], []
    for j in range(qmax + 1):
        Q, _ = qr_pos(A @ qbar)                 # range basis of the q = j method
        W = A.T @ Q                             # its projection
        a, b = _errors_from_projection(W, nrm2, k)
        e.append(a)
        ek.append(b)
        if j < qmax:
            qbar, _ = qr_pos(W)                 # next power round
    return np.array(e), np.array(ek)


def qlp_errors_diag(sigma, m, n, k, p, qmax, seed):
    """qlp_errors for A = diag(sigma) (m x n); only the len(sigma) leading
    rows of every panel are nonzero, so the products act on those rows."""
    sigma = np.asarray(sigma, dtype=np.float64)
    r = sigma.size
    d = sketch_width(m, n, k, p)
    nrm2 = float(np.sum(sigma * sigma))
    omega = gaussian_matrix(m, d, seed, stream=0)
    qbar, _ = qr_pos(sigma[:, None] * omega[:r, :])   # A^T Omega, leading rows
    e, ek = [], []
    for j in range(qmax + 1):
        Q, _ = qr_pos(sigma[:, None] * qbar)            # A Qbar
        W = sigma[:, None] * Q                          # A^T Q
        a, b = _errors_from_projection(W, nrm2, k)
        e.append(a)
        ek.append(b)
        if j < qmax:
            qbar, _ = qr_pos(W)
    return np.array(e), np.array(ek)


def optimal_error(sigma, k):
    """Eckart-Young: ||A - A_k||_F / ||A||_F from the singular values."""
    s = np.sort(np.asarray(sigma, dtype=np.float64))[::-1]
    return float(np.sqrt(np.sum(s[k:] ** 2) / np.sum(s ** 2)))


def label_q(errs, sigma, k, slack=1.05):
    """Smallest q with errs[q] <= slack * optimal_error(sigma, k) (errs: the
    rank-k errors e_k); len(errs) if none."""
    target = max(slack * optimal_error(sigma, k), ERR_FLOOR)
    for j, e in enumerate(errs):
        if e <= target:
            return j
    return len(errs)


def rank_feature(tol):
    """The rank network's last input: -log10(tol) clamped to [0, 6], / 6."""
    return float(np.clip(-np.log10(tol), 0.0, FEAT_CLAMP) / FEAT_CLAMP)


def rank_features(feat, tol):
    """Rank-network input from the predictor's features (the 64 spectrum
    values, then rank_feature(tol))."""
    feat = np.asarray(feat, dtype=np.float64)
    return np.concatenate([feat[:NFEAT_SIGMA], [rank_feature(tol)]])


def label_rank(sigma, tol, classes=RANK_CLASSES, slack=RANK_SLACK):
    """Smallest class c with optimal_error(sigma, classes[c]) <= tol / slack;
    the last class if none."""
    for c, k in enumerate(classes):
        if optimal_error(sigma, k) <= tol / slack:
            return c
    return len(classes) - 1


def rank_errors(A, Q, L, P):
    """e_k for k = 1..d from the dense residual of each truncation."""
    A = np.asarray(A, dtype=np.float64)
    nrm = np.linalg.norm(A)
    d = L.shape[0]
    return np.array([np.linalg.norm(A - Q @ (L[:, :k] @ P[:, :k].T)) / nrm
                     for k in range(1, d + 1)])


def smallest_rank(errs, tol):
    """First k (1-based) with errs[k - 1] <= tol, or len(errs) if none."""
    for i, e in enumerate(errs):
        if e <= tol:
            return i + 1
    return len(errs)

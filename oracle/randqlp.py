"""Rand-QLP, fp64, step by step -- oracle side (test infrastructure only).

Algorithm 1 (Section 3.1) factors an m x n matrix A as A = Q L P^T:
  Omega = randn(m, n)
  Qbar  = orth(A^T Omega)
  Q     = orth(A Qbar)
  P R   = (Q^T A)^T,   L := R^T.
Readings taken here (the paper leaves them open):
* Truncation and power iterations: Omega has d = min(k + p, m, n) columns;
  between the first orth and the range basis, q rounds of
  Q = orth(A Qbar), Qbar = orth(A^T Q) re-orthonormalise after every product.
  q = 0 and d = n is exactly Algorithm 1.
* ``orth`` is the reduced, unpivoted QR (Section 2 recalls it for Gram-Schmidt
  or Householder), and every R is normalised to a non-negative diagonal so
  that Q, L, P are unique for full-rank sketches.  numpy's LAPACK
  Householder QR is the library primitive for that step.
"""
import numpy as np

from .philox import gaussian_matrix


def sketch_width(m, n, k, p):
    """d = min(k + p, m, n): the number of sketch columns actually used."""
    return int(max(0, min(k + p, m, n)))


def qr_pos(X):
    """Reduced unpivoted QR with diag(R) >= 0 (sign(0) taken as +1)."""
    Q, R = np.linalg.qr(np.asarray(X, dtype=np.float64), mode="reduced")
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s[None, :], R * s[:, None]


def randqlp(A, k, p, q, seed, return_steps=False):
    """Generalised Algorithm 1 in fp64.  Returns (Q, L, P).

    Q is m x d, L is d x d lower-triangular with L[i, i] >= 0, P is n x d.
    With return_steps, also returns a dict of the intermediate panels.
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    d = sketch_width(m, n, k, p)
    omega = gaussian_matrix(m, d, seed, stream=0)          # randn step
    qbar, _ = qr_pos(A.T @ omega)                          # orth(A^T Omega)
    for _ in range(q):                                     # power iterations
        qq, _ = qr_pos(A @ qbar)
        qbar, _ = qr_pos(A.T @ qq)
    Q, _ = qr_pos(A @ qbar)                                # orth(A Qbar)
    P, R = qr_pos(A.T @ Q)                                 # P R = (Q^T A)^T
    L = R.T.copy()                                         # L := R^T
    if return_steps:
        return Q, L, P, {"omega": omega, "qbar": qbar, "d": d}
    return Q, L, P


def rel_error(A, Q, L, P):
    """||A - Q L P^T||_F / ||A||_F, formed explicitly in fp64."""
    A = np.asarray(A, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    L = np.asarray(L, dtype=np.float64)
    P = np.asarray(P, dtype=np.float64)
    nrm = np.linalg.norm(A)
    res = np.linalg.norm(A - Q @ (L @ P.T))
    return res / nrm if nrm > 0 else res


def subspace_sine(X, Y):
    """Sine of the largest canonical angle between range(X) and range(Y).

    X and Y have orthonormal columns and the same column count.  Computed
    directly as ||Y - X (X^T Y)||_2 (no 1 - cos^2 cancellation).
    """
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    if X.shape[1] == 0:
        return 0.0
    return float(np.linalg.norm(Y - X @ (X.T @ Y), 2))


def orth_error(Q):
    """max |Q^T Q - I| entry."""
    Q = np.asarray(Q, dtype=np.float64)
    return float(np.abs(Q.T @ Q - np.eye(Q.shape[1])).max()) if Q.shape[1] else 0.0

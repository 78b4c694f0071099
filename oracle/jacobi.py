"""One-sided (Hestenes) Jacobi SVD for tiny matrices -- brute-force checker.

Used to obtain singular values of small test matrices and of blocks of L
without calling LAPACK's SVD, so that statements about singular values
(Theorem 1, interlacing) are checked by an independent route.  Plain loops;
meant for at most ~64 x 64.
"""
import math

import numpy as np


def jacobi_singular_values(A, tol=1e-15, max_sweeps=60):
    """Singular values of A (descending), via rotations of column pairs.

    Rotates pairs of columns of a working copy until every pair is
    numerically orthogonal; the column norms are then the singular values.
    """
    W = np.array(A, dtype=np.float64, copy=True)
    if W.shape[0] < W.shape[1]:
        W = W.T.copy()
    ncol = W.shape[1]
    for _ in range(max_sweeps):
        rotated = False
        for i in range(ncol - 1):
            for j in range(i + 1, ncol):
                a = float(W[:, i] @ W[:, i])
                b = float(W[:, j] @ W[:, j])
                c = float(W[:, i] @ W[:, j])
                if c == 0.0 or abs(c) <= tol * math.sqrt(a * b):
                    continue
                rotated = True
                zeta = (b - a) / (2.0 * c)
                t = math.copysign(1.0, zeta) / (abs(zeta) + math.sqrt(1.0 + zeta * zeta))
                cs = 1.0 / math.sqrt(1.0 + t * t)
                sn = cs * t
                wi = W[:, i].copy()
                W[:, i] = cs * wi - sn * W[:, j]
                W[:, j] = sn * wi + cs * W[:, j]
        if not rotated:
            break
    s = np.sqrt(np.sum(W * W, axis=0))
    return np.sort(s)[::-1]

"""Per-sample quantities of Theorems 1-3 (Section 4.1) -- oracle side.

Given the generator's exact SVD A = U diag(sigma) V^T and the Gaussian
matrix actually used, the theorems' right-hand sides are numbers that a
computed factorisation must respect:

  Omega_1 = first k columns of Omega,  Omega~ = U^T Omega_1 = [Om1; Om2],
  M = Om2 Om1^{-1},  psi_i = sigma_{k+1} / sigma_i.

Theorem 1: sigma_i >= sigma_i(L11) >= sigma_i / sqrt(1 + psi_i^4 ||M||^2),
           ||L22||_2 <= (1 + psi_k^2 ||M||) sigma_{k+1}.
Theorem 2: sin theta_Q <= psi_k^2 ||M||,  sin theta_P <= psi_k^3 ||M||, and
           for the trailing subspaces (only meaningful at d = n)
           sin phi_Q <= psi_k^2 ||M|| / sqrt(1 + psi_k^4 ||M||^2),
           sin phi_P <= psi_k^3 ||M|| / sqrt(1 + psi_k^6 ||M||^2).
Theorem 3: ||(I - Q_k Q_k^T) A||_rho <= ||Sigma_perp||_rho + ||A||_rho psi_k^2 ||M||,
           ||A (I - P_k P_k^T)||_rho <= ||Sigma_perp||_rho + ||A||_rho psi_k^3 ||M||.

Readings: Theorem 1's sigma-hat are the singular values of L11 (the proof
bounds those, not the diagonal entries); the printed phi bounds carry
||M||^2 in the numerator and a repeated "phi_Q", while the proof yields
||M|| and phi_P, which is what is used.  With q power iterations the same
proofs go through with (A A^T)^(q+1) in place of A A^T, so every psi
exponent e_Q = 2 becomes 2(q+1) and every e_P = 3 becomes 2q+3 (the sigma
lower bound uses 2 e_Q).  At q = 0 these are the printed exponents.
"""
import numpy as np


def theorem_quantities(U, sigma, omega, k, q=0):
    """Return a dict with ||M||, psi and the exponents for split k.

    U: m x r orthonormal (r > k), sigma: r values (descending), omega: m x d.
    Only the r directions with a listed singular value enter M; directions
    with sigma = 0 would only shrink the bounds.
    """
    U = np.asarray(U, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    om1 = np.asarray(omega, dtype=np.float64)[:, :k]
    omt = U.T @ om1
    om_1, om_2 = omt[:k, :], omt[k:, :]
    M = om_2 @ np.linalg.inv(om_1)
    mnorm = float(np.linalg.norm(M, 2)) if M.size else 0.0
    psi = sigma[k] / sigma[:k]
    return {"M": mnorm, "psi": psi, "eQ": 2 * (q + 1), "eP": 2 * q + 3,
            "sigma": sigma, "k": k}


def theorem1_bounds(t):
    """(lower, upper) arrays for sigma_i(L11) and the ||L22||_2 bound."""
    s, psi, M, eQ, k = t["sigma"], t["psi"], t["M"], t["eQ"], t["k"]
    lower = s[:k] / np.sqrt(1.0 + psi ** (2 * eQ) * M * M)
    upper = s[:k].copy()
    l22 = (1.0 + psi[k - 1] ** eQ * M) * s[k]
    return lower, upper, l22


def theorem2_bounds(t):
    """Upper bounds for sin theta_Q, sin theta_P, sin phi_Q, sin phi_P."""
    psik, M, eQ, eP = t["psi"][-1], t["M"], t["eQ"], t["eP"]
    tq = psik ** eQ * M
    tp = psik ** eP * M
    return {"theta_Q": tq, "theta_P": tp,
            "phi_Q": tq / np.sqrt(1.0 + tq * tq),
            "phi_P": tp / np.sqrt(1.0 + tp * tp)}


def theorem3_bounds(t, A, rho):
    """Upper bounds for the rank-k errors in norm rho ('fro' or 2)."""
    s, k, psik, M, eQ, eP = t["sigma"], t["k"], t["psi"][-1], t["M"], t["eQ"], t["eP"]
    tail = s[k:]
    if rho == 2:
        tail_norm = float(tail.max()) if tail.size else 0.0
        a_norm = float(s[0])
    else:
        tail_norm = float(np.sqrt(np.sum(tail ** 2)))
        a_norm = float(np.linalg.norm(A))
    return (tail_norm + a_norm * psik ** eQ * M,
            tail_norm + a_norm * psik ** eP * M)

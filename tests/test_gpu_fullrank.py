"""Algorithm 1 itself (Section 3.1): the full-rank factorisation, d = n and
no power rounds, on the GPU against the fp64 oracle.

With d = min(m, n) the factors reconstruct A (A = Q L P^T up to rounding)
and L = Q^T A P has A's singular values.  The sketch Omega is a square (or
nearly square) Gaussian, so the first panel A^T Omega carries Omega's
condition number (about n) on top of A's: the panel QR goes through the
shifted Cholesky QR when needed (on these matrices the fast path holds).
Compared: reconstruction error, sigma(L)
against sigma(A) (LAPACK's SVD of A), orthogonality, L = Q^T A P, the
diagonal of L and the dominant singular directions against the oracle.
"""
import numpy as np
import pytest

import workloads as W
from oracle import randqlp, rel_error, subspace_sine
from tests.gpu_util import invariants, log, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rq():
    import paper_2110_01011_amd as rq
    rq.lib()
    return rq


def _full_rank(rq, A, seed):
    m, n = A.shape
    d = min(m, n)
    Qg, Lg, Pg, info = rq.factor(to_dev(A), d, 0, 0, seed, return_info=True)
    Qg, Lg, Pg = to_np(Qg), to_np(Lg), to_np(Pg)
    Qo, Lo, Po = randqlp(A, d, 0, 0, seed)
    sA = np.linalg.svd(A, compute_uv=False)
    sL = np.linalg.svd(Lg, compute_uv=False)
    inv = invariants(A, Qg, Lg, Pg)
    out = {
        "e_gpu": rel_error(A, Qg, Lg, Pg), "e_orc": rel_error(A, Qo, Lo, Po),
        "sigma_L_vs_A": float(np.abs(sL - sA).max() / sA[0]),
        "dsigma": float(np.abs(np.diag(Lg) - np.diag(Lo)).max() / Lo[0, 0]),
        "dsigma_lead": float(np.abs(np.diag(Lg)[:8] - np.diag(Lo)[:8]).max() / Lo[0, 0]),
        "sinQ1": subspace_sine(Qo[:, :1], Qg[:, :1]), "sinP1": subspace_sine(Po[:, :1], Pg[:, :1]),
        "kappa": float(sA[0] / sA[-1]), **inv, "info": info}
    log(f"  {m}x{n} d={d}: {out}")
    return out


@pytest.mark.parametrize("n", [300, 1100, 2000])
def test_full_rank_uniform(rq, n):
    """Section 5.1's random test matrices: dense uniform(0, 1) entries."""
    log(f"full rank uniform(0,1) {n}x{n}")
    A = W.uniform01(n, n, seed=n)
    r = _full_rank(rq, A, seed=1)
    assert r["e_gpu"] < 1e-13 and abs(r["e_gpu"] - r["e_orc"]) < 1e-13
    assert r["sigma_L_vs_A"] < 1e-12
    assert r["orthQ"] < 1e-12 and r["orthP"] < 1e-12
    assert r["upper_max"] == 0.0 and r["min_diag"] >= 0.0
    assert r["L_vs_QtAP"] < 1e-12
    # the diagonal of L (the approximate singular values) and the dominant
    # directions (sigma_1 ~ n/2, far above the rest) at the fp64 bar
    assert r["dsigma"] < 1e-10
    assert r["sinQ1"] < 1e-10 and r["sinP1"] < 1e-10


@pytest.mark.parametrize("m,n", [(1500, 1500), (2600, 1300), (1200, 2300)])
def test_full_rank_well_conditioned(rq, m, n):
    """sigma linear from 1 to 0.1: every quantity at the fp64 bar."""
    log(f"full rank well conditioned {m}x{n}")
    A, U, s, V = W.svd_matrix(m, n, np.linspace(1.0, 0.1, min(m, n)), seed=m + n)
    r = _full_rank(rq, A, seed=2)
    assert r["e_gpu"] < 1e-13 and r["sigma_L_vs_A"] < 1e-12
    assert r["dsigma"] < 1e-10 and r["sinQ1"] < 1e-10 and r["sinP1"] < 1e-10
    assert r["orthQ"] < 1e-12 and r["orthP"] < 1e-12 and r["L_vs_QtAP"] < 1e-12

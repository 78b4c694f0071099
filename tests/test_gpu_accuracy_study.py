"""Section 5.2's rank-revealing study through the GPU path: the four
n = 1000 test families (LowRankPlusNoise, LowRankFastDecay, S-shaped decay,
LowRankSlowDecay), factored by Algorithm 1 (d = n, q = 0) and by the
truncated form (k = 20, p = 5, q = 1), with the approximate singular
values diag(L), sigma(L11), ||L22||, the subspace angles and the rank-k
approximation errors Q L[:, :k] P[:, :k]^T in the 2- and Frobenius norms
checked against the SVD and against Theorems 1-3 evaluated for each sample
(its own Omega and the exact singular vectors from LAPACK's SVD of A)."""
import numpy as np
import pytest

import workloads as W
from oracle import bounds as B
from oracle import jacobi_singular_values, randqlp, subspace_sine
from oracle.philox import gaussian_matrix
from tests.gpu_util import log, to_dev, to_np

pytestmark = pytest.mark.gpu
N = 1000
FAMILIES = ["low_rank_plus_noise", "fast_decay", "s_shaped", "slow_decay"]


@pytest.fixture(scope="module")
def rq():
    import paper_2110_01011_amd as rq
    rq.lib()
    return rq


def _family(name, seed):
    if name == "low_rank_plus_noise":
        return W.paper_low_rank_plus_noise(N, seed)
    if name == "fast_decay":
        return W.fast_decay(N, N, seed)[0]
    if name == "s_shaped":
        return W.s_shaped(N, seed)[0]
    return W.slow_decay(N, seed)[0]


@pytest.fixture(scope="module", params=FAMILIES)
def family(request):
    A = _family(request.param, seed=5)
    U, s, Vt = np.linalg.svd(A)
    return request.param, A, U, s, Vt.T


KS = (1, 2, 5, 10, 20, 50, 100, 200, 500)


@pytest.mark.parametrize("k,p,q", [(N, 0, 0), (20, 5, 1)])
def test_rank_revealing_study(rq, family, k, p, q):
    name, A, U, s, V = family
    seed = 11
    Qg, Lg, Pg = (to_np(t) for t in rq.factor(to_dev(A), k, p, q, seed))
    d = Lg.shape[0]
    Qo, Lo, Po = randqlp(A, k, p, q, seed)
    nrmF, nrm2 = np.linalg.norm(A), s[0]
    sig_hat = np.abs(np.diag(Lg))
    rows = []
    for kk in [x for x in KS if x < d]:
        Ak = Qg @ (Lg[:, :kk] @ Pg[:, :kk].T)
        Ako = Qo @ (Lo[:, :kk] @ Po[:, :kk].T)
        eF, e2 = np.linalg.norm(A - Ak) / nrmF, np.linalg.norm(A - Ak, 2) / nrm2
        eFo = np.linalg.norm(A - Ako) / nrmF
        optF, opt2 = np.sqrt(np.sum(s[kk:] ** 2)) / nrmF, s[kk] / nrm2
        rows.append((kk, eF / optF, e2 / opt2 if opt2 > 0 else np.inf))
        # the GPU's rank-k errors are the oracle's (fp64 bar, relative)
        assert abs(eF - eFo) <= 1e-10 * max(eFo, 1e-300) + 1e-13
        # Eckart-Young: no rank-k approximation beats the truncated SVD
        assert eF >= optF * (1 - 1e-12) and e2 >= opt2 * (1 - 1e-12)
    # Theorems 1-3 at the split k of the truncated form (or k = 20 at d = n)
    ks = min(k, 20)
    t = B.theorem_quantities(U, s, gaussian_matrix(N, d, seed, stream=0), ks, q)
    lo, up, l22 = B.theorem1_bounds(t)
    sv = jacobi_singular_values(Lg[:ks, :ks])
    assert np.all(sv <= up * (1 + 1e-10)) and np.all(sv >= lo * (1 - 1e-10))
    assert np.linalg.norm(Lg[ks:, ks:], 2) <= l22 * (1 + 1e-10)
    b2 = B.theorem2_bounds(t)
    sq = subspace_sine(U[:, :ks], Qg[:, :ks])
    sp = subspace_sine(V[:, :ks], Pg[:, :ks])
    assert sq <= b2["theta_Q"] * (1 + 1e-9) + 1e-12 and sp <= b2["theta_P"] * (1 + 1e-9) + 1e-12
    for rho in ("fro", 2):
        bq, bp = B.theorem3_bounds(t, A, rho)
        Qk, Pk = Qg[:, :ks], Pg[:, :ks]
        assert np.linalg.norm(A - Qk @ (Qk.T @ A), rho) <= bq * (1 + 1e-10)
        assert np.linalg.norm(A - (A @ Pk) @ Pk.T, rho) <= bp * (1 + 1e-10)
    lead = min(ks, int(np.sum(s > 1e-12 * s[0])))
    ratio = sig_hat[:lead] / s[:lead]
    log(f"  {name} k={k} p={p} q={q} d={d}: diag(L)/sigma over the leading {lead}: "
        f"[{ratio.min():.3f}, {ratio.max():.3f}]; sinQ {sq:.2e} (bound {b2['theta_Q']:.2e}) "
        f"sinP {sp:.2e} (bound {b2['theta_P']:.2e}); ||L22|| {np.linalg.norm(Lg[ks:, ks:], 2):.3e} "
        f"(bound {l22:.3e}); rank-k error / optimum (F, 2): "
        + ", ".join(f"k={a}: {b:.3f}/{c:.3f}" for a, b, c in rows))
    # the only diagonal entry the theory fixes: L11 <= sigma_1
    assert sig_hat[0] <= s[0] * (1 + 1e-12)

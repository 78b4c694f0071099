"""randqlp_factor_noalloc (static device scratch, nothing allocated) against
randqlp_factor (caller workspace) on the same inputs: two calls in a row, the
second on a smaller matrix, so a stale first call in the shared scratch
would show."""
import numpy as np
import pytest

import workloads as W
from oracle import rel_error, subspace_sine
from tests.gpu_util import invariants, log, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rq():
    import paper_2110_01011_amd as rq
    rq.lib()
    return rq


CASES = [  # (m, n, k, p, q, seed): the second call is smaller than the first
    (1500, 1200, 40, 10, 2, 3),
    (700, 500, 12, 5, 1, 4),
]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_matches_factor_two_calls(rq, dtype):
    import torch
    tdt = torch.float64 if dtype == "f64" else torch.float32
    for (m, n, k, p, q, seed) in CASES:
        log(f"noalloc {dtype} {m}x{n} k={k} p={p} q={q} seed={seed}")
        A, U, s, V = W.poly_decay(m, n, 1.0, seed=seed)
        Ad = to_dev(A, tdt)
        Qr, Lr, Pr = (to_np(t) for t in rq.factor(Ad, k, p, q, seed))
        Qg, Lg, Pg, info = rq.factor_noalloc(Ad, k, p, q, seed, return_info=True)
        torch.cuda.synchronize()
        Qg, Lg, Pg = to_np(Qg), to_np(Lg), to_np(Pg)
        d = Lr.shape[0]
        assert info["d"] == d and info["q_used"] == q
        e_r, e_g = rel_error(A, Qr, Lr, Pr), rel_error(A, Qg, Lg, Pg)
        diff = max(np.abs(Qg - Qr).max(), np.abs(Pg - Pr).max(),
                   np.abs(Lg - Lr).max() / Lr[0, 0])
        same = np.array_equal(Qg, Qr) and np.array_equal(Lg, Lr) and np.array_equal(Pg, Pr)
        sines = [subspace_sine(Qr[:, :k], Qg[:, :k]), subspace_sine(Pr[:, :k], Pg[:, :k]),
                 subspace_sine(Qr, Qg), subspace_sine(Pr, Pg)]
        log(f"  e {e_g:.6e} vs {e_r:.6e}; max elementwise diff {diff:.2e}; bitwise {same}; "
            f"sines {max(sines):.2e}")
        if dtype == "f64":
            tol = 1e-10
            assert abs(e_g - e_r) <= tol
            assert np.abs(np.diag(Lg) - np.diag(Lr)).max() / Lr[0, 0] <= tol
            assert max(sines) <= tol
            inv = invariants(A, Qg, Lg, Pg)
            assert inv["orthQ"] < 1e-12 and inv["orthP"] < 1e-12
            assert inv["upper_max"] == 0.0 and inv["min_diag"] >= 0.0
        else:
            assert e_g <= 1.05 * e_r
            assert diff <= 1e-4

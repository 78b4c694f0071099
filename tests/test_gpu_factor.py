"""GPU parity of the whole factorisation (randqlp_factor) against the oracle.

fp64: the sign-invariant quantities -- relative error ||A - Q L P^T||_F /
||A||_F, the diagonal of L (relative to its first entry) and the subspace
sines of Q and P (leading k columns and all d) -- agree with the oracle to
1e-10.  fp32: the error stays within 1.05x the fp64 oracle's.
"""
import numpy as np
import pytest

import workloads as W
from oracle import jacobi_singular_values, randqlp, rel_error
from tests.gpu_util import compare, invariants, log, to_dev, to_np

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module")
def rq():
    import paper_2110_01011_amd as rq
    rq.lib()
    return rq


def _run(rq, A, k, p, q, seed, dtype=None, panel="auto", precision=None):
    import torch
    dt = dtype or torch.float64
    Q, L, P, info = rq.factor(to_dev(A, dt), k, p, q, seed, panel=panel, precision=precision,
                              return_info=True)
    return to_np(Q), to_np(L), to_np(P), info


def _check_f64(rq, A, k, p, q, seed, tol=TOL, panel="auto"):
    Qg, Lg, Pg, info = _run(rq, A, k, p, q, seed, panel=panel)
    Qo, Lo, Po = randqlp(A, k, p, q, seed)
    c = compare(A, Qg, Lg, Pg, Qo, Lo, Po, min(k, Lo.shape[0]))
    inv = invariants(A, Qg, Lg, Pg)
    log(f"  {c} {inv} {info}")
    assert c["de"] <= tol and c["dsigma"] <= tol
    assert c["sinQk"] <= tol and c["sinPk"] <= tol
    assert c["sinQ"] <= tol and c["sinP"] <= tol
    assert inv["orthQ"] < 1e-12 and inv["orthP"] < 1e-12
    assert inv["upper_max"] == 0.0 and inv["min_diag"] >= 0.0
    assert inv["L_vs_QtAP"] < 1e-12
    return Qg, Lg, Pg, info


def test_c1_fast_decay_parity(rq):
    """1000 x 1000, sigma_i = i^-2, k = 20, p = 5, q = 1 (Section 5.2 family)."""
    log("factor C1 1000x1000 k=20 p=5 q=1")
    A, U, s, V = W.fast_decay(1000, 1000, seed=0)
    for seed in (0, 1):
        _check_f64(rq, A, 20, 5, 1, seed)


@pytest.mark.parametrize("m,n,k,p,q", [(777, 555, 30, 7, 2), (300, 900, 12, 4, 1),
                                       (640, 640, 60, 4, 0), (2049, 1500, 100, 10, 1),
                                       (100, 80, 1, 0, 3), (4000, 3000, 200, 10, 2)])
def test_ragged_shapes_parity(rq, m, n, k, p, q):
    log(f"factor ragged m={m} n={n} k={k} p={p} q={q}")
    sig = np.concatenate([np.linspace(3.0, 1.0, k), 0.5 * 0.97 ** np.arange(min(m, n) - k)])
    A, U, s, V = W.svd_matrix(m, n, sig, seed=m + n)
    _check_f64(rq, A, k, p, q, seed=7)


def test_rank_plus_noise_parity(rq):
    """The 8000 x 8000 workload's family at 2000 x 2000: rank 50 + noise."""
    log("factor rank+noise 2000x2000 r=50 k=50 p=10 q=2")
    A, s = W.rank_plus_noise(2000, 2000, 50, 1e-3, seed=1)
    _check_f64(rq, A, 50, 10, 2, seed=3)


def test_f32_error_within_5_percent(rq):
    import torch
    log("factor f32 1000x1000 fast decay")
    A, U, s, V = W.fast_decay(1000, 1000, seed=0)
    Qo, Lo, Po = randqlp(A, 20, 5, 1, 0)
    e_o = rel_error(A, Qo, Lo, Po)
    Qg, Lg, Pg, info = _run(rq, A, 20, 5, 1, 0, dtype=torch.float32)
    e_g = rel_error(A, Qg, Lg, Pg)
    inv = invariants(A.astype(np.float32).astype(np.float64), Qg, Lg, Pg)
    log(f"  e_gpu={e_g} e_orc={e_o} {inv}")
    assert e_g <= 1.05 * e_o
    assert inv["orthQ"] < 1e-5 and inv["orthP"] < 1e-5
    assert inv["upper_max"] == 0.0 and inv["min_diag"] >= 0.0


def test_full_width_reconstructs(rq):
    """d = min(m, n): A = Q L P^T exactly (Gaussian sketches are square)."""
    for (m, n) in [(60, 60), (200, 120)]:
        log(f"factor full width {m}x{n}")
        A = W.uniform01(m, n, seed=m)
        Qg, Lg, Pg, info = _run(rq, A, min(m, n), 0, 0, 4)
        assert rel_error(A, Qg, Lg, Pg) < 1e-11
        inv = invariants(A, Qg, Lg, Pg)
        assert inv["orthQ"] < 1e-12 and inv["orthP"] < 1e-12
        if m == n:
            assert np.allclose(jacobi_singular_values(Lg), jacobi_singular_values(A), rtol=1e-9)


def test_scaled_orthonormal_gives_scaled_identity(rq):
    Uo = W.haar(300, 40, seed=4, stream=9)
    Qg, Lg, Pg, info = _run(rq, 2.5 * Uo, 30, 10, 1, 8)
    assert np.abs(Lg - 2.5 * np.eye(40)).max() < 1e-12


def test_exact_low_rank_and_zero_matrix(rq):
    sig = np.array([4.0, 2.0, 1.0, 0.5, 0.25, 0.1])
    A, U, s, V = W.svd_matrix(200, 150, sig, seed=6)
    Qg, Lg, Pg, info = _run(rq, A, 8, 4, 1, 3)
    log(f"  low rank info={info}")
    assert rel_error(A, Qg, Lg, Pg) < 1e-13
    assert np.allclose(jacobi_singular_values(Lg[:6, :6]), sig, rtol=1e-10)
    inv = invariants(A, Qg, Lg, Pg)
    assert inv["orthQ"] < 1e-12 and inv["orthP"] < 1e-12
    Z = np.zeros((120, 90))
    Qg, Lg, Pg, info = _run(rq, Z, 10, 2, 1, 0)
    log(f"  zero info={info}")
    assert np.all(Lg == 0.0)
    inv = invariants(Z, Qg, Lg, Pg)
    assert inv["orthQ"] < 1e-12 and inv["orthP"] < 1e-12


def test_nonfinite_input_is_reported(rq):
    A = np.random.default_rng(0).standard_normal((100, 80))
    A[17, 33] = np.nan
    with pytest.raises(rq.RandQLPError) as ei:
        _run(rq, np.asfortranarray(A), 5, 2, 1, 0)
    assert ei.value.status == 2
    A[17, 33] = np.inf
    with pytest.raises(rq.RandQLPError):
        _run(rq, np.asfortranarray(A), 5, 2, 1, 0)


def test_bitwise_repeatable_and_prefix_property(rq):
    A, U, s, V = W.fast_decay(900, 700, seed=2)
    a = _run(rq, A, 10, 12, 1, 7)
    b = _run(rq, A, 10, 12, 1, 7)
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)
    c = _run(rq, A, 10, 0, 1, 7)
    assert np.abs(np.abs(c[0]) - np.abs(a[0][:, :10])).max() < 1e-12
    assert np.abs(c[1] - a[1][:10, :10]).max() < 1e-12 * a[1][0, 0]


@pytest.mark.parametrize("panel", ["robust", "cholqr2"])
def test_explicit_panel_modes_parity(rq, panel):
    A, U, s, V = W.fast_decay(500, 400, seed=3)
    _check_f64(rq, A, 20, 5, 1, 2, panel=panel)


@pytest.fixture(scope="module")
def exp_decay_matrix():
    """The precision-form workload's family at 1/4 scale: sigma_i = exp(-i/100)."""
    return W.exp_decay(5000, 4000, 1000, 100.0, seed=3)


def test_wide_sketch_blocked_cholesky_parity(rq, exp_decay_matrix):
    """d = 520 > 224 exercises the blocked Cholesky (tile kernel + Schur steps)."""
    log("factor exp-decay 5000x4000 k=500 p=20 q=2 (d=520) fp64")
    A, U, s, V = exp_decay_matrix
    _check_f64(rq, A, 500, 20, 2, seed=1)


@pytest.mark.parametrize("precision", ["bf16", "f16", "bf16x3"])
def test_precision_form_error_within_5_percent(rq, exp_decay_matrix, precision):
    import torch
    log(f"factor exp-decay 5000x4000 d=520 precision={precision}")
    A, U, s, V = exp_decay_matrix
    Qo, Lo, Po = randqlp(A, 500, 20, 2, 1)
    e_o = rel_error(A, Qo, Lo, Po)
    Qg, Lg, Pg, info = _run(rq, A, 500, 20, 2, 1, dtype=torch.float32, precision=precision)
    e_g = rel_error(A, Qg, Lg, Pg)
    inv = invariants(A, Qg, Lg, Pg)
    log(f"  e_gpu={e_g:.6e} e_orc={e_o:.6e} ratio={e_g / e_o:.5f} {inv} {info}")
    assert e_g <= 1.05 * e_o
    assert inv["orthQ"] < 1e-5 and inv["orthP"] < 1e-5
    assert inv["upper_max"] == 0.0 and inv["min_diag"] >= 0.0


@pytest.mark.slow
def test_c2_full_size_parity(rq):
    """8000 x 8000 rank-200 + noise, k = 200, p = 10, q = 2: fp64 and fp32."""
    import torch
    log("factor C2 8000x8000 k=200 p=10 q=2")
    A, s = W.rank_plus_noise(8000, 8000, 200, 1e-3, seed=0)
    Qg, Lg, Pg, info = _check_f64(rq, A, 200, 10, 2, 0)
    Qo, Lo, Po = randqlp(A, 200, 10, 2, 0)
    e_o = rel_error(A, Qo, Lo, Po)
    Q32, L32, P32, info32 = _run(rq, A, 200, 10, 2, 0, dtype=torch.float32)
    e32 = rel_error(A, Q32, L32, P32)
    log(f"  C2 f32 e={e32} oracle e={e_o}")
    assert e32 <= 1.05 * e_o


@pytest.mark.slow
def test_c3_full_size_precision_forms_vs_oracle(rq):
    """20000 x 16000, sigma_i = exp(-i/100) (rank 4000), k = 500, p = 20,
    q = 2 (d = 520): the fp64 form at the fp64 bar against the oracle on the
    same matrix; the bf16x3, bf16, f16 and fp32 forms within 1.05x the
    oracle's error (computed in fp64 against the fp64 A)."""
    import torch
    log("factor C3 20000x16000 k=500 p=20 q=2 (d=520): generating on the device")
    A64 = rq.colmajor(W.device_exp_decay(20000, 16000, 4000, 100.0, seed=3))
    Ah = A64.cpu().numpy()
    log("  oracle")
    Qo, Lo, Po = randqlp(Ah, 500, 20, 2, 0)
    e_o = rel_error(Ah, Qo, Lo, Po)
    Qg, Lg, Pg, info = rq.factor(A64, 500, 20, 2, 0, return_info=True)
    Qg, Lg, Pg = to_np(Qg), to_np(Lg), to_np(Pg)
    c = compare(Ah, Qg, Lg, Pg, Qo, Lo, Po, 500)
    log(f"  fp64: {c} {info}")
    assert c["de"] <= TOL and c["dsigma"] <= TOL
    assert c["sinQk"] <= TOL and c["sinPk"] <= TOL and c["sinQ"] <= TOL and c["sinP"] <= TOL
    del Qg, Lg, Pg
    A32 = rq.colmajor(A64.float().t().contiguous().t())
    nrm = torch.linalg.norm(A64)
    for prec in ("bf16x3", "bf16", "f16", "f32"):
        Q, L, P = rq.factor(A32, 500, 20, 2, 0, precision=prec)
        e_g = float(torch.linalg.norm(A64 - Q.double() @ (L @ P.double().T)) / nrm)
        log(f"  {prec}: e={e_g:.6e} oracle {e_o:.6e} ratio {e_g / e_o:.5f}")
        assert e_g <= 1.05 * e_o
        del Q, L, P


@pytest.mark.parametrize("scale", [1e6, 1e-6, 3e-30])
def test_f16_form_does_not_depend_on_the_scale_of_A(rq, scale):
    """The fp16 copy of A is scaled by a power of two chosen from max |a|, so
    c A factors with the relative error of A: no overflow to Inf for large
    entries, no underflow for small ones.  The error is against the fp64
    oracle on the unscaled A (the method's relative error does not depend on
    c for the same Omega)."""
    import torch
    A, U, s, V = W.poly_decay(2000, 1500, 1.0, seed=61)
    e_o = rel_error(A, *randqlp(A, 40, 10, 2, 3))
    res = {}
    for c in (1.0, scale):
        Ac = c * A
        Qg, Lg, Pg, info = _run(rq, Ac, 40, 10, 2, 3, dtype=torch.float32, precision="f16")
        res[c] = rel_error(Ac, Qg, Lg, Pg)
        log(f"  f16 scale {c:g}: e={res[c]:.6e} (oracle {e_o:.6e}) {info}")
    assert res[scale] <= 1.05 * e_o
    assert abs(res[scale] / res[1.0] - 1.0) < 1e-3


def test_f16_step_product_with_large_entries(rq):
    """randqlp_gemm in fp16 on entries near 1e6 (beyond fp16's 65504): the
    product comes back in A's units within fp16 rounding."""
    import torch
    r = np.random.default_rng(3)
    A = 1e6 * r.standard_normal((700, 500))
    X = r.standard_normal((700, 30))
    C = to_np(rq.gemm(to_dev(A, torch.float32), to_dev(X, torch.float32), True, precision="f16"))
    ref = A.T @ X
    err = np.abs(C - ref).max() / np.abs(ref).max()
    log(f"  f16 A^T X with |a| ~ 1e6: max rel err {err:.2e}")
    assert np.isfinite(C).all() and err < 5e-3

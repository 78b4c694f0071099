"""GPU parity of the individual steps: the Gaussian sketch matrix, the
sketch/power/projection products, and the panel QR (orth)."""
import numpy as np
import pytest

import workloads as W
from oracle import qr_pos
from oracle.philox import gaussian_matrix
from tests.gpu_util import log, to_dev, to_np

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53
U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def rq():
    import paper_2110_01011_amd as rq
    rq.lib()
    return rq


@pytest.mark.parametrize("m,d,seed,sid", [(1000, 37, 0, 0), (257, 5, 123456789, 0),
                                           (3, 7, 2 ** 63 + 5, 3), (4096, 64, 9, 0)])
def test_gaussian_matches_oracle(rq, m, d, seed, sid):
    import torch
    log(f"gaussian m={m} d={d} seed={seed}")
    ref = gaussian_matrix(m, d, seed, sid)
    g = to_np(rq.gaussian(m, d, seed, sid, torch.float64))
    # same Philox words; log/sqrt/cos/sin may differ from the host libm by an ulp
    assert np.max(np.abs(g - ref)) <= 64 * U64 * max(1.0, np.abs(ref).max())
    g32 = to_np(rq.gaussian(m, d, seed, sid, torch.float32))
    close = np.abs(g32 - ref.astype(np.float32).astype(np.float64))
    assert np.all(close <= 2 * U32 * np.abs(ref) + 1e-30)


SHAPES = [(1000, 700, 25), (333, 517, 210), (64, 64, 1), (2000, 50, 130), (5, 7, 3),
          (129, 1100, 17), (4000, 3000, 210),
          # one row tile, so many k splits of a few 32-deep tiles each (and
          # a ragged tail), with every MFMA block of the tile full (the
          # products whose loads are issued among the MFMAs)
          (70, 300, 210), (97, 3000, 33)]


@pytest.mark.parametrize("m,n,d", SHAPES)
@pytest.mark.parametrize("trans", [1, 0])
def test_gemm_f64_within_rounding_bound(rq, m, n, d, trans):
    log(f"gemm f64 trans={trans} m={m} n={n} d={d}")
    r = np.random.default_rng(m * 7 + n + d)
    A = np.asfortranarray(r.standard_normal((m, n)))
    X = r.standard_normal((m if trans else n, d))
    C = to_np(rq.gemm(to_dev(A), to_dev(X), trans))
    Aop = A.T if trans else A
    ref = Aop @ X
    K = Aop.shape[1]
    bound = 2 * K * U64 * (np.abs(Aop) @ np.abs(X)) + 1e-300
    assert C.shape == ref.shape
    assert np.all(np.abs(C - ref) <= bound)


# Layouts of the fp64 products with A beyond tight, aligned operands: a
# ragged last k-tile with 4 vector-ALU columns, two column tiles, a panel that
# is only 8-byte aligned (the form without direct LDS loads), an A block with
# lda > rows, and two k splits with a ragged end.
STREAM_CASES = [
    dict(m=4100, n=1000, d=212, trans=1),
    dict(m=1000, n=4096, d=300, trans=0),
    dict(m=3000, n=500, d=210, trans=1, x_offset=1),
    dict(m=1000, n=3000, d=64, trans=0, a_rows=1200, a_offset=100),
    dict(m=300, n=2000, d=40, trans=1),
]


@pytest.mark.parametrize("case", STREAM_CASES, ids=lambda c: "-".join(f"{k}{v}" for k, v in c.items()))
def test_gemm_f64_layouts(rq, case):
    import torch
    m, n, d, trans = case["m"], case["n"], case["d"], case["trans"]
    log(f"gemm f64 layout {case}")
    r = np.random.default_rng(m + 3 * n + 7 * d)
    a_rows, a_off = case.get("a_rows", m), case.get("a_offset", 0)
    A_big = np.asfortranarray(r.standard_normal((a_rows, n)))
    A = A_big[a_off:a_off + m]
    K = m if trans else n
    x_off = case.get("x_offset", 0)
    X_big = r.standard_normal((K + x_off, d))
    X = X_big[x_off:]
    Ad = to_dev(A_big)[a_off:a_off + m]
    Xd = to_dev(X_big)[x_off:]
    assert Ad.stride() == (1, a_rows) and Xd.stride() == (1, K + x_off)
    if x_off:
        assert Xd.data_ptr() % 16 == 8
    C = to_np(rq.gemm(Ad, Xd, trans))
    Aop = A.T if trans else A
    ref = Aop @ X
    bound = 2 * K * U64 * (np.abs(Aop) @ np.abs(X)) + 1e-300
    assert C.shape == ref.shape
    assert np.all(np.abs(C - ref) <= bound)


@pytest.mark.parametrize("m,n,d", [(1000, 700, 25), (333, 517, 210), (5, 7, 3),
                                   # fewer rows of op(A) than one remainder tile with a
                                   # long contraction (the judge's d x d product Q^T Z)
                                   (4000, 210, 210), (2000, 100, 40)])
@pytest.mark.parametrize("trans", [1, 0])
def test_gemm_f32_within_rounding_bound(rq, m, n, d, trans):
    import torch
    log(f"gemm f32 trans={trans} m={m} n={n} d={d}")
    r = np.random.default_rng(m + n * 3 + d)
    A = np.asfortranarray(r.standard_normal((m, n)).astype(np.float32))
    X = r.standard_normal((m if trans else n, d)).astype(np.float32)
    C = to_np(rq.gemm(to_dev(A, torch.float32), to_dev(X, torch.float32), trans))
    Aop = (A.T if trans else A).astype(np.float64)
    ref = Aop @ X.astype(np.float64)
    K = Aop.shape[1]
    bound = 2 * (K + 2) * U32 * (np.abs(Aop) @ np.abs(X.astype(np.float64)))
    assert np.all(np.abs(C - ref) <= bound)


def _round16(x, precision):
    """Round float32 values to bf16 / fp16 (nearest even) on the CPU, as float64."""
    import torch
    dt = torch.bfloat16 if precision == "bf16" else torch.float16
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(dt).double().numpy()


@pytest.mark.parametrize("m,n,d", [(1000, 700, 25), (333, 517, 210), (5, 7, 3), (2100, 1500, 520),
                                   (130, 4000, 64), (4000, 130, 272), (777, 901, 273)])
@pytest.mark.parametrize("trans", [1, 0])
@pytest.mark.parametrize("precision", ["bf16", "f16"])
def test_gemm16_within_rounding_bound(rq, m, n, d, trans, precision):
    """Precision-form product: A and X rounded to 16 bits, fp32 accumulation.
    The products of 16-bit values are exact in fp32, so the only error is
    the fp32 summation: |C - op(A16) X16| <= 2 (K + 2) u32 |op(A16)| |X16|."""
    import torch
    log(f"gemm16 {precision} trans={trans} m={m} n={n} d={d}")
    r = np.random.default_rng(m * 5 + n + d)
    A = np.asfortranarray(r.standard_normal((m, n)).astype(np.float32))
    X = r.standard_normal((m if trans else n, d)).astype(np.float32)
    C = to_np(rq.gemm(to_dev(A, torch.float32), to_dev(X, torch.float32), trans,
                      precision=precision))
    A16, X16 = _round16(A, precision), _round16(X, precision)
    Aop = A16.T if trans else A16
    ref = Aop @ X16
    K = Aop.shape[1]
    bound = 2 * (K + 2) * U32 * (np.abs(Aop) @ np.abs(X16))
    assert C.shape == ref.shape
    assert np.all(np.abs(C - ref) <= bound)


@pytest.mark.parametrize("m,n,d", [(1000, 700, 25), (333, 517, 210), (5, 7, 3), (2100, 1500, 520),
                                   (777, 901, 273)])
@pytest.mark.parametrize("trans", [1, 0])
def test_gemm16_split_product(rq, m, n, d, trans):
    """Split bf16 product: A = A1 + A2, X = X1 + X2 with A1, X1 rounded to bf16
    and A2, X2 the rounded residuals; C = A1 X1 + A1 X2 + A2 X1 (each bf16
    product exact in fp32), so |C - ref3| <= 2 (3K + 2) u32 sum of |terms|.
    Against the exact product the three terms leave about 2^-16 relative, far
    below the plain bf16 product's 2^-9: a dropped term fails the second check."""
    import torch
    log(f"gemm16 split trans={trans} m={m} n={n} d={d}")
    r = np.random.default_rng(m * 7 + n + d)
    A = np.asfortranarray(r.standard_normal((m, n)).astype(np.float32))
    X = r.standard_normal((m if trans else n, d)).astype(np.float32)
    C = to_np(rq.gemm(to_dev(A, torch.float32), to_dev(X, torch.float32), trans,
                      precision="bf16x3"))
    A1, X1 = _round16(A, "bf16"), _round16(X, "bf16")
    A2 = _round16((A.astype(np.float64) - A1).astype(np.float32), "bf16")
    X2 = _round16((X.astype(np.float64) - X1).astype(np.float32), "bf16")
    op = (lambda M: M.T) if trans else (lambda M: M)
    ref3 = op(A1) @ X1 + op(A1) @ X2 + op(A2) @ X1
    K = op(A).shape[1]
    absum = np.abs(op(A1)) @ np.abs(X1) + np.abs(op(A1)) @ np.abs(X2) + np.abs(op(A2)) @ np.abs(X1)
    assert C.shape == ref3.shape
    assert np.all(np.abs(C - ref3) <= 2 * (3 * K + 2) * U32 * absum)
    exact = op(A.astype(np.float64)) @ X.astype(np.float64)
    err3 = np.linalg.norm(C - exact)
    err1 = np.linalg.norm(op(A1) @ X1 - exact)
    assert err3 <= 1e-4 * np.linalg.norm(exact)
    assert err3 * 30 <= err1


def _panel(rows, d, kappa, seed):
    r = np.random.default_rng(seed)
    U, _ = np.linalg.qr(r.standard_normal((rows, d)))
    V, _ = np.linalg.qr(r.standard_normal((d, d)))
    s = np.logspace(0, -np.log10(kappa), d)
    return np.asfortranarray((U * s) @ V.T)


@pytest.mark.parametrize("rows,d,kappa", [(1000, 25, 10.0), (8000, 210, 5e3), (333, 17, 1e6),
                                          (500, 224, 1e2), (16, 16, 3.0), (20, 1, 1.0),
                                          (3000, 300, 1e3), (4000, 520, 1e2), (1200, 449, 10.0)])
def test_orth_f64_matches_lapack(rq, rows, d, kappa):
    log(f"orth f64 rows={rows} d={d} kappa={kappa}")
    X = _panel(rows, d, kappa, rows + d)
    Qo, Ro = qr_pos(X)
    Qg, Rg = rq.orth(to_dev(X))
    Qg, Rg = to_np(Qg), to_np(Rg)
    assert np.abs(Qg.T @ Qg - np.eye(d)).max() < 1e-13
    assert np.all(np.tril(Rg, -1) == 0) and np.all(np.diag(Rg) >= 0)
    assert np.abs(Qg @ Rg - X).max() <= 1e-14 * np.abs(X).max() * d
    # QR with a positive diagonal is unique: elementwise agreement to O(u kappa)
    assert np.abs(Qg - Qo).max() <= 1e-13 * kappa
    assert np.abs(Rg - Ro).max() <= 1e-13 * kappa * np.abs(Ro).max()


@pytest.mark.parametrize("rows,d,kappa", [(3000, 64, 1e3), (8001, 210, 1e2), (777, 224, 10.0),
                                          (40, 33, 5.0), (5000, 520, 1e2), (1500, 449, 10.0)])
def test_orth_f32_orthonormal(rq, rows, d, kappa):
    import torch
    log(f"orth f32 rows={rows} d={d} kappa={kappa}")
    X = _panel(rows, d, kappa, 5 + d).astype(np.float32)
    Qg, Rg = rq.orth(to_dev(X, torch.float32))
    Qg, Rg = to_np(Qg), to_np(Rg)
    assert np.abs(Qg.T @ Qg - np.eye(d)).max() < 2e-5
    assert np.all(np.tril(Rg, -1) == 0) and np.all(np.diag(Rg) >= 0)
    assert np.abs(Qg @ Rg - X).max() <= 1e-5 * np.abs(X).max()


@pytest.mark.parametrize("case", ["duplicate", "zero_col", "zero", "low_rank"])
def test_orth_robust_rank_deficient(rq, case):
    log(f"orth robust {case}")
    r = np.random.default_rng(3)
    rows, d = 400, 20
    X = r.standard_normal((rows, d))
    if case == "duplicate":
        X[:, 7] = X[:, 2]
        dep = [7]
    elif case == "zero_col":
        X[:, 0] = 0.0
        X[:, 11] = 0.0
        dep = [0, 11]
    elif case == "zero":
        X[:] = 0.0
        dep = list(range(d))
    else:
        X = r.standard_normal((rows, 5)) @ r.standard_normal((5, d))
        dep = list(range(5, d))
    X = np.asfortranarray(X)
    for panel in ("auto", "robust"):
        Qg, Rg = rq.orth(to_dev(X), panel=panel)
        Qg, Rg = to_np(Qg), to_np(Rg)
        assert np.abs(Qg.T @ Qg - np.eye(d)).max() < 1e-12
        assert np.all(np.tril(Rg, -1) == 0) and np.all(np.diag(Rg) >= 0)
        scale = max(np.abs(X).max(), 1.0)
        assert np.abs(Qg @ Rg - X).max() <= 1e-12 * scale
        # Unique parts: R's diagonal before the first dependent column, and a
        # zero pivot at each dependent column.  (After a dependent column the
        # remaining diagonal depends on the completion direction chosen, for
        # LAPACK as for any other QR.)
        Ro = qr_pos(X)[1]
        first = dep[0]
        assert np.abs(np.diag(Rg)[:first] - np.diag(Ro)[:first]).max(initial=0.0) <= 1e-12 * scale
        assert np.abs(np.diag(Rg)[dep]).max() <= 1e-12 * scale


def test_orth_robust_rank_deficient_wide(rq):
    """d = 300 > 224: the blocked Cholesky and the column-blocked TRSM on a
    panel with a zero column and a duplicate, both beyond the first 224
    columns (the duplicate of a column of the first block).  Same bar as the
    narrow cases."""
    log("orth robust wide d=300")
    r = np.random.default_rng(4)
    rows, d = 1200, 300
    X = r.standard_normal((rows, d))
    X[:, 230] = 0.0
    X[:, 250] = X[:, 10]
    dep = [230, 250]
    X = np.asfortranarray(X)
    for panel in ("auto", "robust"):
        Qg, Rg = rq.orth(to_dev(X), panel=panel)
        Qg, Rg = to_np(Qg), to_np(Rg)
        assert np.abs(Qg.T @ Qg - np.eye(d)).max() < 1e-12
        assert np.all(np.tril(Rg, -1) == 0) and np.all(np.diag(Rg) >= 0)
        scale = max(np.abs(X).max(), 1.0)
        assert np.abs(Qg @ Rg - X).max() <= 1e-12 * scale
        Ro = qr_pos(X)[1]
        assert np.abs(np.diag(Rg)[:dep[0]] - np.diag(Ro)[:dep[0]]).max() <= 1e-12 * scale
        assert np.abs(np.diag(Rg)[dep]).max() <= 1e-12 * scale

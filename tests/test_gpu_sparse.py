"""Sparse input through randqlp_factor_csr against the fp64 oracle on the
dense copy of the same matrix (Section 5.1 factors sparse matrices): the
sparse products A X and A^T X (A^T built on the device) must give the dense
method's results at the fp64 bar."""
import numpy as np
import pytest

import workloads as W
from oracle import randqlp, rel_error
from tests.gpu_util import compare, invariants, log, to_np

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module")
def rq():
    import paper_2110_01011_amd as rq
    rq.lib()
    return rq


def _dev_csr(rowptr, colind, vals, dtype=None):
    import torch
    return (torch.from_numpy(rowptr).cuda(), torch.from_numpy(colind.astype(np.int32)).cuda(),
            torch.from_numpy(vals).to(dtype or torch.float64).cuda())


@pytest.mark.parametrize("m,n,per_row,k,p,q", [(1856, 1856, 6, 50, 10, 1),
                                               (3000, 2000, 4, 40, 5, 2),
                                               (1500, 2500, 8, 30, 10, 0),
                                               (700, 700, 3, 700, 0, 0)])
def test_sparse_parity(rq, m, n, per_row, k, p, q):
    """Square, tall, wide and full width (d = n, Algorithm 1 itself)."""
    log(f"sparse {m}x{n} per_row={per_row} k={k} p={p} q={q}")
    rowptr, colind, vals = W.sparse_standin(m, n, per_row, seed=m + n)
    A = W.csr_to_dense(rowptr, colind, vals, m, n)
    Qg, Lg, Pg, info = rq.factor_csr(*_dev_csr(rowptr, colind, vals), (m, n), k, p, q, 3,
                                     return_info=True)
    Qg, Lg, Pg = to_np(Qg), to_np(Lg), to_np(Pg)
    Qo, Lo, Po = randqlp(A, k, p, q, 3)
    c = compare(A, Qg, Lg, Pg, Qo, Lo, Po, min(k, Lo.shape[0]))
    inv = invariants(A, Qg, Lg, Pg)
    log(f"  nnz={rowptr[-1]}: {c} {inv} {info}")
    assert c["de"] <= TOL and c["dsigma"] <= TOL
    assert c["sinQk"] <= TOL and c["sinPk"] <= TOL and c["sinQ"] <= TOL and c["sinP"] <= TOL
    assert inv["orthQ"] < 1e-12 and inv["orthP"] < 1e-12
    assert inv["upper_max"] == 0.0 and inv["min_diag"] >= 0.0 and inv["L_vs_QtAP"] < 1e-12


def test_sparse_f32_within_5_percent_and_repeatable(rq):
    import torch
    m, n = 2400, 1800
    rowptr, colind, vals = W.sparse_standin(m, n, 5, seed=9)
    A = W.csr_to_dense(rowptr, colind, vals, m, n)
    dev = _dev_csr(rowptr, colind, vals, torch.float32)
    a = [to_np(t) for t in rq.factor_csr(*dev, (m, n), 60, 10, 2, 1)]
    b = [to_np(t) for t in rq.factor_csr(*dev, (m, n), 60, 10, 2, 1)]
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    A32 = A.astype(np.float32).astype(np.float64)
    e_g = rel_error(A32, *a)
    e_o = rel_error(A32, *randqlp(A32, 60, 10, 2, 1))
    log(f"  f32 sparse e={e_g:.6e} oracle {e_o:.6e}")
    assert e_g <= 1.05 * e_o


def test_sparse_empty_rows_columns_and_duplicates(rq):
    """Rows and columns without entries, unsorted columns within a row and a
    repeated position (the two entries add up)."""
    m, n = 400, 300
    rowptr, colind, vals = W.sparse_standin(m, n, 3, seed=4)
    keep = np.ones(m, bool)
    keep[50:80] = False                      # empty rows
    colind = np.where((colind >= 100) & (colind < 120), 7, colind).astype(np.int32)  # empty cols
    rows = [(colind[rowptr[i]:rowptr[i + 1]][::-1], vals[rowptr[i]:rowptr[i + 1]][::-1])
            if keep[i] else (np.zeros(0, np.int32), np.zeros(0)) for i in range(m)]
    rows[5] = (np.concatenate([rows[5][0], [11, 11]]).astype(np.int32),
               np.concatenate([rows[5][1], [0.5, 0.25]]))
    rp = np.zeros(m + 1, np.int64)
    rp[1:] = np.cumsum([r[0].size for r in rows])
    ci = np.concatenate([r[0] for r in rows]).astype(np.int32)
    va = np.concatenate([r[1] for r in rows])
    A = W.csr_to_dense(rp, ci, va, m, n)
    Qg, Lg, Pg = (to_np(t) for t in rq.factor_csr(*_dev_csr(rp, ci, va), (m, n), 20, 5, 1, 2))
    Qo, Lo, Po = randqlp(A, 20, 5, 1, 2)
    c = compare(A, Qg, Lg, Pg, Qo, Lo, Po, 20)
    log(f"  {c}")
    assert c["de"] <= TOL and c["dsigma"] <= TOL and c["sinQk"] <= TOL and c["sinPk"] <= TOL


def test_sparse_zero_matrix(rq):
    import torch
    m, n = 120, 90
    rp = np.zeros(m + 1, np.int64)
    Qg, Lg, Pg = (to_np(t) for t in rq.factor_csr(torch.from_numpy(rp).cuda(),
                                                  torch.zeros(0, dtype=torch.int32).cuda(),
                                                  torch.zeros(0, dtype=torch.float64).cuda(),
                                                  (m, n), 10, 2, 1, 0))
    assert np.all(Lg == 0.0)
    inv = invariants(np.zeros((m, n)), Qg, Lg, Pg)
    assert inv["orthQ"] < 1e-12 and inv["orthP"] < 1e-12


def test_sparse_invalid_structure_is_rejected(rq):
    """A column index outside [0, n) or a falling rowptr is caught by the
    device check before any product reads the arrays."""
    m, n = 200, 150
    rowptr, colind, vals = W.sparse_standin(m, n, 3, seed=5)
    bad = colind.copy()
    bad[17] = n
    with pytest.raises(rq.RandQLPError) as ei:
        rq.factor_csr(*_dev_csr(rowptr, bad, vals), (m, n), 10, 2, 1, 0)
    assert ei.value.status == 1 and "column index" in str(ei.value)
    rp = rowptr.copy()
    rp[40] = rp[41] + 1
    with pytest.raises(rq.RandQLPError) as ei:
        rq.factor_csr(*_dev_csr(rp, colind, vals), (m, n), 10, 2, 1, 0)
    assert ei.value.status == 1 and "rowptr" in str(ei.value)

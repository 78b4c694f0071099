"""Host-side checks of librandqlp: it loads, exports every declared symbol,
and validates arguments before touching the GPU (no device needed)."""
import ctypes
import os
import re

import pytest

import paper_2110_01011_amd as rq

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(rq.LIB_PATH):
        from paper_2110_01011_amd.build_lib import build
        build()
    return rq.lib()


def _declared():
    text = open(os.path.join(ROOT, "include", "randqlp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return set(re.findall(r"\b((?:randqlp|rqlp)_[a-z_]+)\s*\(", text))


def test_every_declared_symbol_is_exported(L):
    declared = _declared()
    assert declared == set(rq.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name


def test_sketch_width(L):
    assert rq.sketch_width(1000, 1000, 20, 5) == 25
    assert rq.sketch_width(8000, 8000, 200, 10) == 210
    assert rq.sketch_width(30, 100, 40, 5) == 30
    assert rq.sketch_width(100, 12, 10, 5) == 12
    assert rq.sketch_width(10, 10, 0, 5) == -1
    assert rq.sketch_width(10, 10, 3, -1) == -1
    assert rq.sketch_width(0, 10, 3, 1) == -1


def test_workspace_size_grows(L):
    a = rq.workspace_size(1000, 1000, 20, 5, 1)
    b = rq.workspace_size(2000, 1000, 20, 5, 1)
    c = rq.workspace_size(1000, 1000, 20, 5, 1, rq.F32)
    assert 0 < a < b and 0 < c < a
    assert rq.workspace_size(10, 10, 0, 1, 1) == 0
    assert rq.workspace_size(10, 10, 2, 1, -1) == 0


@pytest.mark.parametrize("args,what", [
    ((0, 10, 3, 1, 0), "m"), ((10, 0, 3, 1, 0), "n"), ((10, 10, 0, 1, 0), "k"),
    ((10, 10, 3, -1, 0), "p"), ((10, 10, 3, 1, -1), "q"),
])
def test_factor_rejects_bad_sizes(L, args, what):
    m, n, k, p, q = args
    dummy = ctypes.c_void_p(16)
    st = L.randqlp_factor(dummy, m, n, k, p, q, 0, dummy, dummy, dummy, None)
    assert st == 1
    assert what in L.randqlp_last_error().decode()


def test_factor_rejects_null_and_bad_ld_and_options(L):
    dummy = ctypes.c_void_p(16)
    assert L.randqlp_factor(None, 10, 10, 3, 1, 0, 0, dummy, dummy, dummy, None) == 1
    o = rq.default_opts()
    o.lda = 5
    assert L.randqlp_factor(dummy, 10, 10, 3, 1, 0, 0, dummy, dummy, dummy, ctypes.byref(o)) == 1
    o = rq.default_opts()
    o.precision = 7
    assert L.randqlp_factor(dummy, 10, 10, 3, 1, 0, 0, dummy, dummy, dummy, ctypes.byref(o)) == 1
    o = rq.default_opts()
    o.panel_qr = 9
    assert L.randqlp_factor(dummy, 10, 10, 3, 1, 0, 0, dummy, dummy, dummy, ctypes.byref(o)) == 1


def test_undersized_workspace_is_reported(L):
    dummy = ctypes.c_void_p(256)
    o = rq.default_opts()
    o.workspace = ctypes.c_void_p(4096)
    o.workspace_bytes = 16
    st = L.randqlp_factor(dummy, 100, 80, 5, 2, 1, 0, dummy, dummy, dummy, ctypes.byref(o))
    assert st == 4
    assert "workspace" in L.randqlp_last_error().decode()


def test_noalloc_rejects_workspace_and_oversize(L):
    """The no-allocation variant validates like randqlp_factor, refuses a
    caller workspace and rejects sizes whose scratch exceeds its static
    array before touching the device."""
    dummy = ctypes.c_void_p(256)
    assert L.randqlp_factor_noalloc(None, 10, 10, 3, 1, 0, 0, dummy, dummy, dummy, None) == 1
    assert L.randqlp_factor_noalloc(dummy, 10, 10, 0, 1, 0, 0, dummy, dummy, dummy, None) == 1
    o = rq.default_opts()
    o.workspace = ctypes.c_void_p(4096)
    o.workspace_bytes = 1 << 30
    assert L.randqlp_factor_noalloc(dummy, 100, 80, 5, 2, 1, 0, dummy, dummy, dummy,
                                    ctypes.byref(o)) == 1
    assert "workspace" in L.randqlp_last_error().decode()
    m = n = 20000
    assert rq.workspace_size(m, n, 500, 20, 2) > rq.NOALLOC_SCRATCH_BYTES
    st = L.randqlp_factor_noalloc(dummy, m, n, 500, 20, 2, 0, dummy, dummy, dummy, None)
    assert st == 4
    assert "static scratch" in L.randqlp_last_error().decode()


def test_step_entry_points_validate(L):
    dummy = ctypes.c_void_p(16)
    assert L.randqlp_gaussian(dummy, 10, 3, 5, 0, 0, 0, None) == 1          # ld < m
    assert L.randqlp_gaussian(dummy, 10, 3, 10, 0, 0, 5, None) == 1         # precision
    assert L.randqlp_gemm(1, dummy, 10, 8, 4, dummy, 3, 10, dummy, 8, 0, None) == 1  # lda < m
    assert L.randqlp_orth(dummy, 5, 8, 5, dummy, 5, None, 0, 0, 0, None) == 1      # rows < d


def test_status_strings(L):
    for code, name in rq.STATUS.items():
        assert L.randqlp_status_string(code).decode() == name


def test_predictor_entry_points_validate(L):
    dummy = ctypes.c_void_p(256)
    nul = None
    # randqlp_factor_auto: null parameters, bad k, bad q_fallback
    assert L.randqlp_factor_auto(dummy, 10, 10, 3, 1, 2, 0, nul, dummy, dummy, dummy, None,
                                 None) == 1
    assert L.randqlp_factor_auto(dummy, 10, 10, 0, 1, 2, 0, dummy, dummy, dummy, dummy, None,
                                 None) == 1
    assert L.randqlp_factor_auto(dummy, 10, 10, 3, 1, -1, 0, dummy, dummy, dummy, dummy, None,
                                 None) == 1
    assert L.randqlp_features(dummy, 10, 10, 5, 3, 0, 0, dummy, None) == 1       # lda < m
    assert L.randqlp_features(dummy, 10, 10, 10, 3, 0, 2, dummy, None) == 1      # precision
    assert L.randqlp_mlp_forward(dummy, dummy, 0, dummy, None) == 1              # batch
    assert L.randqlp_mlp_loss_grad(dummy, dummy, nul, 4, dummy, dummy, None) == 1
    assert L.randqlp_mlp_adam(dummy, dummy, dummy, dummy, 0, ctypes.c_float(1e-3), None) == 1
    assert L.randqlp_mlp_adam(dummy, dummy, dummy, dummy, 1, ctypes.c_float(0.0), None) == 1
    step = ctypes.c_int64(0)
    assert L.randqlp_mlp_train(dummy, dummy, dummy, dummy, dummy, 0, 1, 8,
                               ctypes.c_float(1e-3), 0, ctypes.byref(step), dummy, None) == 1
    assert L.randqlp_mlp_train(dummy, dummy, dummy, dummy, dummy, 10, 1, 0,
                               ctypes.c_float(1e-3), 0, ctypes.byref(step), dummy, None) == 1


def test_batched_entry_points_validate(L):
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    d = vp(256)
    A = (vp * 2)(d, d)
    m = (i64 * 2)(100, 80)
    n = (i64 * 2)(90, 70)
    k = (i32 * 2)(5, 4)
    seeds = (ctypes.c_uint64 * 2)(1, 2)
    h = vp()
    # bad count, bad precision, bad p / q, k = 0 in one matrix, lda < m
    assert L.randqlp_batch_create(0, A, m, n, None, k, 2, 1, seeds, A, None, A, None, A, None,
                                  1, 0, ctypes.byref(h)) == 1
    assert L.randqlp_batch_create(2, A, m, n, None, k, 2, 1, seeds, A, None, A, None, A, None,
                                  2, 0, ctypes.byref(h)) == 1
    assert L.randqlp_batch_create(2, A, m, n, None, k, -1, 1, seeds, A, None, A, None, A, None,
                                  1, 0, ctypes.byref(h)) == 1
    k0 = (i32 * 2)(5, 0)
    assert L.randqlp_batch_create(2, A, m, n, None, k0, 2, 1, seeds, A, None, A, None, A, None,
                                  1, 0, ctypes.byref(h)) == 1
    assert "matrix 1" in L.randqlp_last_error().decode()
    lda = (i64 * 2)(100, 10)
    assert L.randqlp_batch_create(2, A, m, n, lda, k, 2, 1, seeds, A, None, A, None, A, None,
                                  1, 0, ctypes.byref(h)) == 1
    assert h.value is None
    assert L.randqlp_batch_run(None, 1, None) == 1
    assert L.randqlp_tune_save(None) == 1
    assert L.randqlp_tune_load(b"/nonexistent/dir/tune.txt") == 1


def test_auto_rank_mode_validates(L):
    """k <= 0 asks for the rank to be predicted: opts with tol in (0, 1] and
    k_max >= 1 (k_max + p <= 4096) are required; checked before any work."""
    dummy = ctypes.c_void_p(256)
    args = (dummy, 500, 400, 0, 10, 2, 0, dummy, dummy, dummy, dummy)
    assert L.randqlp_factor_auto(*args, None, None) == 1
    assert "tol" in L.randqlp_last_error().decode()
    o = rq.default_opts()
    o.tol, o.k_max = 0.0, 64
    assert L.randqlp_factor_auto(*args, ctypes.byref(o), None) == 1
    o.tol, o.k_max = 1.5, 64
    assert L.randqlp_factor_auto(*args, ctypes.byref(o), None) == 1
    o.tol, o.k_max = 0.1, 0
    assert L.randqlp_factor_auto(*args, ctypes.byref(o), None) == 1
    o.tol, o.k_max = 0.1, 5000
    assert L.randqlp_factor_auto(*args, ctypes.byref(o), None) == 6


def test_csr_entry_validates_on_the_host(L):
    dummy = ctypes.c_void_p(256)
    # nnz < 0, null arrays, 16-bit precision, too many rows
    assert L.randqlp_factor_csr(dummy, dummy, dummy, 10, 10, -1, 3, 1, 0, 0, dummy, dummy,
                                dummy, None) == 1
    assert L.randqlp_factor_csr(dummy, None, dummy, 10, 10, 5, 3, 1, 0, 0, dummy, dummy,
                                dummy, None) == 1
    o = rq.default_opts()
    o.precision = rq.MIXED_BF16
    assert L.randqlp_factor_csr(dummy, dummy, dummy, 10, 10, 5, 3, 1, 0, 0, dummy, dummy,
                                dummy, ctypes.byref(o)) == 6
    assert L.randqlp_factor_csr(dummy, dummy, dummy, 1 << 21, 10, 5, 3, 1, 0, 0, dummy, dummy,
                                dummy, None) == 6


def test_async_entry_validates(L):
    dummy = ctypes.c_void_p(256)
    o = rq.default_opts()
    # null status, no opts, no workspace
    assert L.randqlp_factor_async(dummy, 100, 80, 5, 2, 1, 0, dummy, dummy, dummy,
                                  ctypes.byref(o), None) == 1
    assert L.randqlp_factor_async(dummy, 100, 80, 5, 2, 1, 0, dummy, dummy, dummy, None,
                                  dummy) == 1
    assert L.randqlp_factor_async(dummy, 100, 80, 5, 2, 1, 0, dummy, dummy, dummy,
                                  ctypes.byref(o), dummy) == 1
    assert "workspace" in L.randqlp_last_error().decode()

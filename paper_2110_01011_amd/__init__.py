"""Randomized QLP decomposition on the AMD Instinct MI355X (gfx950).

Thin binding over librandqlp.so (C ABI in include/randqlp.h).  It only
marshals arguments: torch provides device memory and the current stream;
every step of the factorisation runs in the library's HIP kernels.  There is
no CPU fallback -- importing works without a GPU (for argument checks), but
any compute call needs the built library and a device.

Matrices are column-major: a tensor of shape (rows, cols) with stride
(1, ld), ld >= rows.  `colmajor()` makes such a copy of any 2-D tensor.
"""
import contextlib
import ctypes
import os

__all__ = ["factor", "factor_async", "factor_noalloc", "factor_csr", "factor_auto", "Batch", "factor_batched", "tune_save", "tune_load", "features", "mlp_forward", "mlp_loss_grad", "mlp_adam",
           "mlp_train", "gaussian", "gemm", "orth", "sketch_width", "workspace_size",
           "colmajor", "empty_colmajor", "lib", "RandQLPError", "F64", "F32", "MIXED_BF16",
           "MIXED_F16", "MIXED_BF16X3",
           "PANEL_AUTO", "PANEL_CHOLQR2", "PANEL_ROBUST"]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librandqlp.so")

F64, F32, MIXED_BF16, MIXED_F16, MIXED_BF16X3 = 0, 1, 2, 3, 4
_PRECISIONS = {"f64": F64, "f32": F32, "bf16": MIXED_BF16, "f16": MIXED_F16,
               "bf16x3": MIXED_BF16X3}
PANEL_AUTO, PANEL_CHOLQR2, PANEL_ROBUST = 0, 1, 2
_PANELS = {"auto": PANEL_AUTO, "cholqr2": PANEL_CHOLQR2, "robust": PANEL_ROBUST}
STATUS = {0: "RQLP_OK", 1: "RQLP_E_INVALID_ARG", 2: "RQLP_E_NONFINITE", 3: "RQLP_E_NOMEM",
          4: "RQLP_E_WORKSPACE", 5: "RQLP_E_HIP", 6: "RQLP_E_UNSUPPORTED"}

# Every symbol include/randqlp.h declares.
EXPORTS = ["rqlp_opts_default", "randqlp_sketch_width", "randqlp_workspace_size",
           "randqlp_factor", "randqlp_factor_async", "randqlp_factor_noalloc",
           "randqlp_factor_csr",
           "randqlp_factor_auto", "randqlp_features", "randqlp_mlp_forward",
           "randqlp_mlp_loss_grad", "randqlp_mlp_adam", "randqlp_mlp_train",
           "randqlp_batch_create", "randqlp_batch_run", "randqlp_batch_query",
           "randqlp_batch_destroy", "randqlp_factor_batched", "randqlp_tune_save",
           "randqlp_tune_load",
           "randqlp_gaussian", "randqlp_gemm", "randqlp_orth",
           "randqlp_profile_enable", "randqlp_profile_read",
           "randqlp_status_string", "randqlp_last_error", "randqlp_build_id"]


class RandQLPError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class Info(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("q_used", ctypes.c_int32),
                ("breakdowns", ctypes.c_int32), ("robust_rerun", ctypes.c_int32),
                ("completed", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


MLP_INPUTS, MLP_HIDDEN, MLP_CLASSES, MLP_PARAMS = 65, 128, 6, 25734


class AutoInfo(ctypes.Structure):
    _fields_ = [("q_predicted", ctypes.c_int32), ("q_used", ctypes.c_int32),
                ("judged", ctypes.c_int32), ("resumed", ctypes.c_int32),
                ("judge_ratio", ctypes.c_double), ("est_rel_err", ctypes.c_double),
                ("k_predicted", ctypes.c_int32), ("k_used", ctypes.c_int32),
                ("d", ctypes.c_int32), ("rank_fallback", ctypes.c_int32),
                ("rank_err", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class BatchInfo(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("grouped", ctypes.c_int32),
                ("fallbacks", ctypes.c_int32), ("wn_tn", ctypes.c_int32),
                ("wn_nn", ctypes.c_int32), ("dmax", ctypes.c_int32), ("tune_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("panel_qr", ctypes.c_int32),
                ("lda", ctypes.c_int64), ("ldq", ctypes.c_int64), ("ldl", ctypes.c_int64),
                ("ldp", ctypes.c_int64), ("stream", ctypes.c_void_p),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
                ("info", ctypes.POINTER(Info)), ("tol", ctypes.c_double),
                ("k_max", ctypes.c_int32)]


_lib = None


def lib():
    """Load librandqlp.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2110_01011_amd.build_lib`")
    L = ctypes.CDLL(LIB_PATH)
    L.randqlp_build_id.argtypes = []
    L.randqlp_build_id.restype = ctypes.c_char_p
    from .build_lib import source_id
    built, want = L.randqlp_build_id().decode(), source_id()
    if built != want:
        raise ImportError(f"{LIB_PATH} was built from other sources (build id {built[:12]}, "
                          f"sources {want[:12]}): rebuild it with "
                          "`python -m paper_2110_01011_amd.build_lib`")
    i64, i32, u64, vp, sz = ctypes.c_int64, ctypes.c_int, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_size_t
    L.rqlp_opts_default.argtypes = [ctypes.POINTER(Opts)]
    L.rqlp_opts_default.restype = None
    L.randqlp_sketch_width.argtypes = [i64, i64, i32, i32]
    L.randqlp_sketch_width.restype = i64
    L.randqlp_workspace_size.argtypes = [i64, i64, i32, i32, i32, ctypes.POINTER(Opts)]
    L.randqlp_workspace_size.restype = sz
    L.randqlp_factor.argtypes = [vp, i64, i64, i32, i32, i32, u64, vp, vp, vp, ctypes.POINTER(Opts)]
    L.randqlp_factor.restype = i32
    L.randqlp_factor_noalloc.argtypes = [vp, i64, i64, i32, i32, i32, u64, vp, vp, vp,
                                         ctypes.POINTER(Opts)]
    L.randqlp_factor_csr.argtypes = [vp, vp, vp, i64, i64, i64, i32, i32, i32, u64, vp, vp, vp,
                                     ctypes.POINTER(Opts)]
    L.randqlp_factor_csr.restype = i32
    L.randqlp_factor_async.argtypes = [vp, i64, i64, i32, i32, i32, u64, vp, vp, vp,
                                       ctypes.POINTER(Opts), vp]
    L.randqlp_factor_async.restype = i32
    L.randqlp_factor_noalloc.restype = i32
    L.randqlp_factor_auto.argtypes = [vp, i64, i64, i32, i32, i32, u64, vp, vp, vp, vp,
                                      ctypes.POINTER(Opts), ctypes.POINTER(AutoInfo)]
    L.randqlp_factor_auto.restype = i32
    L.randqlp_features.argtypes = [vp, i64, i64, i64, i32, u64, i32, vp, vp]
    L.randqlp_features.restype = i32
    L.randqlp_mlp_forward.argtypes = [vp, vp, i32, vp, vp]
    L.randqlp_mlp_forward.restype = i32
    L.randqlp_mlp_loss_grad.argtypes = [vp, vp, vp, i32, vp, vp, vp]
    L.randqlp_mlp_loss_grad.restype = i32
    L.randqlp_mlp_adam.argtypes = [vp, vp, vp, vp, i64, ctypes.c_float, vp]
    L.randqlp_mlp_adam.restype = i32
    L.randqlp_mlp_train.argtypes = [vp, vp, vp, vp, vp, i64, i32, i32, ctypes.c_float, u64,
                                    ctypes.POINTER(i64), vp, vp]
    L.randqlp_mlp_train.restype = i32
    P64 = ctypes.POINTER(i64)
    PVP = ctypes.POINTER(vp)
    L.randqlp_batch_create.argtypes = [i32, PVP, P64, P64, P64, ctypes.POINTER(i32), i32, i32,
                                       ctypes.POINTER(u64), PVP, P64, PVP, P64, PVP, P64, i32, i32,
                                       ctypes.POINTER(vp)]
    L.randqlp_batch_create.restype = i32
    L.randqlp_batch_run.argtypes = [vp, i32, vp]
    L.randqlp_batch_run.restype = i32
    L.randqlp_batch_query.argtypes = [vp, ctypes.POINTER(BatchInfo)]
    L.randqlp_batch_query.restype = i32
    L.randqlp_batch_destroy.argtypes = [vp]
    L.randqlp_batch_destroy.restype = None
    L.randqlp_factor_batched.argtypes = [i32, PVP, P64, P64, ctypes.POINTER(i32), i32, i32,
                                         ctypes.POINTER(u64), PVP, PVP, PVP, i32, vp]
    L.randqlp_factor_batched.restype = i32
    L.randqlp_tune_save.argtypes = [ctypes.c_char_p]
    L.randqlp_tune_save.restype = i32
    L.randqlp_tune_load.argtypes = [ctypes.c_char_p]
    L.randqlp_tune_load.restype = i32
    L.randqlp_gaussian.argtypes = [vp, i64, i64, i64, u64, u64, i32, vp]
    L.randqlp_gaussian.restype = i32
    L.randqlp_gemm.argtypes = [i32, vp, i64, i64, i64, vp, i64, i64, vp, i64, i32, vp]
    L.randqlp_gemm.restype = i32
    L.randqlp_orth.argtypes = [vp, i64, i64, i64, vp, i64, vp, i64, i32, i32, vp]
    L.randqlp_orth.restype = i32
    L.randqlp_profile_enable.argtypes = [i32]
    L.randqlp_profile_enable.restype = None
    L.randqlp_profile_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64),
                                       ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    L.randqlp_profile_read.restype = None
    L.randqlp_status_string.argtypes = [i32]
    L.randqlp_status_string.restype = ctypes.c_char_p
    L.randqlp_last_error.argtypes = []
    L.randqlp_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(status):
    if status != 0:
        msg = lib().randqlp_last_error().decode(errors="replace")
        raise RandQLPError(status, msg)


def profile_enable(on=True):
    """Time the A-streaming product kernel with HIP events inside factor()."""
    lib().randqlp_profile_enable(1 if on else 0)


def profile_read():
    """(total ms, launches, algorithmic flops, algorithmic bytes); resets."""
    ms, fl, by = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    n = ctypes.c_int64()
    lib().randqlp_profile_read(ctypes.byref(ms), ctypes.byref(n), ctypes.byref(fl), ctypes.byref(by))
    return ms.value, n.value, fl.value, by.value


def sketch_width(m, n, k, p):
    return int(lib().randqlp_sketch_width(m, n, k, p))


def default_opts():
    o = Opts()
    lib().rqlp_opts_default(ctypes.byref(o))
    return o


def workspace_size(m, n, k, p, q, precision=F64):
    o = default_opts()
    o.precision = precision
    return int(lib().randqlp_workspace_size(m, n, k, p, q, ctypes.byref(o)))


# --------------------------------------------------------------- torch glue
def _torch():
    import torch
    return torch


def empty_colmajor(rows, cols, dtype, device):
    torch = _torch()
    return torch.empty((cols, rows), dtype=dtype, device=device).t()


def colmajor(t):
    """Column-major view or copy of a 2-D tensor (stride (1, ld))."""
    if t.dim() != 2:
        raise ValueError("expected a 2-D tensor")
    if t.stride(0) == 1 and t.stride(1) >= max(1, t.shape[0]):
        return t
    return t.t().contiguous().t()


def _precision(dtype):
    torch = _torch()
    if dtype == torch.float64:
        return F64
    if dtype == torch.float32:
        return F32
    raise TypeError(f"unsupported dtype {dtype} (float64 or float32)")


def _stream_ptr(device):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ld(t):
    return max(1, t.stride(1)) if t.shape[1] > 1 else max(1, t.shape[0])


def _on_device(dev):
    """Context that makes `dev` current (a no-op when it already is)."""
    torch = _torch()
    if dev.index is None or dev.index == torch.cuda.current_device():
        return contextlib.nullcontext()
    return torch.cuda.device(dev)


def _prepare(A, k, p, q, panel, precision):
    torch = _torch()
    if not A.is_cuda:
        raise ValueError("A must be a device tensor")
    A = colmajor(A)
    m, n = A.shape
    prec = _precision(A.dtype)
    if precision is not None:
        prec = _PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        if (prec == F64) != (A.dtype == torch.float64):
            raise TypeError("precision does not match A's dtype (f64 needs float64, "
                            "f32/bf16/f16/bf16x3 need float32)")
    d = sketch_width(m, n, k, p)
    if d < 1:
        _check(lib().randqlp_factor(None, m, n, k, p, q, 0, None, None, None, None))
    dev = A.device
    Q = empty_colmajor(m, d, A.dtype, dev)
    P = empty_colmajor(n, d, A.dtype, dev)
    L = empty_colmajor(d, d, torch.float64, dev)
    o = default_opts()
    o.precision = prec
    o.panel_qr = _PANELS[panel] if isinstance(panel, str) else int(panel)
    o.lda, o.ldq, o.ldl, o.ldp = _ld(A), _ld(Q), _ld(L), _ld(P)
    o.stream = _stream_ptr(dev)
    return A, Q, L, P, o


def factor(A, k, p, q, seed, panel="auto", precision=None, return_info=False):
    """Rand-QLP of a device matrix A (m x n, float64 or float32).

    precision: None (from A's dtype), "f64", "f32", or the precision forms
    "bf16" / "f16" (A float32; the products with A run on a 16-bit copy) and
    "bf16x3" (as "bf16", with the final projection as the split bf16 product).
    Returns (Q, L, P): Q (m x d) and P (n x d) in A's dtype, L (d x d)
    float64, all column-major, with d = min(k + p, m, n).
    """
    torch = _torch()
    A, Q, L, P, o = _prepare(A, k, p, q, panel, precision)
    m, n = A.shape
    ws_bytes = lib().randqlp_workspace_size(m, n, k, p, q, ctypes.byref(o))
    ws = torch.empty(max(ws_bytes, 256), dtype=torch.uint8, device=A.device)
    o.workspace = ctypes.c_void_p(ws.data_ptr())
    o.workspace_bytes = ws.numel()
    info = Info()
    o.info = ctypes.pointer(info)
    with _on_device(A.device):
        _check(lib().randqlp_factor(ctypes.c_void_p(A.data_ptr()), m, n, k, p, q, seed,
                                    ctypes.c_void_p(Q.data_ptr()), ctypes.c_void_p(L.data_ptr()),
                                    ctypes.c_void_p(P.data_ptr()), ctypes.byref(o)))
    del ws
    if return_info:
        return Q, L, P, info.as_dict()
    return Q, L, P


class AsyncFactor:
    """Buffers and arguments of one asynchronous factorisation
    (randqlp_factor_async), allocated once: Q, L, P, the workspace and the
    device status words.  launch() only enqueues on the current stream, so
    it can be captured into a graph (torch.cuda.graph) and replayed."""

    def __init__(self, A, k, p, q, seed, panel="auto", precision=None):
        torch = _torch()
        self.A, self.Q, self.L, self.P, self.opts = _prepare(A, k, p, q, panel, precision)
        m, n = self.A.shape
        nb = lib().randqlp_workspace_size(m, n, k, p, q, ctypes.byref(self.opts))
        self.ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=self.A.device)
        self.opts.workspace = ctypes.c_void_p(self.ws.data_ptr())
        self.opts.workspace_bytes = self.ws.numel()
        self.status = torch.zeros(4, dtype=torch.int32, device=self.A.device)
        self.args = (k, p, q, seed)

    def launch(self):
        k, p, q, seed = self.args
        m, n = self.A.shape
        self.opts.stream = _stream_ptr(self.A.device)
        _check(lib().randqlp_factor_async(
            ctypes.c_void_p(self.A.data_ptr()), m, n, k, p, q, seed,
            ctypes.c_void_p(self.Q.data_ptr()), ctypes.c_void_p(self.L.data_ptr()),
            ctypes.c_void_p(self.P.data_ptr()), ctypes.byref(self.opts),
            ctypes.c_void_p(self.status.data_ptr())))
        return self.Q, self.L, self.P, self.status


def factor_async(A, k, p, q, seed, panel="auto", precision=None):
    """Enqueue one factorisation without synchronising; returns (Q, L, P,
    status) -- status (4 int32, device) is valid once the stream has reached
    the end of the work, and status[0] != 0 means the factors are not to be
    trusted (use factor())."""
    return AsyncFactor(A, k, p, q, seed, panel, precision).launch()


def factor_csr(rowptr, colind, vals, shape, k, p, q, seed, panel="auto", return_info=False):
    """Rand-QLP of a sparse device matrix in CSR form: rowptr (m + 1, int64),
    colind (nnz, int32), vals (nnz, float64 or float32), shape = (m, n).
    Returns (Q, L, P) as factor() does for the dense matrix."""
    torch = _torch()
    m, n = int(shape[0]), int(shape[1])
    if not (rowptr.is_cuda and colind.is_cuda and vals.is_cuda):
        raise ValueError("CSR arrays must be device tensors")
    if rowptr.dtype != torch.int64 or colind.dtype != torch.int32:
        raise TypeError("rowptr must be int64 and colind int32")
    if rowptr.numel() != m + 1 or colind.numel() != vals.numel():
        raise ValueError("rowptr needs m + 1 entries and colind / vals nnz each")
    rowptr, colind, vals = rowptr.contiguous(), colind.contiguous(), vals.contiguous()
    nnz = vals.numel()
    d = sketch_width(m, n, k, p)
    if d < 1:
        _check(lib().randqlp_factor(None, m, n, k, p, q, 0, None, None, None, None))
    dev = vals.device
    Q = empty_colmajor(m, d, vals.dtype, dev)
    P = empty_colmajor(n, d, vals.dtype, dev)
    L = empty_colmajor(d, d, torch.float64, dev)
    o = default_opts()
    o.precision = _precision(vals.dtype)
    o.panel_qr = _PANELS[panel] if isinstance(panel, str) else int(panel)
    o.ldq, o.ldl, o.ldp = _ld(Q), _ld(L), _ld(P)
    o.stream = _stream_ptr(dev)
    info = Info()
    o.info = ctypes.pointer(info)
    with _on_device(dev):
        _check(lib().randqlp_factor_csr(ctypes.c_void_p(rowptr.data_ptr()),
                                        ctypes.c_void_p(colind.data_ptr()),
                                        ctypes.c_void_p(vals.data_ptr()), m, n, nnz, k, p, q,
                                        seed, ctypes.c_void_p(Q.data_ptr()),
                                        ctypes.c_void_p(L.data_ptr()),
                                        ctypes.c_void_p(P.data_ptr()), ctypes.byref(o)))
    if return_info:
        return Q, L, P, info.as_dict()
    return Q, L, P


NOALLOC_SCRATCH_BYTES = 128 << 20


def factor_noalloc(A, k, p, q, seed, panel="auto", precision=None, return_info=False,
                   out=None):
    """factor() through randqlp_factor_noalloc: the library's static device
    scratch instead of a workspace (nothing allocated by the call).  out:
    optional (Q, L, P) column-major tensors to write into (allocated here
    when None).  Raises RandQLPError (RQLP_E_WORKSPACE) when the sizes need
    more than NOALLOC_SCRATCH_BYTES of scratch."""
    A, Q, L, P, o = _prepare(A, k, p, q, panel, precision)
    if out is not None:
        Q, L, P = out
        o.ldq, o.ldl, o.ldp = _ld(Q), _ld(L), _ld(P)
    m, n = A.shape
    info = Info()
    o.info = ctypes.pointer(info)
    with _on_device(A.device):
        _check(lib().randqlp_factor_noalloc(ctypes.c_void_p(A.data_ptr()), m, n, k, p, q, seed,
                                            ctypes.c_void_p(Q.data_ptr()),
                                            ctypes.c_void_p(L.data_ptr()),
                                            ctypes.c_void_p(P.data_ptr()), ctypes.byref(o)))
    if return_info:
        return Q, L, P, info.as_dict()
    return Q, L, P


def factor_auto(A, k, p, seed, params, q_fallback=2, panel="auto", precision=None,
                return_info=False, tol=None, k_max=256):
    """Rand-QLP with the number of power rounds predicted from a first sketch
    (params: float32 device tensor of MLP_PARAMS), judged one round ahead and
    resumed up to q_fallback when the prediction was too low.  With k <= 0
    the rank is predicted too: params then holds 2 * MLP_PARAMS values (the
    power-round network, then the rank network), tol is the target relative
    error of the rank-k approximation Q L[:, :k] P[:, :k]^T and k_max the
    largest rank; the returned factors have auto_info["d"] columns and
    auto_info["k_used"] is the smallest rank meeting tol.  Uses the
    library's workspace cache.  Returns (Q, L, P) or, with return_info,
    (Q, L, P, info, auto_info)."""
    torch = _torch()
    rank = k <= 0
    want = (2 if rank else 1) * MLP_PARAMS
    if params.dtype != torch.float32 or params.numel() != want or not params.is_cuda:
        raise ValueError(f"params must be a float32 device tensor of {want} values")
    if rank and tol is None:
        raise ValueError("k <= 0 (predict the rank) needs tol")
    A, Q, L, P, o = _prepare(A, k_max if rank else k, p, q_fallback, panel, precision)
    if rank:
        o.tol = float(tol)
        o.k_max = int(k_max)
    m, n = A.shape
    info, ainfo = Info(), AutoInfo()
    o.info = ctypes.pointer(info)
    params = params.contiguous()
    with _on_device(A.device):
        _check(lib().randqlp_factor_auto(ctypes.c_void_p(A.data_ptr()), m, n, k, p, q_fallback,
                                         seed, ctypes.c_void_p(params.data_ptr()),
                                         ctypes.c_void_p(Q.data_ptr()),
                                         ctypes.c_void_p(L.data_ptr()),
                                         ctypes.c_void_p(P.data_ptr()), ctypes.byref(o),
                                         ctypes.byref(ainfo)))
    d = ainfo.d
    Q, L, P = Q[:, :d], L[:d, :d], P[:, :d]
    if return_info:
        return Q, L, P, info.as_dict(), ainfo.as_dict()
    return Q, L, P


def features(A, k, seed):
    """The predictor's 65 features of a device matrix (float64 or float32)."""
    torch = _torch()
    A = colmajor(A)
    m, n = A.shape
    out = torch.empty(MLP_INPUTS, dtype=torch.float32, device=A.device)
    _check(lib().randqlp_features(ctypes.c_void_p(A.data_ptr()), m, n, _ld(A), k, seed,
                                  _precision(A.dtype), ctypes.c_void_p(out.data_ptr()),
                                  _stream_ptr(A.device)))
    return out


def _rows(X, cols, dtype):
    torch = _torch()
    if X.dim() != 2 or X.shape[1] != cols or X.dtype != dtype or not X.is_cuda:
        raise ValueError(f"expected a device {dtype} tensor with {cols} columns")
    return X.contiguous()


def mlp_forward(params, X):
    """Logits (B x 6) of the predictor MLP for features X (B x 65, float32)."""
    torch = _torch()
    X = _rows(X, MLP_INPUTS, torch.float32)
    out = torch.empty((X.shape[0], MLP_CLASSES), dtype=torch.float32, device=X.device)
    _check(lib().randqlp_mlp_forward(ctypes.c_void_p(params.data_ptr()),
                                     ctypes.c_void_p(X.data_ptr()), X.shape[0],
                                     ctypes.c_void_p(out.data_ptr()), _stream_ptr(X.device)))
    return out


def mlp_loss_grad(params, X, y):
    """(mean cross-entropy, gradient) of the predictor MLP on a batch."""
    torch = _torch()
    X = _rows(X, MLP_INPUTS, torch.float32)
    y = y.to(torch.int32).contiguous()
    grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=X.device)
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    _check(lib().randqlp_mlp_loss_grad(ctypes.c_void_p(params.data_ptr()),
                                       ctypes.c_void_p(X.data_ptr()),
                                       ctypes.c_void_p(y.data_ptr()), X.shape[0],
                                       ctypes.c_void_p(grad.data_ptr()),
                                       ctypes.c_void_p(loss.data_ptr()), _stream_ptr(X.device)))
    return loss, grad


def mlp_adam(params, grad, m, v, t, lr):
    """One Adam step in place (t >= 1)."""
    _check(lib().randqlp_mlp_adam(ctypes.c_void_p(params.data_ptr()),
                                  ctypes.c_void_p(grad.data_ptr()), ctypes.c_void_p(m.data_ptr()),
                                  ctypes.c_void_p(v.data_ptr()), int(t), float(lr),
                                  _stream_ptr(params.device)))


def mlp_train(params, m, v, X, y, epochs, batch, lr, seed, step=0):
    """Train in place on (X, y); returns (per-epoch mean loss tensor, step)."""
    torch = _torch()
    X = _rows(X, MLP_INPUTS, torch.float32)
    y = y.to(torch.int32).contiguous()
    losses = torch.empty(max(epochs, 1), dtype=torch.float32, device=X.device)
    st = ctypes.c_int64(step)
    _check(lib().randqlp_mlp_train(ctypes.c_void_p(params.data_ptr()),
                                   ctypes.c_void_p(m.data_ptr()), ctypes.c_void_p(v.data_ptr()),
                                   ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                   X.shape[0], epochs, batch, float(lr), seed, ctypes.byref(st),
                                   ctypes.c_void_p(losses.data_ptr()), _stream_ptr(X.device)))
    return losses[:epochs], st.value


class Batch:
    """A batched plan over device matrices As (float64 or float32, one dtype):
    outputs self.Q, self.L, self.P (lists of column-major tensors) are
    allocated here and bound to the plan together with As; run() replays the
    captured graph.  Keep the object alive while the plan is used."""

    def __init__(self, As, ks, p, q, seeds, tune=False):
        torch = _torch()
        if not As:
            raise ValueError("empty batch")
        self.A = [colmajor(a) for a in As]
        dtype = self.A[0].dtype
        if any(a.dtype != dtype for a in self.A):
            raise TypeError("all matrices must share one dtype")
        cnt = len(self.A)
        dev = self.A[0].device
        self.Q, self.L, self.P = [], [], []
        for a, k in zip(self.A, ks):
            m, n = a.shape
            d = sketch_width(m, n, k, p)
            if d < 1:
                raise ValueError("bad k or p")
            self.Q.append(empty_colmajor(m, d, dtype, dev))
            self.L.append(empty_colmajor(d, d, torch.float64, dev))
            self.P.append(empty_colmajor(n, d, dtype, dev))
        vp, i64 = ctypes.c_void_p, ctypes.c_int64
        arr = lambda T, xs: (T * cnt)(*xs)
        self._keep = [
            arr(vp, [t.data_ptr() for t in self.A]),
            arr(i64, [t.shape[0] for t in self.A]), arr(i64, [t.shape[1] for t in self.A]),
            arr(i64, [_ld(t) for t in self.A]), arr(ctypes.c_int32, list(ks)),
            arr(ctypes.c_uint64, list(seeds)),
            arr(vp, [t.data_ptr() for t in self.Q]), arr(i64, [_ld(t) for t in self.Q]),
            arr(vp, [t.data_ptr() for t in self.L]), arr(i64, [_ld(t) for t in self.L]),
            arr(vp, [t.data_ptr() for t in self.P]), arr(i64, [_ld(t) for t in self.P])]
        k_ = self._keep
        h = ctypes.c_void_p()
        with torch.cuda.device(dev):
            _check(lib().randqlp_batch_create(cnt, k_[0], k_[1], k_[2], k_[3], k_[4], p, q, k_[5],
                                              k_[6], k_[7], k_[8], k_[9], k_[10], k_[11],
                                              _precision(dtype), 1 if tune else 0,
                                              ctypes.byref(h)))
        self._h = h
        self.device = dev

    def run(self, use_graph=True):
        _check(lib().randqlp_batch_run(self._h, 1 if use_graph else 0, _stream_ptr(self.device)))
        return self.Q, self.L, self.P

    def info(self):
        i = BatchInfo()
        _check(lib().randqlp_batch_query(self._h, ctypes.byref(i)))
        return i.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            lib().randqlp_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def factor_batched(As, ks, p, q, seeds, tune=False):
    """Factor a list of device matrices together; returns (Qs, Ls, Ps, info)."""
    b = Batch(As, ks, p, q, seeds, tune=tune)
    try:
        Q, L, P = b.run()
        return Q, L, P, b.info()
    finally:
        b.close()


def tune_save(path):
    _check(lib().randqlp_tune_save(str(path).encode()))


def tune_load(path):
    _check(lib().randqlp_tune_load(str(path).encode()))


def gaussian(m, d, seed, stream_id=0, dtype=None, device="cuda"):
    """The randn step: Omega (m x d) from (seed, stream_id), column-major."""
    torch = _torch()
    dtype = dtype or torch.float64
    out = empty_colmajor(m, d, dtype, device)
    _check(lib().randqlp_gaussian(ctypes.c_void_p(out.data_ptr()), m, d, max(1, m), seed,
                                  stream_id, _precision(dtype), _stream_ptr(out.device)))
    return out


def gemm(A, X, trans_a, precision=None):
    """C = A^T X (trans_a) or A X, on the sketch-product kernels.

    precision: None (from the dtype), or "bf16" / "f16" for the precision-form
    kernel (A, X float32, rounded to 16 bits inside; C float32), or "bf16x3"
    for the split bf16 product (rounded parts and residuals, three terms)."""
    A = colmajor(A)
    X = colmajor(X)
    m, n = A.shape
    rows = n if trans_a else m
    if X.shape[0] != (m if trans_a else n) or X.dtype != A.dtype:
        raise ValueError("shape or dtype mismatch")
    prec = _precision(A.dtype)
    if precision is not None:
        prec = _PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    d = X.shape[1]
    C = empty_colmajor(rows, d, A.dtype, A.device)
    _check(lib().randqlp_gemm(1 if trans_a else 0, ctypes.c_void_p(A.data_ptr()), m, n, _ld(A),
                              ctypes.c_void_p(X.data_ptr()), d, _ld(X),
                              ctypes.c_void_p(C.data_ptr()), max(1, rows),
                              prec, _stream_ptr(A.device)))
    return C


def orth(X, panel="auto"):
    """Reduced QR X = Qx R (diag R >= 0) of a tall panel; returns (Qx, R)."""
    torch = _torch()
    X = colmajor(X)
    rows, d = X.shape
    Qx = empty_colmajor(rows, d, X.dtype, X.device)
    R = empty_colmajor(d, d, torch.float64, X.device)
    pq = _PANELS[panel] if isinstance(panel, str) else int(panel)
    _check(lib().randqlp_orth(ctypes.c_void_p(X.data_ptr()), rows, d, _ld(X),
                              ctypes.c_void_p(Qx.data_ptr()), max(1, rows),
                              ctypes.c_void_p(R.data_ptr()), max(1, d), _precision(X.dtype), pq,
                              _stream_ptr(X.device)))
    return Qx, R

"""Seeded synthetic input matrices for Rand-QLP tests and benchmarks.

Holds none of the factorisation's arithmetic: it only builds the test
matrices A (column-major fp64 numpy arrays) and, where it knows them, their
exact singular triplets.  Shared by the oracle-side tests, the GPU tests and
the benchmark.  Random streams come from numpy's Philox bit generator keyed
by (seed, stream id); these streams are disjoint from the sketch matrix's
stream 0, which each side of the factorisation draws itself.

Families (Section 5.2 describes the first four; sizes are the workloads'):
  fast_decay      sigma_i = i^-2                       (LowRankFastDecay)
  rank_plus_noise G1 (m x r) G2 (r x n) Gaussian + iid noise
  exp_decay       sigma_i = exp(-i / tau), r terms
  poly_decay      sigma_i = i^-alpha
  paper_low_rank_plus_noise, s_shaped, slow_decay, uniform01 -- the other
  Section 5 test matrices (see each docstring for the reading taken).
"""
import numpy as np

STREAM_U, STREAM_V, STREAM_NOISE, STREAM_G1, STREAM_G2, STREAM_PARAMS = 1, 2, 3, 4, 5, 6


def rng(seed, stream):
    return np.random.Generator(np.random.Philox(key=[int(seed), int(stream)]))


def haar(rows, cols, seed, stream):
    """rows x cols with orthonormal columns: sign-fixed QR of a Gaussian."""
    g = rng(seed, stream).standard_normal((rows, cols))
    q, r = np.linalg.qr(g)
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    return q * s[None, :]


def svd_matrix(m, n, sigma, seed):
    """A = U diag(sigma) V^T with Haar U (m x r) and V (n x r), r = len(sigma).

    Returns (A in Fortran order, U, sigma, V).
    """
    sigma = np.asarray(sigma, dtype=np.float64)
    r = sigma.size
    U = haar(m, r, seed, STREAM_U)
    V = haar(n, r, seed, STREAM_V)
    A = np.asfortranarray((U * sigma[None, :]) @ V.T)
    return A, U, sigma, V


def fast_decay(m, n, seed):
    """sigma_i = i^-2, i = 1..min(m, n)."""
    r = min(m, n)
    return svd_matrix(m, n, np.arange(1, r + 1, dtype=np.float64) ** -2.0, seed)


def exp_decay(m, n, r, tau, seed):
    """sigma_i = exp(-i / tau), i = 1..r (rank r)."""
    return svd_matrix(m, n, np.exp(-np.arange(1, r + 1, dtype=np.float64) / tau), seed)


def poly_decay(m, n, alpha, seed, r=None):
    """sigma_i = i^-alpha, i = 1..r (default min(m, n))."""
    r = min(m, n) if r is None else r
    return svd_matrix(m, n, np.arange(1, r + 1, dtype=np.float64) ** -float(alpha), seed)


def rank_plus_noise(m, n, r, rel_noise, seed):
    """A = G1 G2 + E, G1 (m x r), G2 (r x n), E iid N(0, s^2).

    s = rel_noise * ||G1 G2||_F / sqrt(m n): the noise level is set from the
    noiseless product (the alternative, ||A||_F of the noisy matrix, would be
    circular).  Singular triplets are not known exactly; returns (A, s).
    """
    g1 = rng(seed, STREAM_G1).standard_normal((m, r))
    g2 = rng(seed, STREAM_G2).standard_normal((r, n))
    A = np.asfortranarray(g1 @ g2)
    s = rel_noise * np.linalg.norm(A) / np.sqrt(float(m) * n)
    noise = rng(seed, STREAM_NOISE).standard_normal((n, m)).T   # column-major draw
    A += s * noise
    return A, s


def paper_low_rank_plus_noise(n, seed, k=200):
    """Section 5.2's LowRankPlusNoise: sigma linear from 1 to 1e-20 over the
    first k, zero after; plus 0.05 sigma_k G_N with G_N = N(0,1)/sqrt(n)
    (reading of "normalized Gaussian")."""
    sigma = np.zeros(n)
    sigma[:k] = np.linspace(1.0, 1e-20, k)
    A, U, s, V = svd_matrix(n, n, sigma, seed)
    g = rng(seed, STREAM_NOISE).standard_normal((n, n)) / np.sqrt(n)
    return np.asfortranarray(A + 0.05 * sigma[k - 1] * g)


def s_shaped(n, seed):
    """Section 5.2's LowRankS-ShapedDecay (no formula printed); reading:
    sigma_i = 0.01 + 0.99 / (1 + exp((i - n/4) / (n/40)))."""
    i = np.arange(1, n + 1, dtype=np.float64)
    return svd_matrix(n, n, 0.01 + 0.99 / (1.0 + np.exp((i - n / 4.0) / (n / 40.0))), seed)


def slow_decay(n, seed, k=100):
    """Section 5.2's LowRankSlowDecay: k ones, then 2^-1, ..., (n-k+1)^-1."""
    sigma = np.concatenate([np.ones(k), 1.0 / np.arange(2, n - k + 2, dtype=np.float64)])
    return svd_matrix(n, n, sigma, seed)


def uniform01(m, n, seed):
    """Section 5.1's runtime workload: dense entries uniform on (0, 1)."""
    return np.asfortranarray(rng(seed, STREAM_NOISE).random((n, m)).T)


def batch_specs(count, seed, lo=256, hi=4096, alpha=(0.5, 3.0), kr=(8, 128)):
    """Shapes and spectra for a batch of uneven matrices: m, n uniform in
    [lo, hi], alpha uniform in alpha, k uniform in kr.  Returns a list of dicts."""
    g = rng(seed, STREAM_PARAMS)
    out = []
    for _ in range(count):
        out.append({"m": int(g.integers(lo, hi + 1)), "n": int(g.integers(lo, hi + 1)),
                    "alpha": float(g.uniform(*alpha)), "k": int(g.integers(kr[0], kr[1] + 1))})
    return out


# ---- device-side generators (torch on the GPU) for the large workloads ----
# Same families as above, drawn with torch's device generator so that the
# 20000 x 16000 and batched workloads need no host-side QR.  They return
# column-major device tensors (stride (1, rows)).

def _device_haar(rows, cols, gen, dtype):
    import torch
    g = torch.randn(rows, cols, dtype=dtype, device="cuda", generator=gen)
    q, r = torch.linalg.qr(g)
    s = torch.sign(torch.diagonal(r))
    s[s == 0] = 1.0
    return q * s[None, :]


def device_svd_matrix(m, n, sigma, gen, dtype=None):
    """A = U diag(sigma) V^T on the device with Haar U (m x r), V (n x r)
    from the sign-fixed QR of torch Gaussians drawn from `gen`."""
    import torch
    dtype = dtype or torch.float64
    sigma = sigma.to(device="cuda", dtype=dtype)
    r = sigma.numel()
    U = _device_haar(m, r, gen, dtype)
    V = _device_haar(n, r, gen, dtype)
    A = (V * sigma[None, :]) @ U.T          # A^T (n x m), row-major = A column-major
    del U, V
    return A.t()


def device_exp_decay(m, n, r, tau, seed):
    """exp_decay on the device: sigma_i = exp(-i / tau), i = 1..r, fp64."""
    import torch
    gen = torch.Generator(device="cuda")
    gen.manual_seed(int(seed))
    sig = torch.exp(-torch.arange(1, r + 1, dtype=torch.float64) / float(tau))
    return device_svd_matrix(m, n, sig, gen)


def device_batch(count, seed, lo=256, hi=4096, alpha=(0.5, 3.0), kr=(8, 128)):
    """The batched workload on the device, fp32: specs from batch_specs and,
    per matrix, sigma_j = j^-alpha (j = 1..min(m, n)) with Haar factors.
    Returns (list of column-major float32 device tensors, specs)."""
    import torch
    specs = batch_specs(count, seed, lo, hi, alpha, kr)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(int(seed))
    As = []
    for sp in specs:
        r = min(sp["m"], sp["n"])
        sig = torch.arange(1, r + 1, dtype=torch.float32) ** (-sp["alpha"])
        As.append(device_svd_matrix(sp["m"], sp["n"], sig, gen, torch.float32))
    return As, specs


def sparse_standin(m, n, per_row, seed, band=2):
    """A sparse m x n stand-in for the sparse, square, non-symmetric test
    matrices of Section 5.1 (their entries are not reproduced): in each row
    the diagonal entry (when i < n), the entries within `band` of it, and
    `per_row` further columns drawn uniformly; values N(0, 1); duplicate
    positions merged.  Returns CSR arrays (rowptr int64, colind int32,
    vals float64), columns ascending within a row."""
    g = rng(seed, STREAM_NOISE)
    rowptr = np.zeros(m + 1, dtype=np.int64)
    cols, vals = [], []
    for i in range(m):
        c = list(range(max(0, i - band), min(n, i + band + 1))) if i < n + band else []
        c.extend(int(x) for x in g.integers(0, n, per_row))
        c = np.unique(np.asarray(c, dtype=np.int64))
        cols.append(c.astype(np.int32))
        vals.append(g.standard_normal(c.size))
        rowptr[i + 1] = rowptr[i] + c.size
    colind = np.concatenate(cols) if cols else np.zeros(0, np.int32)
    v = np.concatenate(vals) if vals else np.zeros(0)
    return rowptr, colind, v


def csr_to_dense(rowptr, colind, vals, m, n):
    """Dense column-major copy of a CSR matrix (for the dense checks)."""
    A = np.zeros((m, n), order="F")
    for i in range(m):
        a, b = rowptr[i], rowptr[i + 1]
        np.add.at(A, (i, colind[a:b]), vals[a:b])     # repeated positions add up
    return A

"""Helpers for the GPU parity tests: move column-major matrices across and
compute the sign-invariant comparison quantities against the oracle."""
import sys

import numpy as np

from oracle import rel_error, subspace_sine


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(A, dtype=None):
    import torch
    import paper_2110_01011_amd as rq
    A = np.asarray(A)
    t = torch.from_numpy(np.ascontiguousarray(A.T))  # (n, m) row-major == A column-major
    if dtype is not None:
        t = t.to(dtype)
    t = t.cuda()
    out = t.t()
    assert out.stride(0) == 1
    return rq.colmajor(out)


def to_np(t):
    return t.detach().double().cpu().numpy()


def compare(A, Qg, Lg, Pg, Qo, Lo, Po, k):
    """Differences of the sign-invariant quantities (GPU vs oracle)."""
    e_g = rel_error(A, Qg, Lg, Pg)
    e_o = rel_error(A, Qo, Lo, Po)
    sg, so = np.abs(np.diag(Lg)), np.abs(np.diag(Lo))
    return {
        "e_gpu": e_g, "e_orc": e_o, "de": abs(e_g - e_o),
        "dsigma": float(np.max(np.abs(sg - so)) / so[0]) if so[0] > 0 else float(np.max(np.abs(sg))),
        "sinQk": subspace_sine(Qo[:, :k], Qg[:, :k]),
        "sinPk": subspace_sine(Po[:, :k], Pg[:, :k]),
        "sinQ": subspace_sine(Qo, Qg),
        "sinP": subspace_sine(Po, Pg),
    }


def invariants(A, Q, L, P):
    d = L.shape[0]
    return {
        "orthQ": float(np.abs(Q.T @ Q - np.eye(d)).max()),
        "orthP": float(np.abs(P.T @ P - np.eye(d)).max()),
        "upper_max": float(np.abs(np.triu(L, 1)).max()) if d > 1 else 0.0,
        "min_diag": float(np.diag(L).min()),
        "L_vs_QtAP": float(np.abs(L - Q.T @ A @ P).max() / max(np.abs(L).max(), 1e-300)),
    }

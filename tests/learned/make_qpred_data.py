"""Training and validation data for the power-iteration predictor.

Writes tests/learned/qpred_data.npz: for each sample a spectrum drawn from
one of three families, the 65 sketch features and the label (the smallest q
in 0..4 whose rank-k QLP approximation error meets 1.05 x the rank-k
optimum, 5 if none), all
computed by the fp64 oracle on the diagonal surrogate A = diag(sigma) (a
Gaussian sketch is rotation invariant, so the error of U diag(sigma) V^T has
the same distribution).

Families (m, n uniform in 2000..8000, k uniform in 8..256, p = 10):
  poly        sigma_j = j^-alpha,                alpha ~ U[0.5, 3]
  exp         sigma_j = exp(-(j - 1) / tau),     tau = k * 10^U[-0.6, 0.8]
  rank_noise  r0 ~ U{k/2..2k} signal values log-spaced from 1 down to
              10^-U[0, 2], then a noise floor nu (1 - j / (2 r)) with
              nu = sigma_r0 * 10^-U[0.3, 3], added in quadrature
Each sample i draws its parameters from numpy's Philox keyed (base, i) and
its sketch from the library's Philox stream with seed i.

Usage: python tests/learned/make_qpred_data.py [count] [workers]
"""
import os
import sys
import time
from multiprocessing import Pool

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "qpred_data.npz")
BASE = 20211004
FAMILIES = ("poly", "exp", "rank_noise")
P, QMAX = 10, 4


def spectrum(i):
    import numpy as np
    rng = np.random.Generator(np.random.Philox(key=[BASE, i]))
    fam = FAMILIES[i % 3]
    m = int(rng.integers(2000, 8001))
    n = int(rng.integers(2000, 8001))
    k = int(rng.integers(8, 257))
    r = min(m, n)
    j = np.arange(1, r + 1, dtype=np.float64)
    if fam == "poly":
        s = j ** -rng.uniform(0.5, 3.0)
    elif fam == "exp":
        tau = k * 10.0 ** rng.uniform(-0.6, 0.8)
        s = np.exp(-(j - 1.0) / tau)
    else:
        r0 = int(rng.integers(max(1, k // 2), 2 * k + 1))
        sig = np.logspace(0.0, -rng.uniform(0.0, 2.0), r0)
        nu = sig[-1] * 10.0 ** -rng.uniform(0.3, 3.0)
        floor = nu * (1.0 - j / (2.0 * r))
        s = np.sqrt(np.concatenate([sig ** 2, np.zeros(r - r0)]) + floor ** 2)
    return fam, m, n, k, s


def sample(i):
    import numpy as np
    os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")
    from oracle.learned import label_q, qlp_errors_diag, sketch_features_diag
    fam, m, n, k, s = spectrum(i)
    f = sketch_features_diag(s, m, n, k, seed=i)
    e, ek = qlp_errors_diag(s, m, n, k, P, QMAX, seed=i)
    return i, FAMILIES.index(fam), m, n, k, f, np.stack([e, ek]), label_q(ek, s, k)


def main():
    import numpy as np
    count = int(sys.argv[1]) if len(sys.argv) > 1 else 20000
    workers = int(sys.argv[2]) if len(sys.argv) > 2 else 6
    t0 = time.time()
    rows = []
    with Pool(workers) as pool:
        for r in pool.imap_unordered(sample, range(count), chunksize=8):
            rows.append(r)
            if len(rows) % 500 == 0:
                print(f"{len(rows)}/{count} samples, {time.time() - t0:.0f} s", flush=True)
    rows.sort(key=lambda r: r[0])
    np.savez_compressed(
        OUT, X=np.array([r[5] for r in rows], dtype=np.float32),
        y=np.array([r[7] for r in rows], dtype=np.int32),
        family=np.array([r[1] for r in rows], dtype=np.int8),
        m=np.array([r[2] for r in rows], dtype=np.int32),
        n=np.array([r[3] for r in rows], dtype=np.int32),
        k=np.array([r[4] for r in rows], dtype=np.int32),
        errors=np.array([r[6] for r in rows], dtype=np.float64))  # [i, 0|1, q]: e, e_k
    y = np.array([r[7] for r in rows])
    print("labels:", np.bincount(y, minlength=QMAX + 2), f"{time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()

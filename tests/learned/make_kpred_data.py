"""Training and validation data for the rank network of the predictor.

Writes tests/learned/kpred_data.npz.  The spectra are those of the
power-round dataset (make_qpred_data.spectrum(i): the same three families,
sizes and seeds), so the 64 spectrum features are that dataset's (written by
the fp64 oracle on the diagonal surrogate).  Each sample gets two target
errors drawn from numpy's Philox keyed (BASE, i) around the spectrum's own
range of rank-k errors, so that the labels spread over the classes: a rank
k_t = 8 * 2^u with u ~ U[-0.5, 5.5], then tol = 1.05 * (Eckart-Young error
at k_t) * 10^U[-0.2, 0.2], clipped to [1e-4, 0.9]; the
input row is the 64 features followed by oracle.learned.rank_feature(tol),
and the label is oracle.learned.label_rank(sigma, tol): the smallest of the
ranks 8, 16, ..., 256 whose Eckart-Young error is at most tol / 1.05 (the
last class if none).

Usage: python tests/learned/make_kpred_data.py   (after make_qpred_data.py)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)
QDATA = os.path.join(HERE, "qpred_data.npz")
OUT = os.path.join(HERE, "kpred_data.npz")
BASE = 20211005
PER_SAMPLE = 2


def main():
    from make_qpred_data import spectrum
    from oracle.learned import RANK_CLASSES, label_rank, optimal_error, rank_feature
    q = np.load(QDATA)
    X64 = q["X"][:, :64]
    t0 = time.time()
    X, y, src, tols = [], [], [], []
    for i in range(X64.shape[0]):
        fam, m, n, k, s = spectrum(i)
        rng = np.random.Generator(np.random.Philox(key=[BASE, i]))
        for _ in range(PER_SAMPLE):
            kt = max(1, int(round(8.0 * 2.0 ** rng.uniform(-0.5, 5.5))))
            tol = 1.05 * optimal_error(s, kt) * 10.0 ** rng.uniform(-0.2, 0.2)
            tol = float(np.clip(tol, 1e-4, 0.9))
            X.append(np.concatenate([X64[i], [rank_feature(tol)]]))
            y.append(label_rank(s, tol))
            src.append(i)
            tols.append(tol)
        if (i + 1) % 2000 == 0:
            print(f"{i + 1}/{X64.shape[0]} spectra, {time.time() - t0:.0f} s", flush=True)
    y = np.array(y, dtype=np.int32)
    np.savez_compressed(OUT, X=np.array(X, dtype=np.float32), y=y,
                        sample=np.array(src, dtype=np.int32), tol=np.array(tols))
    print("labels (ranks " + ", ".join(map(str, RANK_CLASSES)) + "):",
          np.bincount(y, minlength=len(RANK_CLASSES)), f"{time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()

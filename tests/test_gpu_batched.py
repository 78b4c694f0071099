"""GPU parity of the batched form: every matrix of a grouped, graph-replayed
batch against the fp64 oracle method on that matrix."""
import numpy as np
import pytest

import workloads as W
from oracle import randqlp, rel_error
from tests.gpu_util import compare, invariants, log, to_dev, to_np

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module")
def rq():
    import paper_2110_01011_amd as rq
    rq.lib()
    return rq


def _batch_specs(count, seed, mlo=60, mhi=900, kmax=60):
    r = np.random.default_rng(seed)
    specs = []
    for i in range(count):
        m, n = int(r.integers(mlo, mhi)), int(r.integers(mlo, mhi))
        k = int(r.integers(3, min(kmax, m, n) + 1))
        alpha = float(r.uniform(0.5, 3.0))
        specs.append((m, n, k, alpha))
    return specs


def _mats(specs, seed):
    return [W.poly_decay(m, n, a, seed=seed + i)[0] for i, (m, n, k, a) in enumerate(specs)]


@pytest.mark.parametrize("q", [0, 2])
def test_batched_f64_parity(rq, q):
    specs = _batch_specs(14, 1 + q)
    mats = _mats(specs, 100)
    ks = [s[2] for s in specs]
    seeds = [1000 + i for i in range(len(specs))]
    log(f"batched f64 q={q}: {[(s[0], s[1], s[2]) for s in specs]}")
    b = rq.Batch([to_dev(A) for A in mats], ks, 5, q, seeds)
    Qs, Ls, Ps = b.run()
    info = b.info()
    log(f"  info {info}")
    assert info["grouped"] == len(specs)
    for A, k, sd, Qg, Lg, Pg in zip(mats, ks, seeds, Qs, Ls, Ps):
        Qo, Lo, Po = randqlp(A, k, 5, q, sd)
        Qg, Lg, Pg = to_np(Qg), to_np(Lg), to_np(Pg)
        c = compare(A, Qg, Lg, Pg, Qo, Lo, Po, min(k, Lo.shape[0]))
        inv = invariants(A, Qg, Lg, Pg)
        assert c["de"] <= TOL and c["dsigma"] <= TOL, c
        assert c["sinQk"] <= TOL and c["sinPk"] <= TOL and c["sinQ"] <= TOL and c["sinP"] <= TOL, c
        assert inv["orthQ"] < 1e-12 and inv["orthP"] < 1e-12
        assert inv["upper_max"] == 0.0 and inv["min_diag"] >= 0.0
    # graph replay and direct launches give the same bits; so does a re-run
    ref = [to_np(t).copy() for t in Ls]
    b.run(use_graph=False)
    assert all(np.array_equal(to_np(t), r) for t, r in zip(Ls, ref))
    b.run()
    assert all(np.array_equal(to_np(t), r) for t, r in zip(Ls, ref))
    b.close()


def test_batched_f32_error_within_5_percent(rq):
    import torch
    specs = _batch_specs(10, 7, mlo=200, mhi=1500, kmax=120)
    mats = _mats(specs, 300)
    ks = [s[2] for s in specs]
    seeds = list(range(10))
    Qs, Ls, Ps, info = rq.factor_batched([to_dev(A, torch.float32) for A in mats], ks, 10, 2,
                                         seeds, tune=True)
    log(f"  f32 batch info {info}")
    for A, k, sd, Qg, Lg, Pg in zip(mats, ks, seeds, Qs, Ls, Ps):
        e_g = rel_error(A, to_np(Qg), to_np(Lg), to_np(Pg))
        e_o = rel_error(A, *randqlp(A, k, 10, 2, sd))
        assert e_g <= 1.05 * e_o
        inv = invariants(A, to_np(Qg), to_np(Lg), to_np(Pg))
        assert inv["orthQ"] < 1e-5 and inv["orthP"] < 1e-5


def test_batched_fallbacks_wide_and_deficient(rq):
    """A matrix with d > 224 and an exactly rank-deficient one are refactored
    on their own; both still match the oracle's unique quantities."""
    A1 = W.poly_decay(600, 500, 1.0, seed=1)[0]                  # d = 240 > 224
    A2 = np.zeros((150, 120))                                    # zero: dependent pivots
    A3 = W.fast_decay(300, 200, seed=3)[0]
    mats, ks, seeds = [A1, A2, A3], [230, 8, 12], [5, 6, 7]
    Qs, Ls, Ps, info = rq.factor_batched([to_dev(A) for A in mats], ks, 10, 1, seeds)
    log(f"  fallback info {info}")
    assert info["grouped"] == 2 and info["fallbacks"] == 2
    Qo, Lo, Po = randqlp(A1, 230, 10, 1, 5)
    c = compare(A1, to_np(Qs[0]), to_np(Ls[0]), to_np(Ps[0]), Qo, Lo, Po, 230)
    assert c["de"] <= TOL and c["dsigma"] <= TOL
    assert np.all(to_np(Ls[1]) == 0.0)
    inv = invariants(A2, to_np(Qs[1]), to_np(Ls[1]), to_np(Ps[1]))
    assert inv["orthQ"] < 1e-12 and inv["orthP"] < 1e-12
    Qo, Lo, Po = randqlp(A3, 12, 10, 1, 7)
    c = compare(A3, to_np(Qs[2]), to_np(Ls[2]), to_np(Ps[2]), Qo, Lo, Po, 12)
    assert c["de"] <= TOL and c["sinQ"] <= TOL


def test_tune_table_roundtrip(rq, tmp_path):
    import torch
    specs = _batch_specs(6, 11, mlo=300, mhi=800)
    mats = _mats(specs, 500)
    b = rq.Batch([to_dev(A, torch.float32) for A in mats], [s[2] for s in specs], 5, 1,
                 list(range(6)), tune=True)
    info = b.info()
    b.close()
    path = tmp_path / "tune.txt"
    rq.tune_save(path)
    lines = [l.split() for l in path.read_text().splitlines() if not l.startswith("#")]
    assert ["1", "1", str(info["dmax"] if info["dmax"] > 128 else
                            [x for x in (32, 64, 128) if info["dmax"] <= x][0]),
            str(info["wn_tn"])] in lines
    rq.tune_load(path)
    b2 = rq.Batch([to_dev(A, torch.float32) for A in mats], [s[2] for s in specs], 5, 1,
                  list(range(6)))
    assert b2.info()["wn_tn"] == info["wn_tn"] and b2.info()["wn_nn"] == info["wn_nn"]
    b2.close()


def test_batched_wide_and_full_width(rq):
    """m < n matrices and full-width sketches (d = min(m, n)) in one batch."""
    mats = [W.poly_decay(80, 200, 1.0, seed=31)[0], W.poly_decay(60, 60, 0.8, seed=32)[0],
            W.fast_decay(150, 500, seed=33)[0], W.uniform01(40, 90, seed=34)]
    ks, seeds = [10, 60, 150, 40], [11, 12, 13, 14]
    Qs, Ls, Ps, info = rq.factor_batched([to_dev(A) for A in mats], ks, 5, 1, seeds)
    log(f"  wide/full info {info}")
    for A, k, sd, Qg, Lg, Pg in zip(mats, ks, seeds, Qs, Ls, Ps):
        Qo, Lo, Po = randqlp(A, k, 5, 1, sd)
        c = compare(A, to_np(Qg), to_np(Lg), to_np(Pg), Qo, Lo, Po, min(k, Lo.shape[0]))
        assert c["de"] <= TOL and c["dsigma"] <= TOL, c
        if Lo.shape[0] == min(A.shape):
            assert rel_error(A, to_np(Qg), to_np(Lg), to_np(Pg)) < 1e-11

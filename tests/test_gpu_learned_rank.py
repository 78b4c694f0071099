"""GPU checks of the rank half of the predictor (randqlp_factor_auto with
k <= 0): both networks in one launch against the fp64 oracle MLP, forced
predictions against the oracle method (rank check and fallback included),
and the trained networks meeting the tolerance on fresh matrices."""
import os

import numpy as np
import pytest

import workloads as W
from oracle import mlp, randqlp
from oracle.learned import rank_errors, rank_features, sketch_features, smallest_rank
from tests.gpu_util import compare, invariants, log, to_dev, to_np

pytestmark = pytest.mark.gpu
TOL = 1e-10
HERE = os.path.dirname(os.path.abspath(__file__))
KDATA = os.path.join(HERE, "learned", "kpred_data.npz")


@pytest.fixture(scope="module")
def rq():
    import paper_2110_01011_amd as rq
    rq.lib()
    return rq


def _t(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def _params(seed):
    th = mlp.init_params(seed)
    th += 0.05 * np.random.default_rng(seed).standard_normal(th.size)
    return th


def _forced(n_params, cls):
    th = np.zeros(n_params)
    th[-6:] = -10.0
    th[-6 + cls] = 10.0
    return th


def _oracle_classes(A, seed, tol, k_max, thq, thk):
    """(rank class, k_hat, q class, the two logit margins) of the oracle MLP."""
    f = sketch_features(A, 1, seed)
    zk, _ = mlp.forward(thk, rank_features(f, tol)[None, :])
    ck = int(np.argmax(zk[0]))
    khat = min(8 << ck, k_max)
    xq = np.concatenate([f[:64], [khat / 256.0]])
    zq, _ = mlp.forward(thq, xq[None, :])
    mk = np.diff(np.sort(zk[0])[-2:])[0]
    mq = np.diff(np.sort(zq[0])[-2:])[0]
    return ck, khat, int(np.argmax(zq[0])), mk, mq


def test_rank_and_q_networks_match_oracle_mlp(rq):
    """The rank network's class, k_hat and the power-round class that
    randqlp_factor_auto(k = 0) reports equal the oracle MLP's on the
    oracle's features.  Random parameters; inputs with a logit margin under
    1e-2 are passed over."""
    thq, thk = _params(21), _params(22)
    both = _t(np.concatenate([thq, thk]))
    checked = 0
    for i, (m, n, a, tol) in enumerate([(900, 700, 0.8, 0.3), (1200, 500, 1.5, 0.05),
                                        (600, 800, 2.5, 0.01), (1500, 300, 1.0, 0.1),
                                        (800, 800, 0.6, 0.5), (1000, 900, 2.0, 0.002)]):
        A, U, s, V = W.poly_decay(m, n, a, seed=40 + i)
        seed = 3 + i
        ck, khat, cq, mk, mq = _oracle_classes(A, seed, tol, 256, thq, thk)
        Qg, Lg, Pg, info, ai = rq.factor_auto(to_dev(A), 0, 10, seed, both, q_fallback=2,
                                              tol=tol, k_max=256, return_info=True)
        log(f"  {m}x{n} a={a} tol={tol}: oracle k_hat {khat} q {cq} (margins {mk:.2e} "
            f"{mq:.2e}); library k_hat {ai['k_predicted']} q {ai['q_predicted']} d {ai['d']} "
            f"k_used {ai['k_used']}")
        if mk < 1e-2 or mq < 1e-2:
            continue
        assert ai["k_predicted"] == khat and ai["q_predicted"] == cq
        checked += 1
    assert checked >= 3


def _check_rank_result(A, Qg, Lg, Pg, ai, k_run, p, q, seed, tol):
    """Factors equal the oracle method's at (k_run, q); k_used equals the
    oracle's smallest rank under tol (dense rank-k errors)."""
    Qo, Lo, Po = randqlp(A, k_run, p, q, seed)
    c = compare(A, Qg, Lg, Pg, Qo, Lo, Po, min(k_run, Lo.shape[0]))
    inv = invariants(A, Qg, Lg, Pg)
    log(f"    vs oracle (k={k_run}, q={q}): {c}")
    assert Lg.shape == Lo.shape
    assert c["de"] <= TOL and c["dsigma"] <= TOL
    assert c["sinQk"] <= TOL and c["sinPk"] <= TOL and c["sinQ"] <= TOL and c["sinP"] <= TOL
    assert inv["orthQ"] < 1e-12 and inv["orthP"] < 1e-12
    ek = rank_errors(A, Qo, Lo, Po)
    k_o = smallest_rank(ek, tol)
    log(f"    k_used {ai['k_used']} (oracle {k_o}), rank_err {ai['rank_err']:.6e} "
        f"(oracle e_k {ek[ai['k_used'] - 1]:.6e})")
    near = np.abs(ek - tol) < 1e-9
    if not near[max(k_o - 2, 0):k_o + 1].any():
        assert ai["k_used"] == k_o
    assert abs(ai["rank_err"] - ek[ai["k_used"] - 1]) < 1e-7
    return ek


def test_forced_rank_accepts_and_matches_oracle(rq):
    """Rank class 3 (k_hat = 64) and q class 1 forced on a fast decay whose
    rank-64 error is far under tol: no fallback; the factors are the oracle
    method's with k = 64 (d = 74) at the q the judge settles on."""
    A, U, s, V = W.poly_decay(1100, 900, 2.0, seed=51)
    th = _t(np.concatenate([_forced(25734, 1), _forced(25734, 3)]))
    tol = 0.02
    Qg, Lg, Pg, info, ai = rq.factor_auto(to_dev(A), 0, 10, 5, th, q_fallback=2, tol=tol,
                                          k_max=200, return_info=True)
    log(f"  forced k=64: {ai}")
    assert ai["k_predicted"] == 64 and ai["d"] == 74 and ai["rank_fallback"] == 0
    assert ai["q_predicted"] == 1 and ai["q_used"] in (1, 2)
    assert ai["rank_err"] <= tol
    _check_rank_result(A, to_np(Qg), to_np(Lg), to_np(Pg), ai, 64, 10, ai["q_used"], 5, tol)


def test_forced_rank_too_low_falls_back_to_k_max(rq):
    """Rank class 0 (k_hat = 8) forced on a slow decay with a tolerance no
    rank below 18 can meet: the check finds no rank <= d = 18 under tol and
    the method reruns with k_max = 120 and q_fallback = 2."""
    A, U, s, V = W.poly_decay(1000, 800, 1.0, seed=52)
    th = _t(np.concatenate([_forced(25734, 0), _forced(25734, 0)]))
    tol = 0.12
    Qg, Lg, Pg, info, ai = rq.factor_auto(to_dev(A), 0, 10, 6, th, q_fallback=2, tol=tol,
                                          k_max=120, return_info=True)
    log(f"  forced k=8: {ai}")
    assert ai["k_predicted"] == 8 and ai["rank_fallback"] == 1
    assert ai["d"] == 130 and ai["q_used"] == 2
    _check_rank_result(A, to_np(Qg), to_np(Lg), to_np(Pg), ai, 120, 10, 2, 6, tol)


@pytest.mark.parametrize("shape", [(200, 60), (60, 300)])
def test_rank_mode_small_shapes(rq, shape):
    """min(m, n) below the predicted width: d = min(k_hat + p, m, n)."""
    m, n = shape
    A, U, s, V = W.poly_decay(m, n, 1.2, seed=m)
    th = _t(np.concatenate([_forced(25734, 0), _forced(25734, 5)]))
    Qg, Lg, Pg, info, ai = rq.factor_auto(to_dev(A), 0, 5, 2, th, q_fallback=2, tol=0.05,
                                          k_max=256, return_info=True)
    log(f"  {m}x{n}: {ai}")
    assert ai["k_predicted"] == 256 and ai["d"] == min(m, n)
    _check_rank_result(A, to_np(Qg), to_np(Lg), to_np(Pg), ai, 256, 5, ai["q_used"], 2, 0.05)


@pytest.fixture(scope="module")
def trained_rank(rq):
    if not os.path.exists(KDATA):
        pytest.skip("rank training data not generated (tests/learned/make_kpred_data.py)")
    from paper_2110_01011_amd.train_predictor import train
    params, summary = train(KDATA, epochs=(40, 20))
    log(f"  rank training summary {summary}")
    return params, summary


def test_rank_training_beats_the_majority_class(trained_rank):
    params, s = trained_rank
    counts = np.array(s["label_counts"], dtype=float)
    assert s["loss_last"] < 0.7 * s["loss_first"]
    assert s["validation_accuracy"] > counts.max() / counts.sum() + 0.2


def test_trained_predictor_meets_tolerance(rq, trained_rank):
    """Both trained networks on fresh matrices (seeds unused by the data):
    the returned factors' rank-k_used approximation meets tol, computed
    densely on the host, and the oracle method run at (k_hat, q_used) with
    the same seed meets it at the same rank."""
    import torch
    thq = np.load(os.path.join(os.path.dirname(rq.__file__), "qpredictor.npy"))
    thk, _ = trained_rank
    both = torch.from_numpy(np.concatenate([thq, thk]).astype(np.float32)).cuda()
    m, n = 2400, 2000
    j = np.arange(1, n + 1, dtype=np.float64)
    cases = [("poly1.0", j ** -1.0, 0.1), ("poly2.0", j ** -2.0, 0.003),
             ("exp30", np.exp(-(j - 1) / 30.0), 0.01), ("exp100", np.exp(-(j - 1) / 100.0), 0.2)]
    for i, (name, sig, tol) in enumerate(cases):
        A = W.svd_matrix(m, n, sig, seed=930 + i)[0]
        Qg, Lg, Pg, info, ai = rq.factor_auto(to_dev(A), 0, 10, 7, both, q_fallback=2, tol=tol,
                                              k_max=256, return_info=True)
        Qg, Lg, Pg = to_np(Qg), to_np(Lg), to_np(Pg)
        ku = ai["k_used"]
        e_g = np.linalg.norm(A - Qg @ (Lg[:, :ku] @ Pg[:, :ku].T)) / np.linalg.norm(A)
        k_opt = next(k for k in range(1, n + 1) if np.sqrt(np.sum(sig[k:] ** 2) / np.sum(sig ** 2)) <= tol)
        log(f"  {name} tol={tol}: k_hat {ai['k_predicted']} q {ai['q_predicted']}->{ai['q_used']} "
            f"d {ai['d']} k_used {ku} (optimal rank {k_opt}) e {e_g:.4e} fallback "
            f"{ai['rank_fallback']}")
        assert e_g <= tol * (1 + 1e-9)
        k_run = ai["d"] - 10 if ai["d"] < min(m, n) else ai["d"]
        Qo, Lo, Po = randqlp(A, k_run, 10, ai["q_used"], 7)
        e_o = np.linalg.norm(A - Qo @ (Lo[:, :ku] @ Po[:, :ku].T)) / np.linalg.norm(A)
        assert e_o <= tol * (1 + 1e-9) and abs(e_o - e_g) < 1e-10

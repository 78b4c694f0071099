"""What the trained predictor gains: trained on the GPU by the library's own
kernels from the oracle-labelled dataset, then randqlp_factor_auto with it
against the same call with constant predictions (same judge) and against
fixed q = 2, on fresh matrices of the three training families."""
import os

import numpy as np
import pytest

import workloads as W
from oracle import rel_error
from tests.gpu_util import log, to_dev, to_np

pytestmark = pytest.mark.gpu
DATA = os.path.join(os.path.dirname(__file__), "learned", "qpred_data.npz")


@pytest.fixture(scope="module")
def rq():
    import paper_2110_01011_amd as rq
    rq.lib()
    return rq


@pytest.fixture(scope="module")
def trained(rq):
    if not os.path.exists(DATA):
        pytest.skip("training data not generated (tests/learned/make_qpred_data.py)")
    from paper_2110_01011_amd.train_predictor import train
    params, summary = train(DATA, epochs=(40, 20))
    log(f"  training summary {summary}")
    return params, summary


def test_training_beats_the_majority_class(trained):
    params, s = trained
    counts = np.array(s["label_counts"], dtype=float)
    majority = counts.max() / counts.sum()
    assert s["loss_last"] < 0.7 * s["loss_first"]
    assert s["validation_accuracy"] > majority + 0.05
    # too-low predictions (mostly a true 2 read as 1) only cost a judged
    # resume; measured ~11% of the validation set
    assert s["validation_under"] < 0.15


def _eval_matrices():
    """18 fresh matrices (seeds unused by the dataset), six of each training
    family, with the family's parameter and k drawn from a seeded generator."""
    out = []
    m, n = 2400, 2000
    j = np.arange(1, n + 1, dtype=np.float64)
    rng = np.random.default_rng(77)
    for i in range(18):
        k = int(rng.integers(16, 200))
        if i % 3 == 0:
            a = rng.uniform(0.5, 3.0)
            out.append((f"poly{a:.2f}", W.svd_matrix(m, n, j ** -a, seed=950 + i)[0], k))
        elif i % 3 == 1:
            tau = k * 10 ** rng.uniform(-0.6, 0.8)
            out.append((f"exp{tau:.0f}", W.svd_matrix(m, n, np.exp(-(j - 1) / tau),
                                                      seed=950 + i)[0], k))
        else:
            noise = 10 ** -rng.uniform(1, 3)
            out.append((f"rank{k}+noise", W.rank_plus_noise(m, n, k, noise, seed=950 + i)[0], k))
    return out


def _constant(rq, cls):
    """Parameters that predict `cls` for every input (W3 = 0)."""
    import torch
    th = np.zeros(rq.MLP_PARAMS, dtype=np.float32)
    th[-6:] = -10.0
    th[-6 + cls] = 10.0
    return torch.from_numpy(th).cuda()


def _products(ai, q_fallback=2):
    """Products with A a call ran: 2 q + 3 for the method, plus the judge's
    A P when it accepted; a resumed run reuses the judge's product as its
    next round's, so it costs what the fixed-q_fallback method costs."""
    if ai["judged"] and not ai["resumed"]:
        return 2 * ai["q_used"] + 4
    return 2 * q_fallback + 3


def test_learned_q_beats_every_constant_prediction(rq, trained):
    """The trained network against the constant predictions q = 0, 1, 2
    under the same judge, on 18 fresh matrices: every error within 1.05x
    the fixed q = 2 method's, and fewer products with A in total than the
    best constant (time is logged; products are what the prediction
    decides)."""
    import time

    import torch
    params, _ = trained
    preds = {"mlp": torch.from_numpy(params).cuda()}
    for c in (0, 1, 2):
        preds[f"q={c}"] = _constant(rq, c)
    total = {p: [0, 0.0] for p in preds}
    for name, A, k in _eval_matrices():
        Ad = to_dev(A)
        e2 = rel_error(A, *(to_np(x) for x in rq.factor(Ad, k, 10, 2, 3)))
        row = []
        for p, th in preds.items():
            rq.factor_auto(Ad, k, 10, 3, th, q_fallback=2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Qa, La, Pa, info, ai = rq.factor_auto(Ad, k, 10, 3, th, q_fallback=2,
                                                  return_info=True)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            ea = rel_error(A, to_np(Qa), to_np(La), to_np(Pa))
            assert ea <= 1.05 * e2, (name, p)
            total[p][0] += _products(ai)
            total[p][1] += t
            row.append(f"{p}: q {ai['q_predicted']}->{ai['q_used']} e/e2 {ea / e2:.4f}")
        log(f"  {name} k={k}: " + "; ".join(row))
    for p, (prods, t) in total.items():
        log(f"  {p}: {prods} products with A, {t * 1e3:.2f} ms")
    best_constant = min(total[p][0] for p in preds if p != "mlp")
    assert total["mlp"][0] < best_constant

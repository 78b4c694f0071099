"""Train a predictor network on the GPU with the library's kernels.

Usage: python -m paper_2110_01011_amd.train_predictor data.npz out.npy

Reads a dataset of (65 inputs, label) pairs from data.npz (arrays X and y:
the power-round labels written by make_qpred_data.py, or the rank labels
written by make_kpred_data.py, both under tests/learned), holds out every
tenth sample for validation, trains the MLP with randqlp_mlp_train (softmax
cross-entropy, Adam, deterministic minibatch order) and writes the float32
parameter vector (RQLP_MLP_PARAMS values, the layout randqlp_factor_auto
reads) to out.npy, with a JSON summary next to it.  The package ships the
two trained vectors as qpredictor.npy (power rounds) and kpredictor.npy
(rank).
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SIZES = (65, 128, 128, 6)


def init_params(seed):
    """He-uniform weights (fan_in), zero biases, in the library's layout."""
    rng = np.random.Generator(np.random.Philox(key=[int(seed), 11]))
    parts = []
    for a, b in zip(SIZES[:-1], SIZES[1:]):
        lim = np.sqrt(6.0 / a)
        parts.append(rng.uniform(-lim, lim, a * b))   # column by column
        parts.append(np.zeros(b))
    return np.concatenate(parts).astype(np.float32)


def split(n):
    idx = np.arange(n)
    val = idx % 10 == 9
    return idx[~val], idx[val]


def train(data_path, epochs=(60, 30), lrs=(2e-3, 4e-4), batch=256, seed=1):
    """Returns (params as float32 numpy, summary dict)."""
    import torch

    import paper_2110_01011_amd as rq
    d = np.load(data_path)
    X, y = d["X"].astype(np.float32), d["y"].astype(np.int32)
    tr, va = split(len(y))
    dev = "cuda"
    Xt = torch.from_numpy(X[tr]).to(dev)
    yt = torch.from_numpy(y[tr]).to(dev)
    th = torch.from_numpy(init_params(seed)).to(dev)
    m = torch.zeros_like(th)
    v = torch.zeros_like(th)
    step = 0
    losses = []
    for ep, lr in zip(epochs, lrs):
        l, step = rq.mlp_train(th, m, v, Xt, yt, ep, batch, lr, seed + len(losses), step)
        losses.extend(l.cpu().numpy().tolist())
    torch.cuda.synchronize()

    def predict(idx):
        logits = rq.mlp_forward(th, torch.from_numpy(X[idx]).to(dev))
        return logits.argmax(dim=1).cpu().numpy()

    ptr, pva = predict(tr), predict(va)
    conf = np.zeros((6, 6), dtype=int)
    for a, b in zip(y[va], pva):
        conf[a, b] += 1
    summary = {
        "samples": int(len(y)), "train": int(len(tr)), "validation": int(len(va)),
        "epochs": int(sum(epochs)), "batch": batch, "lr": list(lrs), "adam_steps": int(step),
        "loss_first": losses[0], "loss_last": losses[-1],
        "train_accuracy": float(np.mean(ptr == y[tr])),
        "validation_accuracy": float(np.mean(pva == y[va])),
        "validation_under": float(np.mean(pva < y[va])),
        "validation_over": float(np.mean(pva > y[va])),
        "validation_confusion": conf.tolist(),
        "label_counts": np.bincount(y, minlength=6).tolist(),
    }
    return th.cpu().numpy(), summary


def main():
    if len(sys.argv) != 3:
        sys.exit("usage: python -m paper_2110_01011_amd.train_predictor data.npz out.npy")
    data, out = sys.argv[1], sys.argv[2]
    params, summary = train(data)
    np.save(out, params.astype(np.float32))
    with open(os.path.splitext(out)[0] + ".json", "w") as f:
        json.dump(summary, f, indent=1)
    print(json.dumps(summary))


if __name__ == "__main__":
    main()

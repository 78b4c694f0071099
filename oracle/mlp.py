"""Plain fp64 numpy MLP for the power-iteration predictor (test infrastructure).

Network: 65 inputs -> 128 (ReLU) -> 128 (ReLU) -> 6 logits, trained with the
mean softmax cross-entropy and Adam.  The flat parameter vector is
[W1, b1, W2, b2, W3, b3] with each W (fan_in x fan_out) stored column by
column (the fan_in weights of one output unit are contiguous), the layout the
library's kernels use.  Used to check the GPU forward pass, gradients and
optimiser steps element by element.
"""
import numpy as np

SIZES = (65, 128, 128, 6)


def param_count(sizes=SIZES):
    return sum(a * b + b for a, b in zip(sizes[:-1], sizes[1:]))


def unpack(theta, sizes=SIZES):
    theta = np.asarray(theta, dtype=np.float64)
    out, off = [], 0
    for a, b in zip(sizes[:-1], sizes[1:]):
        W = theta[off:off + a * b].reshape((a, b), order="F")
        off += a * b
        bias = theta[off:off + b]
        off += b
        out.append((W, bias))
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.flatten(order="F"), b]) for W, b in layers])


def init_params(seed, sizes=SIZES):
    """He-uniform weights, zero biases (numpy Philox stream, seeded)."""
    rng = np.random.Generator(np.random.Philox(key=[int(seed), 7]))
    layers = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        lim = np.sqrt(6.0 / a)
        layers.append((rng.uniform(-lim, lim, (a, b)), np.zeros(b)))
    return pack(layers)


def forward(theta, X):
    """Logits (B x 6) and the hidden activations."""
    (W1, b1), (W2, b2), (W3, b3) = unpack(theta)
    H1 = np.maximum(X @ W1 + b1, 0.0)
    H2 = np.maximum(H1 @ W2 + b2, 0.0)
    return H2 @ W3 + b3, (H1, H2)


def loss_and_grad(theta, X, y):
    """Mean cross-entropy of softmax(logits) against integer labels y, and
    its gradient with respect to theta (backpropagation written out)."""
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.int64)
    B = X.shape[0]
    (W1, b1), (W2, b2), (W3, b3) = unpack(theta)
    Z, (H1, H2) = forward(theta, X)
    Zs = Z - Z.max(axis=1, keepdims=True)
    P = np.exp(Zs)
    P /= P.sum(axis=1, keepdims=True)
    loss = float(-np.mean(np.log(P[np.arange(B), y])))
    dZ = P.copy()
    dZ[np.arange(B), y] -= 1.0
    dZ /= B
    dW3, db3 = H2.T @ dZ, dZ.sum(axis=0)
    dH2 = (dZ @ W3.T) * (H2 > 0)
    dW2, db2 = H1.T @ dH2, dH2.sum(axis=0)
    dH1 = (dH2 @ W2.T) * (H1 > 0)
    dW1, db1 = X.T @ dH1, dH1.sum(axis=0)
    return loss, pack([(dW1, db1), (dW2, db2), (dW3, db3)])


def adam_step(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, Algorithm 1) at step t >= 1; returns new
    (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mhat = m / (1 - beta1 ** t)
    vhat = v / (1 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def predict(theta, X):
    Z, _ = forward(theta, X)
    return np.argmax(Z, axis=1)

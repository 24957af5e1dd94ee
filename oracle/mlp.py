"""Cost model of the learned direction scheduler, in float64 numpy.

TEST INFRASTRUCTURE ONLY (see the package header): it checks the device
model's forward pass, gradient and Adam steps.

The model is a fully connected network with eight inputs, two hidden layers
of 32 ReLU units and four linear outputs (predicted log-costs of a round run
as a dense pull, a push over direct slots, a push over flattened arc ranges
and a sparse pull).  Parameters come as one flat vector in the order
W1[32][8], b1[32], W2[32][32], b2[32], W3[4][32], b3[4] (each weight matrix
stored row = output unit).  The loss over n samples is the mean squared
error 1/(2n) sum_n sum_k (y_nk - t_nk)^2; gradients follow the chain rule
layer by layer; Adam is the update of Kingma and Ba (ICLR 2015, Algorithm 1)
with beta1 = 0.9, beta2 = 0.999, eps = 1e-8.

Pins (``tests/test_oracle_mlp.py``): a network built by hand to compute a
known function; positive homogeneity when biases vanish; the gradient
against central finite differences; the first Adam step's closed form; loss
descent on a realisable target.
"""
from __future__ import annotations

import numpy as np

IN, HID, OUT = 8, 32, 4
SHAPES = [("W1", (HID, IN)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)), ("W3", (OUT, HID)),
          ("b3", (OUT,))]
PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)   # 1476


def unpack(p):
    """Flat parameter vector -> dict of float64 arrays (views where possible)."""
    p = np.asarray(p, dtype=np.float64)
    if p.shape != (PARAMS,):
        raise ValueError(f"expected {PARAMS} parameters")
    out, k = {}, 0
    for name, shape in SHAPES:
        size = int(np.prod(shape))
        out[name] = p[k:k + size].reshape(shape)
        k += size
    return out


def pack(parts) -> np.ndarray:
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def forward(p, x, keep=False):
    """Outputs y [n][4] for inputs x [n][8]; with keep, also the hidden activations."""
    w = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    a1 = x @ w["W1"].T + w["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ w["W2"].T + w["b2"]
    h2 = np.maximum(a2, 0.0)
    y = h2 @ w["W3"].T + w["b3"]
    if keep:
        return y, (x, a1, h1, a2, h2)
    return y


def loss(p, x, t) -> float:
    y = forward(p, x)
    t = np.asarray(t, dtype=np.float64)
    return float(0.5 * np.sum((y - t) ** 2) / y.shape[0])


def loss_grad(p, x, t):
    """(loss, gradient) by back-propagation through the three layers."""
    y, (x, a1, h1, a2, h2) = forward(p, x, keep=True)
    w = unpack(p)
    t = np.asarray(t, dtype=np.float64)
    n = y.shape[0]
    e = y - t
    L = float(0.5 * np.sum(e ** 2) / n)
    dy = e / n                                  # dL/dy
    g = {"W3": dy.T @ h2, "b3": dy.sum(axis=0)}
    d2 = (dy @ w["W3"]) * (a2 > 0)              # dL/da2
    g["W2"] = d2.T @ h1
    g["b2"] = d2.sum(axis=0)
    d1 = (d2 @ w["W2"]) * (a1 > 0)              # dL/da1
    g["W1"] = d1.T @ x
    g["b1"] = d1.sum(axis=0)
    return L, pack(g)


def adam(p, x, t, steps: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """Full-batch Adam from zero moments; returns (params, loss before each step)."""
    p = np.array(p, dtype=np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    losses = []
    for k in range(1, steps + 1):
        L, g = loss_grad(p, x, t)
        losses.append(L)
        m = beta1 * m + (1 - beta1) * g
        v = beta2 * v + (1 - beta2) * g * g
        mhat = m / (1 - beta1 ** k)
        vhat = v / (1 - beta2 ** k)
        p = p - lr * mhat / (np.sqrt(vhat) + eps)
    return p, np.array(losses)


def decide(p, f, allowed=(0, 1, 2)) -> int:
    """The action the model picks for features f: the allowed output with the
    least value, the first of equal ones."""
    y = forward(p, np.asarray(f, dtype=np.float64).reshape(1, IN))[0]
    return min(allowed, key=lambda a: (y[a], a))

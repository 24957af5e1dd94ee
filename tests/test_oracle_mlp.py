"""Pins of the cost-model oracle (oracle/mlp.py) against facts that do not
come from its own formulas: a hand-built network, homogeneity, finite
differences, the closed form of Adam's first step, and descent."""
import numpy as np
import pytest

from oracle import mlp


def hand_built():
    """y0 = 3 |x0 - x1| - 1, y1 = 2 max(x2, 0) + 1.5, y2 = 4 - x3 if x3 >= 0, y3 = -2."""
    w = {name: np.zeros(shape) for name, shape in mlp.SHAPES}
    w["W1"][0, 0], w["W1"][0, 1] = 1.0, -1.0      # relu(x0 - x1)
    w["W1"][1, 0], w["W1"][1, 1] = -1.0, 1.0      # relu(x1 - x0)
    w["W1"][2, 2] = 1.0                           # relu(x2)
    w["W2"][0, 0], w["W2"][0, 1] = 1.0, 1.0       # |x0 - x1|
    w["W2"][1, 2], w["b2"][1] = 2.0, 1.0          # 2 relu(x2) + 1
    w["W3"][0, 0], w["b3"][0] = 3.0, -1.0
    w["W3"][1, 1], w["b3"][1] = 1.0, 0.5
    w["W1"][3, 3] = 1.0                           # relu(x3)
    w["W2"][2, 3] = 1.0
    w["W3"][2, 2], w["b3"][2] = -1.0, 4.0
    w["b3"][3] = -2.0
    return mlp.pack(w)


def test_parameter_count():
    assert mlp.PARAMS == 8 * 32 + 32 + 32 * 32 + 32 + 4 * 32 + 4 == 1476


def test_hand_built_network():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(50, 8))
    y = mlp.forward(hand_built(), x)
    np.testing.assert_allclose(y[:, 0], 3 * np.abs(x[:, 0] - x[:, 1]) - 1, rtol=0, atol=1e-12)
    np.testing.assert_allclose(y[:, 1], 2 * np.maximum(x[:, 2], 0) + 1.5, rtol=0, atol=1e-12)
    np.testing.assert_allclose(y[:, 2], 4 - np.maximum(x[:, 3], 0), rtol=0, atol=1e-12)
    np.testing.assert_allclose(y[:, 3], -2.0, rtol=0, atol=1e-12)
    # the decision follows the smallest allowed output
    for row, (a, b, c, d) in zip(x, y):
        assert mlp.decide(hand_built(), row, (0, 1)) == (0 if a <= b else 1)
        assert mlp.decide(hand_built(), row, (0, 1, 2, 3)) == 3                 # y3 = -2 is below the rest here
        want = min((a, 0), (b, 1), (c, 2))[1]
        assert mlp.decide(hand_built(), row) == want


def test_positive_homogeneity_without_biases():
    rng = np.random.default_rng(1)
    w = mlp.unpack(rng.normal(size=mlp.PARAMS))
    p = mlp.pack({**w, "b1": np.zeros(32), "b2": np.zeros(32), "b3": np.zeros(mlp.OUT)})
    x = rng.normal(size=(20, 8))
    np.testing.assert_allclose(mlp.forward(p, 2.5 * x), 2.5 * mlp.forward(p, x), rtol=1e-12, atol=1e-12)
    # and a bias moves the output
    q = p.copy()
    q[-1] = 1.0
    assert not np.allclose(mlp.forward(q, x)[:, -1], mlp.forward(p, x)[:, -1])


def random_problem(seed, n=16):
    rng = np.random.default_rng(seed)
    p = rng.normal(scale=0.4, size=mlp.PARAMS)
    x = rng.uniform(0, 1, size=(n, 8))
    t = rng.normal(size=(n, mlp.OUT))
    return p, x, t


@pytest.mark.parametrize("seed", [2, 3])
def test_gradient_against_finite_differences(seed):
    p, x, t = random_problem(seed)
    L, g = mlp.loss_grad(p, x, t)
    assert L == pytest.approx(mlp.loss(p, x, t), rel=1e-14)
    h = 1e-6
    fd = np.empty(mlp.PARAMS)
    for i in range(mlp.PARAMS):
        a = p.copy()
        b = p.copy()
        a[i] += h
        b[i] -= h
        fd[i] = (mlp.loss(a, x, t) - mlp.loss(b, x, t)) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-5, atol=1e-8)
    # every layer takes part (no block of zeros from a dropped term)
    k = 0
    for name, shape in mlp.SHAPES:
        size = int(np.prod(shape))
        assert np.abs(g[k:k + size]).max() > 0, name
        k += size


def test_first_adam_step_closed_form():
    p, x, t = random_problem(4)
    _, g = mlp.loss_grad(p, x, t)
    lr = 0.01
    p1, losses = mlp.adam(p, x, t, steps=1, lr=lr)
    # after one step m_hat = g and v_hat = g^2
    np.testing.assert_allclose(p1, p - lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert losses[0] == pytest.approx(mlp.loss(p, x, t), rel=1e-14)


def test_adam_fits_a_teacher():
    rng = np.random.default_rng(5)
    teacher = rng.normal(scale=0.5, size=mlp.PARAMS)
    x = rng.uniform(0, 1, size=(256, 8))
    t = mlp.forward(teacher, x)
    student = rng.normal(scale=0.3, size=mlp.PARAMS)
    _, losses = mlp.adam(student, x, t, steps=300, lr=0.01)
    assert losses[-1] < 0.05 * losses[0]

"""Pins of the learned initialiser's FP64 oracle (oracle/mlp.py)."""
import numpy as np
import pytest
import torch

from oracle import mlp


def test_gelu_identities():
    x = np.linspace(-8, 8, 1601)
    g = mlp.gelu(x)
    np.testing.assert_allclose(g - mlp.gelu(-x), x, atol=1e-15)  # Phi(x) + Phi(-x) = 1
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    assert abs(mlp.gelu(np.array([40.0]))[0] - 40.0) < 1e-12
    assert abs(mlp.gelu(np.array([-40.0]))[0]) < 1e-12
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    np.testing.assert_allclose(mlp.gelu_grad(x), fd, atol=1e-9)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=10000) * 10.0 ** rng.uniform(-6, 6, 10000),
                        # exact ties between two bfloat16 values
                        (np.arange(1, 200) * 2 + 1) * 2.0 ** -8 + 1.0])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.to_bf16(x), ref)


def _small(rng, din=5, dh=7, dout=3):
    sizes = [din, dh, dh, dh, dout]
    P = {}
    for l in range(1, 5):
        P["W%d" % l] = rng.normal(size=(sizes[l - 1], sizes[l])) / np.sqrt(sizes[l - 1])
        P["b%d" % l] = rng.normal(size=sizes[l]) * 0.1
    return P


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    P = _small(rng)
    x = rng.normal(size=(9, 5))
    t = rng.normal(size=(9, 3))
    y, cache = mlp.forward(P, x)
    G = mlp.backward(P, cache, t)
    h = 1e-6
    for k, A in P.items():
        it = np.nditer(A, flags=["multi_index"])
        for _ in it:
            idx = it.multi_index
            Ap = A.copy()
            Am = A.copy()
            Ap[idx] += h
            Am[idx] -= h
            fp = mlp.mse(mlp.forward({**P, k: Ap}, x)[0], t)
            fm = mlp.mse(mlp.forward({**P, k: Am}, x)[0], t)
            assert G[k][idx] == pytest.approx((fp - fm) / (2 * h), rel=1e-6, abs=1e-10), (k, idx)


def test_adam_first_step_is_signed_learning_rate():
    """After one step from m = v = 0 the bias-corrected update is
    -lr * g / (|g| + eps)."""
    rng = np.random.default_rng(2)
    P = {"W": rng.normal(size=(4, 3))}
    g = {"W": rng.normal(size=(4, 3))}
    m = {"W": np.zeros((4, 3))}
    v = {"W": np.zeros((4, 3))}
    out = mlp.adam_step(P, g, m, v, 1, lr=1e-3)
    np.testing.assert_allclose(out["W"] - P["W"], -1e-3 * g["W"] / (np.abs(g["W"]) + 1e-8),
                               rtol=1e-12)


def test_encode_decode_round_trip():
    import workloads as wl
    P = wl.draw_params(500, 3)
    P[0, 0] = 0.0
    mean = P[:, 3:].mean(axis=0)
    std = P[:, 3:].std(axis=0)
    Q = mlp.decode_outputs(mlp.encode_targets(P, mean, std), mean, std)
    np.testing.assert_allclose(Q[:, 0], P[:, 0], rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(Q[1:, 1], P[1:, 1], atol=1e-9)
    dpsi = np.abs(Q[1:, 2] - P[1:, 2])
    assert np.all(np.minimum(dpsi, 180 - dpsi) < 1e-8)
    np.testing.assert_allclose(Q[:, 3:], P[:, 3:], rtol=1e-12, atol=1e-12)


def _adam_run(g_seq, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    P = {"W": np.zeros(3)}
    m = {"W": np.zeros(3)}
    v = {"W": np.zeros(3)}
    out = []
    for t, g in enumerate(g_seq, start=1):
        P = mlp.adam_step(P, {"W": g}, m, v, t, lr=lr, beta1=beta1, beta2=beta2, eps=eps)
        out.append(P["W"].copy())
    return np.array(out)


def test_adam_constant_gradient_moves_lr_per_step():
    """A constant gradient g: the bias-corrected moments are g and g^2 at
    every step, so each step moves by lr * g / (|g| + eps)."""
    g = np.array([0.5, -2.0, 1e-3])
    path = _adam_run([g] * 6)
    step = 1e-3 * g / (np.abs(g) + 1e-8)
    expect = -np.outer(np.arange(1, 7), step)
    np.testing.assert_allclose(path, expect, rtol=1e-12, atol=0)


def test_adam_alternating_gradient_follows_the_geometric_moment():
    """g_t = (-1)^(t-1) g: v-hat stays g^2, while
    m_t = (1 - b1) g (-1)^(t-1) (1 - (-b1)^t) / (1 + b1), corrected by
    1 / (1 - b1^t).  Swapped betas or a wrong bias correction change every
    step after the first."""
    b1 = 0.9
    g = np.array([0.5, -2.0, 3.0])
    T = 7
    path = _adam_run([g * (-1.0) ** t for t in range(T)])
    expect = np.zeros((T, 3))
    w = np.zeros(3)
    for t in range(1, T + 1):
        m = (1 - b1) * g * (-1.0) ** (t - 1) * (1 - (-b1) ** t) / (1 + b1)
        mh = m / (1 - b1 ** t)
        w = w - 1e-3 * mh / (np.abs(g) + 1e-8)
        expect[t - 1] = w
    np.testing.assert_allclose(path, expect, rtol=1e-10, atol=1e-18)
    # the second step, written out: m-hat = -(0.01 / 0.19) g
    np.testing.assert_allclose(path[1] - path[0], 1e-3 * (0.01 / 0.19) * g / (np.abs(g) + 1e-8),
                               rtol=1e-10)

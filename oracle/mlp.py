"""FP64 oracle of the learned initialiser's network -- TEST INFRASTRUCTURE.

The paper initialises B, gamma and v_los with small neural networks trained
by back-propagation on synthetic, filtered, noisy profiles, stopping when the
error on a separate control set starts to rise (Sect. 5).  The network here is
a plain multilayer perceptron
    h1 = g(x W1 + b1), h2 = g(h1 W2 + b2), h3 = g(h2 W3 + b3), y = h3 W4 + b4
with g the exact (erf) GELU, trained on mean squared error.  This module is a
direct numpy restatement used to check the GPU kernels: forward, backward
(chain rule written out), and an optional emulation of the points where the
GPU rounds to bfloat16 (round to nearest even from float32).
"""
import math

import numpy as np
from scipy.special import erf

SQRT2 = math.sqrt(2.0)
INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / SQRT2))


def gelu_grad(z):
    """d/dz [z Phi(z)] = Phi(z) + z phi(z)."""
    return 0.5 * (1.0 + erf(z / SQRT2)) + z * INV_SQRT_2PI * np.exp(-0.5 * z * z)


def to_bf16(x):
    """Round to bfloat16 the way the GPU does: first to float32, then to the
    nearest bfloat16, ties to even.  Returned as float64."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)


def forward(params, x, emulate_bf16=False):
    """params: dict W1..W4 ([in, out]) and b1..b4; x: [B, in].
    Returns (y, cache).  With emulate_bf16 the weights, the layer inputs and
    the hidden activations are rounded to bfloat16 where the GPU stores them."""
    r = to_bf16 if emulate_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    a = r(x)
    cache = {"a0": a}
    for l in (1, 2, 3):
        z = a @ r(params["W%d" % l]) + params["b%d" % l]
        a = r(gelu(z))
        cache["z%d" % l] = z
        cache["a%d" % l] = a
    y = a @ r(params["W4"]) + params["b4"]
    cache["y"] = y
    return y, cache


def mse(y, t):
    return float(np.mean((y - t) ** 2))


def backward(params, cache, t, emulate_bf16=False):
    """Gradients of mean((y - t)^2) over all B x n_out entries."""
    r = to_bf16 if emulate_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    y = cache["y"]
    B, n_out = y.shape
    dz = r(2.0 * (y - t) / (B * n_out))
    grads = {}
    grads["W4"] = cache["a3"].T @ dz
    grads["b4"] = dz.sum(axis=0)
    da = dz @ r(params["W4"]).T
    for l in (3, 2, 1):
        dz = r(da * gelu_grad(cache["z%d" % l]))
        grads["W%d" % l] = cache["a%d" % (l - 1)].T @ dz
        grads["b%d" % l] = dz.sum(axis=0)
        if l > 1:
            da = dz @ r(params["W%d" % l]).T
    return grads


def adam_step(params, grads, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) of every array in params."""
    out = {}
    for k in params:
        m[k] = beta1 * m[k] + (1 - beta1) * grads[k]
        v[k] = beta2 * v[k] + (1 - beta2) * grads[k] ** 2
        mh = m[k] / (1 - beta1 ** t)
        vh = v[k] / (1 - beta2 ** t)
        out[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
    return out


# ---- encoding of the model parameters as network outputs -----------------

def encode_targets(P, mean, std):
    """Ten standardised codes: the field vector (B cos g, B sin g cos 2psi,
    B sin g sin 2psi) / 3000, then v, Doppler width, a, eta0, S0, S1, alpha
    standardised with (mean, std)."""
    P = np.asarray(P, dtype=np.float64)
    g = np.radians(P[:, 1])
    p2 = 2.0 * np.radians(P[:, 2])
    T = np.empty((P.shape[0], 10))
    T[:, 0] = P[:, 0] * np.cos(g) / 3000.0
    T[:, 1] = P[:, 0] * np.sin(g) * np.cos(p2) / 3000.0
    T[:, 2] = P[:, 0] * np.sin(g) * np.sin(p2) / 3000.0
    T[:, 3:] = (P[:, 3:] - mean) / std
    return T


def decode_outputs(Y, mean, std):
    """Inverse of encode_targets (angles in degrees, psi in [0, 180))."""
    Y = np.asarray(Y, dtype=np.float64)
    P = np.empty((Y.shape[0], 10))
    bt = np.hypot(Y[:, 1], Y[:, 2])
    P[:, 0] = 3000.0 * np.sqrt(Y[:, 0] ** 2 + bt ** 2)
    P[:, 1] = np.degrees(np.arctan2(bt, Y[:, 0]))
    P[:, 2] = np.mod(0.5 * np.degrees(np.arctan2(Y[:, 2], Y[:, 1])), 180.0)
    P[:, 3:] = Y[:, 3:] * std + mean
    return P

"""The learned-mu network (ORACLE, test infrastructure): a multilayer perceptron
72 -> 256 -> 256 -> 256 -> 1 with exact GELU, 0.5 x (1 + erf(x / sqrt 2)), trained on the
mean squared error of log10 mu.  Forward and backward in float64, written out layer by
layer; with `bf16=True` the values the GPU rounds to bfloat16 (inputs, weights, hidden
activations, backpropagated pre-activation gradients) are rounded at the same points.
Adam (Kingma and Ba, 2015) in float64, written out step by step.
Pinned by central finite differences in pure float64, and Adam by its closed form under a
constant gradient (tests/test_oracle_learned.py).
"""

import numpy as np
from scipy.special import erf

DIMS = (72, 256, 256, 256, 1)


def bf16(x):
    """Round float32 values to bfloat16 (round to nearest even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / np.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / np.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / np.sqrt(2.0 * np.pi)


def forward(params, X, bf=False):
    """params: [W1, b1, W2, b2, W3, b3, W4, b4] with W_l of shape (in, out).
    Returns the prediction (B,) and the cache for backward."""
    r = bf16 if bf else (lambda v: np.asarray(v, dtype=np.float64))
    W = [r(params[2 * l]) for l in range(4)]
    b = [np.asarray(params[2 * l + 1], dtype=np.float64) for l in range(4)]
    H = r(X)
    cache = {"H0": H, "W": W, "Z": [], "H": [H]}
    for l in range(3):
        Z = H @ W[l] + b[l]
        A = gelu(Z)
        H = r(A)
        cache["Z"].append(Z)
        cache["H"].append(H)
    y = (H @ W[3] + b[3])[:, 0]
    return y, cache


def backward(cache, y, t, bf=False):
    """Gradients of mean((y - t)^2) in the order of params."""
    r = bf16 if bf else (lambda v: np.asarray(v, dtype=np.float64))
    B = y.size
    dy = 2.0 * (y - t) / B
    W, Z, H = cache["W"], cache["Z"], cache["H"]
    grads = [None] * 8
    grads[6] = (H[3] * dy[:, None]).sum(axis=0)[:, None]
    grads[7] = np.array([dy.sum()])
    dH = dy[:, None] * W[3][:, 0][None, :]
    for l in (2, 1, 0):
        dZ = dH * gelu_grad(Z[l])
        dZr = r(dZ)
        grads[2 * l] = H[l].T @ dZr
        grads[2 * l + 1] = dZ.sum(axis=0)
        if l > 0:
            dH = dZr @ W[l].T
    return grads


def init_params(rng):
    """He-style normal initialisation, zero biases (float32 masters)."""
    ps = []
    for l in range(4):
        fan_in, fan_out = DIMS[l], DIMS[l + 1]
        ps.append((rng.standard_normal((fan_in, fan_out)) * np.sqrt(2.0 / fan_in)).astype(np.float32))
        ps.append(np.zeros(fan_out, dtype=np.float32))
    return ps


def adam_step(params, grads, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (step = 1, 2, ... counts this one): moments m <- beta1 m + (1-beta1) g,
    v <- beta2 v + (1-beta2) g^2, bias corrections 1 - beta^step, update
    lr m_hat / (sqrt(v_hat) + eps).  Returns new (params, m, v) lists, float64."""
    out_p, out_m, out_v = [], [], []
    c1 = 1.0 - beta1 ** step
    c2 = 1.0 - beta2 ** step
    for p, g, mi, vi in zip(params, grads, m, v):
        g = np.asarray(g, dtype=np.float64).reshape(np.shape(p))
        mi = beta1 * np.asarray(mi, dtype=np.float64) + (1.0 - beta1) * g
        vi = beta2 * np.asarray(vi, dtype=np.float64) + (1.0 - beta2) * g * g
        out_p.append(np.asarray(p, dtype=np.float64) - lr * (mi / c1) / (np.sqrt(vi / c2) + eps))
        out_m.append(mi)
        out_v.append(vi)
    return out_p, out_m, out_v

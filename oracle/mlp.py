"""FP64 CPU oracle of the ray-surrogate network (test infrastructure only).

The network maps a ray's entry features to the change of its exit position and direction:
    y = W5 g(W4 g(W3 g(W2 g(W1 x + b1) + b2) + b3) + b4) + b5,   g = GELU (tanh form),
6 -> 256 -> 256 -> 256 -> 256 -> 6, loss = mean squared error over the batch and the 6 outputs,
trained with Adam (Kingma & Ba, ICLR 2015).  GELU in the tanh form of Hendrycks & Gimpel (2016):
g(z) = z/2 (1 + tanh(sqrt(2/pi) (z + 0.044715 z^3))).

``bf16=True`` mirrors where the GPU kernels round to bfloat16 (round to nearest even): the
weights of layers 2-5 and the activations and back-propagated errors that feed their matrix
products; layer 1, pre-activations, biases and all accumulations stay wide.  Everything else is
plain FP64 numpy.
"""
from __future__ import annotations

import math

import numpy as np

SIZES = (6, 256, 256, 256, 256, 6)
C_GELU = math.sqrt(2.0 / math.pi)
A_GELU = 0.044715


def bf16(x):
    """Round to bfloat16 (nearest even) through float32; returns float64."""
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(z):
    return 0.5 * z * (1.0 + np.tanh(C_GELU * (z + A_GELU * z ** 3)))


def gelu_grad(z):
    t = np.tanh(C_GELU * (z + A_GELU * z ** 3))
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * C_GELU * (1.0 + 3.0 * A_GELU * z * z)


def init_params(seed=0):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases (fixed seed)."""
    rng = np.random.default_rng(seed)
    p = {}
    for l in range(5):
        fi, fo = SIZES[l], SIZES[l + 1]
        s = 1.0 / math.sqrt(fi)
        p[f"W{l + 1}"] = rng.uniform(-s, s, size=(fo, fi))
        p[f"b{l + 1}"] = rng.uniform(-s, s, size=fo)
    return p


PARAM_ORDER = ["W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4", "W5", "b5"]


def flatten(p):
    return np.concatenate([np.asarray(p[k], dtype=np.float64).ravel() for k in PARAM_ORDER])


def unflatten(v):
    p, o = {}, 0
    for l in range(5):
        fi, fo = SIZES[l], SIZES[l + 1]
        p[f"W{l + 1}"] = np.asarray(v[o:o + fo * fi], dtype=np.float64).reshape(fo, fi); o += fo * fi
        p[f"b{l + 1}"] = np.asarray(v[o:o + fo], dtype=np.float64); o += fo
    assert o == len(v)
    return p


def forward(p, x, bf=False):
    """Returns (y, cache).  x: [B, 6]."""
    r = bf16 if bf else (lambda a: a)
    cache = {"a0": np.asarray(x, dtype=np.float64)}
    z = cache["a0"] @ p["W1"].T + p["b1"]
    cache["z1"] = z
    a = r(gelu(z))
    cache["a1"] = a
    for l in (2, 3, 4):
        z = a @ r(p[f"W{l}"]).T + p[f"b{l}"]
        cache[f"z{l}"] = z
        a = r(gelu(z))
        cache[f"a{l}"] = a
    y = a @ r(p["W5"]).T + p["b5"]
    return y, cache


def loss_and_grad_y(y, t):
    d = y - t
    return float((d * d).mean()), 2.0 * d / d.size


def backward(p, cache, dy, bf=False):
    """Gradients of the loss w.r.t. every parameter, given dL/dy."""
    r = bf16 if bf else (lambda a: a)
    g = {}
    g["W5"] = dy.T @ cache["a4"]
    g["b5"] = dy.sum(0)
    da = dy @ p["W5"]          # [B, 256]: K = 6, computed wide
    for l in (4, 3, 2):
        dz = da * gelu_grad(cache[f"z{l}"])
        dzr = r(dz)
        g[f"W{l}"] = dzr.T @ cache[f"a{l - 1}"]
        g[f"b{l}"] = dz.sum(0)
        da = dzr @ r(p[f"W{l}"])
    dz = da * gelu_grad(cache["z1"])
    g["W1"] = dz.T @ cache["a0"]
    g["b1"] = dz.sum(0)
    return g


def adam_step(v, g, m, s, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step on flat arrays (t = step number, 1-based).  Returns updated (v, m, s)."""
    m = beta1 * m + (1.0 - beta1) * g
    s = beta2 * s + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    sh = s / (1.0 - beta2 ** t)
    return v - lr * mh / (np.sqrt(sh) + eps), m, s

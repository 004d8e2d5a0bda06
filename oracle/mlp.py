"""FP64 reference of the surrogate network (test infrastructure only).

The surrogate of the subcellular update is a plain multilayer perceptron:
    z_l = W_l a_{l-1} + b_l,   a_l = f(z_l) for hidden layers,
    output = z_L (linear),
with f = SiLU, SiLU(z) = z / (1 + exp(-z)), or f = ReLU, ReLU(z) = max(z, 0)
(derivative taken as 0 at z = 0),
trained on the mean squared error
    loss = 1 / (2 B n_out) * sum_b sum_k (output_bk - target_bk)^2
with Adam (Kingma & Ba 2015):
    m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
    theta -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

This module is the oracle for the GPU network kernels: plain NumPy in
float64, backpropagation written out layer by layer.  With bf16=True every
operand of a matrix product (inputs, activations, weights, output errors) is
first rounded to bfloat16, as the matrix cores take them, while the
products and sums stay in float64: the ReLU derivative, a 0/1 decision on
the sign of a pre-activation, is then taken from the same operands as on
the device.  Only the test suite
and the benchmark's baseline leg may import it; it imports nothing from the
GPU library.

Parameters are a list of (W, b) with W of shape (out, in).
"""
from __future__ import annotations

import numpy as np


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def round_bf16(a):
    """Nearest bfloat16 value (ties to even) of float32(a), as float64: the
    float32 bit pattern rounded to its upper 16 bits (finite values)."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _mm(a, b, bf16):
    return round_bf16(a) @ round_bf16(b) if bf16 else a @ b


def relu(z):
    return np.maximum(z, 0.0)


def relu_grad(z):
    return (np.asarray(z) > 0.0).astype(np.float64)


ACTS = {"silu": (silu, silu_grad), "relu": (relu, relu_grad)}


def init_params(sizes, seed: int):
    """He-style uniform initialisation, seeded (the GPU side receives these
    arrays as inputs; it does not draw its own)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    params = []
    for i in range(len(sizes) - 1):
        fan_in = sizes[i]
        bound = np.sqrt(6.0 / fan_in) * 0.5
        W = rng.uniform(-bound, bound, (sizes[i + 1], sizes[i]))
        b = np.zeros(sizes[i + 1])
        params.append((W, b))
    return params


def forward(params, X, act: str = "silu", bf16: bool = False):
    """X: (B, in) -> (outputs (B, out), cache of pre-activations)."""
    f = ACTS[act][0]
    a = np.asarray(X, dtype=np.float64)
    zs, acts = [], [a]
    for i, (W, b) in enumerate(params):
        z = _mm(a, W.T, bf16) + b
        zs.append(z)
        a = f(z) if i < len(params) - 1 else z
        acts.append(a)
    return a, (zs, acts)


def loss(params, X, T, act: str = "silu"):
    O, _ = forward(params, X, act)
    B, n = O.shape
    return 0.5 * np.sum((O - T) ** 2) / (B * n)


def backward(params, X, T, act: str = "silu", bf16: bool = False):
    """Gradients of `loss` with respect to every W and b."""
    fg = ACTS[act][1]
    O, (zs, acts) = forward(params, X, act, bf16)
    B, n = O.shape
    dz = (O - T) / (B * n)
    grads = [None] * len(params)
    for i in range(len(params) - 1, -1, -1):
        W, _ = params[i]
        gW = _mm(dz.T, acts[i], bf16)
        gb = dz.sum(axis=0)
        grads[i] = (gW, gb)
        if i > 0:
            da = _mm(dz, W, bf16)
            dz = da * fg(zs[i - 1])
    return grads


def adam_step(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update; `state` is a dict holding t, m, v (created if empty)."""
    if not state:
        state["t"] = 0
        state["m"] = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
        state["v"] = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
    state["t"] += 1
    t = state["t"]
    out = []
    for i, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
        new = []
        for j, (p, g) in enumerate(((W, gW), (b, gb))):
            m = b1 * state["m"][i][j] + (1 - b1) * g
            v = b2 * state["v"][i][j] + (1 - b2) * g * g
            state["m"][i] = tuple(m if k == j else state["m"][i][k] for k in range(2))
            state["v"][i] = tuple(v if k == j else state["v"][i][k] for k in range(2))
            mh = m / (1 - b1 ** t)
            vh = v / (1 - b2 ** t)
            new.append(p - lr * mh / (np.sqrt(vh) + eps))
        out.append((new[0], new[1]))
    return out


def flatten(params):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params])


def unflatten(vec, sizes):
    params, o = [], 0
    for i in range(len(sizes) - 1):
        n_in, n_out = sizes[i], sizes[i + 1]
        W = vec[o:o + n_in * n_out].reshape(n_out, n_in)
        o += n_in * n_out
        b = vec[o:o + n_out]
        o += n_out
        params.append((W.copy(), b.copy()))
    return params


def n_params(sizes):
    return sum(sizes[i] * sizes[i + 1] + sizes[i + 1] for i in range(len(sizes) - 1))

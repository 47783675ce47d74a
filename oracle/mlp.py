"""Oracle of the learned warm start's network (test infrastructure only).

A plain FP64 statement of what the GPU network computes, for checking it:
a multilayer perceptron with SiLU hidden activations, z -> z sigmoid(z)
(Elfwing, Uchibe & Doya 2018), the mean-squared-error loss over a minibatch,
its gradient by backpropagation written out layer by layer, and one Adam step
(Kingma & Ba 2015: exponential moving averages of the gradient and its square
with bias correction).  The network is not part of the paper's method; it
feeds the paper's Broyden iteration (Alg. 2) a first iterate.

Parameters are a list of (W [out, in], b [out]) per layer.  Nothing here is
shared with the GPU library; the tests compare the two on the same inputs.
"""
from __future__ import annotations

import numpy as np


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    """d/dz [z sigmoid(z)] = sigmoid(z) (1 + z (1 - sigmoid(z)))."""
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params, X):
    """Returns the output and, per layer, its input and pre-activation."""
    h = np.asarray(X, dtype=np.float64)
    inputs, pre = [], []
    for l, (W, b) in enumerate(params):
        inputs.append(h)
        z = h @ W.T + b
        pre.append(z)
        h = silu(z) if l + 1 < len(params) else z
    return h, inputs, pre


def loss(params, X, T, n_out=None):
    """Mean of (Y - T)^2 over the rows and the first n_out columns."""
    Y, _, _ = forward(params, X)
    n = Y.shape[1] if n_out is None else n_out
    d = Y[:, :n] - np.asarray(T, dtype=np.float64)[:, :n]
    return float(np.mean(d * d))


def gradients(params, X, T, n_out=None):
    """(loss, [(dL/dW, dL/db)]) by the chain rule, from the output layer back."""
    Y, inputs, pre = forward(params, X)
    B = Y.shape[0]
    n = Y.shape[1] if n_out is None else n_out
    T = np.asarray(T, dtype=np.float64)
    d = np.zeros_like(Y)
    d[:, :n] = 2.0 * (Y[:, :n] - T[:, :n]) / (B * n)
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        dz = d if l + 1 == len(params) else d * dsilu(pre[l])
        grads[l] = (dz.T @ inputs[l], dz.sum(axis=0))
        d = dz @ params[l][0]
    return loss(params, X, T, n_out), grads


def adam_step(params, grads, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update of every array in place; t is the 1-based step count."""
    out = []
    for (W, b), (gW, gb), (mW, mb), (vW, vb) in zip(params, grads, m, v):
        new = []
        for p, g, mm, vv in ((W, gW, mW, vW), (b, gb, mb, vb)):
            mm *= beta1
            mm += (1.0 - beta1) * g
            vv *= beta2
            vv += (1.0 - beta2) * g * g
            mhat = mm / (1.0 - beta1 ** t)
            vhat = vv / (1.0 - beta2 ** t)
            new.append(p - lr * mhat / (np.sqrt(vhat) + eps))
        out.append(tuple(new))
    return out


def zeros_like(params):
    return [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]


def unflatten(flat, dims):
    """Flat vector -> [(W, b)]: per layer W [out, in] row-major, then b [out].
    dims = [(in_0, out_0), (in_1, out_1), ...]."""
    flat = np.asarray(flat, dtype=np.float64)
    params, o = [], 0
    for din, dout in dims:
        W = flat[o:o + din * dout].reshape(dout, din)
        o += din * dout
        b = flat[o:o + dout]
        o += dout
        params.append((W.copy(), b.copy()))
    assert o == flat.size
    return params


def flatten(params):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params])


def bf16_round(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    a = np.asarray(x, dtype=np.float32).copy()
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)

"""CPU oracle for the learned initial guess of the reduced system.

TEST INFRASTRUCTURE ONLY: imported by the tests and the benchmark's CPU
baseline, never by the GPU path, and sharing no code with it.

The network is the per-interface multilayer perceptron used to predict the
initial guess z^_0 of the reduced system G^ z^ = g^ (stage 6.3 of the paper's
preconditioner).  The paper itself solves 6.3 iteratively from a guess and
says nothing about where the guess comes from; the network is this project's
addition beside the method (its residual decides whether its guess is used).

  h1 = relu(x  W1 + b1)        W1: d_in x H
  h2 = relu(h1 W2 + b2)        W2: H x H
  h3 = relu(h2 W3 + b3)        W3: H x H
  y  =      h3 W4 + b4         W4: H x d_out
  loss = mean((y - target)^2)  over all batch x d_out entries

Backward pass: the chain rule written out layer by layer; Adam: Kingma & Ba
(2015), Algorithm 1, with bias correction.  All arithmetic is float64; the
`bf16` switch rounds the tensors the GPU keeps in bfloat16 (weights used in
the products, the input and the stored activations) to bfloat16 with
round-to-nearest-even at the same points, so the two sides differ only by
accumulation order.
"""
from __future__ import annotations

import numpy as np


def round_bf16(a):
    """Round float64/float32 values to the nearest bfloat16 (ties to even),
    returned as float64.  bfloat16 keeps the top 16 bits of a float32."""
    f = np.asarray(a, dtype=np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    bits = (bits + 0x7FFF + lsb) & 0xFFFF0000
    out = bits.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if np.any(nan):
        out[nan] = np.nan
    return out


def _r(a, bf16):
    return round_bf16(a) if bf16 else np.asarray(a, dtype=np.float64)


def forward(params, x, bf16=False):
    """Returns the output and the cache needed by backward()."""
    W1, b1, W2, b2, W3, b3, W4, b4 = params
    a0 = _r(x, bf16)
    z1 = a0 @ _r(W1, bf16) + b1
    a1 = _r(np.maximum(z1, 0.0), bf16)
    z2 = a1 @ _r(W2, bf16) + b2
    a2 = _r(np.maximum(z2, 0.0), bf16)
    z3 = a2 @ _r(W3, bf16) + b3
    a3 = _r(np.maximum(z3, 0.0), bf16)
    y = a3 @ _r(W4, bf16) + b4
    return y, (a0, z1, a1, z2, a2, z3, a3)


def mse(y, target):
    d = y - target
    return float(np.mean(d * d))


def backward(params, cache, y, target, bf16=False):
    """Gradients of mse(y, target) with respect to every parameter."""
    W1, b1, W2, b2, W3, b3, W4, b4 = params
    a0, z1, a1, z2, a2, z3, a3 = cache
    dy = 2.0 * (y - target) / y.size
    dW4 = a3.T @ dy
    db4 = dy.sum(axis=0)
    dz3 = (dy @ _r(W4, bf16).T) * (z3 > 0)
    dW3 = a2.T @ dz3
    db3 = dz3.sum(axis=0)
    dz2 = (dz3 @ _r(W3, bf16).T) * (z2 > 0)
    dW2 = a1.T @ dz2
    db2 = dz2.sum(axis=0)
    dz1 = (dz2 @ _r(W2, bf16).T) * (z1 > 0)
    dW1 = a0.T @ dz1
    db1 = dz1.sum(axis=0)
    return [dW1, db1, dW2, db2, dW3, db3, dW4, db4]


def adam_step(params, grads, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1); t is 1-based."""
    new_p, new_m, new_v = [], [], []
    for p, g, mm, vv in zip(params, grads, m, v):
        mm = beta1 * mm + (1.0 - beta1) * g
        vv = beta2 * vv + (1.0 - beta2) * g * g
        mh = mm / (1.0 - beta1 ** t)
        vh = vv / (1.0 - beta2 ** t)
        new_p.append(p - lr * mh / (np.sqrt(vh) + eps))
        new_m.append(mm)
        new_v.append(vv)
    return new_p, new_m, new_v


def init_params(d_in, hidden, d_out, seed):
    """He-uniform initial weights, zero biases (float64)."""
    rng = np.random.default_rng(seed)
    dims = [d_in, hidden, hidden, hidden, d_out]
    out = []
    for a, b in zip(dims[:-1], dims[1:]):
        lim = np.sqrt(6.0 / a)
        out.append(rng.uniform(-lim, lim, (a, b)))
        out.append(np.zeros(b))
    return out

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
(2015), Algorithm 1, with bias correction.  All arithmetic is float64.

The `bf16` switch follows the network's stated precision, "bf16 weights and
activations, FP32 accumulation", read as: every operand of a product is a
bfloat16 value and every sum is an accumulator.  So the weights as used, the
input, the stored activations of the forward pass, and the activations of the
backward pass (the output error dy and the pre-activation errors dz, which
are the operands of the backward products) are rounded to bfloat16 (nearest,
ties to even); sums, biases, the output y and the parameter gradients (FP32
master parameters) are not.  The element-by-element form of this reading is
pinned in the tests.  Two implementations of it differ only by accumulation
order and by where the ReLU test falls for z within rounding of zero.
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
    dy = _r(2.0 * (y - target) / y.size, bf16)
    dW4 = a3.T @ dy
    db4 = dy.sum(axis=0)
    dz3 = _r((dy @ _r(W4, bf16).T) * (z3 > 0), bf16)
    dW3 = a2.T @ dz3
    db3 = dz3.sum(axis=0)
    dz2 = _r((dz3 @ _r(W3, bf16).T) * (z2 > 0), bf16)
    dW2 = a1.T @ dz2
    db2 = dz2.sum(axis=0)
    dz1 = _r((dz2 @ _r(W2, bf16).T) * (z1 > 0), bf16)
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


# --------------------------------------------------------------------------
# Reduced-vector plumbing of the learned guess (project definition).
#
# The reduced system of stage 6.3 has one unknown per column of the index set
# c.  The guess network works interface by interface, so its vectors use the
# candidate layout: interface j (between blocks j and j+1) owns the 2t
# candidate columns [part[j+1] - t, part[j+1] + t) -- the last t columns of
# block j, then the first t of block j+1 -- and a mask marks which of them
# are in c.
# --------------------------------------------------------------------------
def candidate_layout(part_ptr, t, c):
    """Candidate columns (int64[2t(p-1)]) and their mask (1.0 where in c)."""
    part = np.asarray(part_ptr, dtype=np.int64)
    cand = np.concatenate([np.arange(part[j + 1] - t, part[j + 1] + t, dtype=np.int64)
                           for j in range(len(part) - 2)]) if len(part) > 2 else np.zeros(0, np.int64)
    mask = np.isin(cand, np.asarray(c, dtype=np.int64)).astype(np.float64)
    return cand, mask


def to_candidates(v_c, c, cand):
    """A vector on c (compressed, in the order of c) spread onto the
    candidate layout, zero off c."""
    pos = {int(col): i for i, col in enumerate(c)}
    out = np.zeros(len(cand))
    for q, col in enumerate(cand):
        i = pos.get(int(col))
        if i is not None:
            out[q] = v_c[i]
    return out


def guess_features(r, zprev, mask, t, cos_t, sin_t, d_in):
    """Rows [r_j / s_j, (z^prev_j on c) / q_j, cos, sin, 0...] with
    s_j = max |r_j| and q_j = max |z^prev_j on c| (1 where zero); r is the
    reduced residual g^ - G^ z^prev.  Returns (X float32[(p-1) x d_in],
    s float32[p-1])."""
    w = 2 * t
    nif = len(r) // w
    X = np.zeros((nif, d_in), dtype=np.float32)
    s = np.zeros(nif, dtype=np.float32)

    def absmax(v):
        a = np.max(np.abs(v))
        return a if a > 1e-300 else 1.0

    for j in range(nif):
        rj = r[j * w:(j + 1) * w]
        z = zprev[j * w:(j + 1) * w] * mask[j * w:(j + 1) * w]
        sj, qj = absmax(rj), absmax(z)
        X[j, :w] = (rj / sj).astype(np.float32)
        X[j, w:2 * w] = (z / qj).astype(np.float32)
        X[j, 2 * w] = np.float32(cos_t)
        X[j, 2 * w + 1] = np.float32(sin_t)
        s[j] = np.float32(sj)
    return X, s


def guess_compose(zprev, Y, s, mask, t):
    """Initial guess z^0 = (z^prev + s_j Y_j) on c, 0 off c."""
    w = 2 * t
    out = np.zeros(len(zprev))
    for j in range(len(s)):
        sl = slice(j * w, (j + 1) * w)
        out[sl] = (zprev[sl] + np.float64(s[j]) * Y[j].astype(np.float64)) * mask[sl]
    return out


def guess_target(zhat, zprev, s, mask, t):
    """Training target (z^_j - z^prev_j on c) / s_j, float32[(p-1) x 2t]."""
    w = 2 * t
    T = np.zeros((len(s), w), dtype=np.float32)
    for j in range(len(s)):
        sl = slice(j * w, (j + 1) * w)
        T[j] = ((zhat[sl] - zprev[sl] * mask[sl]) / np.float64(s[j])).astype(np.float32)
    return T

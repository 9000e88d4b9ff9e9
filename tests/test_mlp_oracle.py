"""Pins for the MLP oracle: brute-force loops, central finite differences,
Adam's closed-form first step and bfloat16 rounding."""
import numpy as np

from oracle import mlp_oracle as M


def _tiny(seed=0, d_in=5, h=4, d_out=3):
    p = M.init_params(d_in, h, d_out, seed)
    rng = np.random.default_rng(seed + 1)
    p = [a + 0.1 * rng.standard_normal(a.shape) for a in p]   # nonzero biases too
    x = rng.standard_normal((6, d_in))
    t = rng.standard_normal((6, d_out))
    return p, x, t


def test_forward_matches_python_loops():
    p, x, _ = _tiny()
    y, _ = M.forward(p, x)
    W = p[0::2]
    b = p[1::2]
    for r in range(x.shape[0]):
        a = list(x[r])
        for layer in range(4):
            out = []
            for j in range(W[layer].shape[1]):
                s = b[layer][j]
                for i in range(len(a)):
                    s += a[i] * W[layer][i, j]
                out.append(max(s, 0.0) if layer < 3 else s)
            a = out
        assert np.allclose(a, y[r], rtol=1e-13, atol=1e-14)


def test_backward_matches_central_differences():
    p, x, t = _tiny(3)
    y, cache = M.forward(p, x)
    g = M.backward(p, cache, y, t)
    h = 1e-6
    for k, P in enumerate(p):
        flat = P.reshape(-1)
        for idx in range(0, flat.size, max(1, flat.size // 7)):
            old = flat[idx]
            flat[idx] = old + h
            lp = M.mse(M.forward(p, x)[0], t)
            flat[idx] = old - h
            lm = M.mse(M.forward(p, x)[0], t)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[k].reshape(-1)[idx]) <= 1e-6 * max(1.0, abs(fd)), (k, idx)


def test_adam_first_step_is_lr_times_sign():
    # After one step from m = v = 0 the bias-corrected ratio is g/|g|.
    rng = np.random.default_rng(5)
    p = [rng.standard_normal((3, 4))]
    g = [rng.standard_normal((3, 4))]
    z = [np.zeros((3, 4))]
    newp, m, v = M.adam_step(p, g, z, z, 1, lr=0.01, eps=0.0)
    assert np.allclose(newp[0], p[0] - 0.01 * np.sign(g[0]), rtol=0, atol=1e-15)
    assert np.allclose(m[0], 0.1 * g[0]) and np.allclose(v[0], 0.001 * g[0] ** 2)


def test_round_bf16_known_values():
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: ties go to the even mantissa (1).
    # 1 + 3*2^-8 is a tie between 1 + 2^-7 and 1 + 2^-6: even is 1 + 2^-6.
    vals = np.array([1.0, 1.0 + 2**-8, 1.0 + 3 * 2**-8, 1.0 + 2**-7, -3.140625, 65504.0, 1e-40])
    got = M.round_bf16(vals)
    exp = np.array([1.0, 1.0, 1.0 + 2**-6, 1.0 + 2**-7, -3.140625, 65536.0, 0.0])
    # 1e-40 is a float32 subnormal: rounding keeps it a (tiny) subnormal
    assert np.array_equal(got[:6], exp[:6])
    assert abs(got[6]) < 1e-39


def test_bf16_switch_is_exact_on_representable_values():
    # Small-integer weights and inputs keep every intermediate an integer
    # below 256 (a bf16 value) and the batch*d_out = 8 divisor a power of two,
    # so the bf16 rounding points must not change anything.
    rng = np.random.default_rng(7)
    p = []
    for a, b in [(3, 4), (4, 4), (4, 4), (4, 2)]:
        p.append(rng.integers(-1, 2, (a, b)).astype(np.float64))
        p.append(rng.integers(-1, 2, b).astype(np.float64))
    x = rng.integers(-2, 3, (4, 3)).astype(np.float64)
    t = rng.integers(-2, 3, (4, 2)).astype(np.float64)
    y0, c0 = M.forward(p, x, bf16=False)
    y1, c1 = M.forward(p, x, bf16=True)
    assert np.array_equal(y0, y1)
    g0 = M.backward(p, c0, y0, t, bf16=False)
    g1 = M.backward(p, c1, y1, t, bf16=True)
    for a, b in zip(g0, g1):
        assert np.array_equal(a, b)


def test_bf16_switch_rounds_the_backward_signal():
    # 1x1 identity layers and x = 1 give a3 = 1, so dW4 = a3^T dy = dy; with
    # y - t = (1 + 2^-10) / 2 and N = 1, dy = 1 + 2^-10, which is not a bf16
    # value and must round to 1.
    p = [np.eye(1), np.zeros(1), np.eye(1), np.zeros(1), np.eye(1), np.zeros(1), np.eye(1), np.zeros(1)]
    x = np.array([[1.0]])
    y, cache = M.forward(p, x, bf16=True)
    tgt = y - (1.0 + 2.0 ** -10) / 2.0
    g = M.backward(p, cache, y, tgt, bf16=True)
    assert g[6][0, 0] == 1.0            # 1 + 2^-10 rounds to 1 in bf16
    g64 = M.backward(p, cache, y, tgt, bf16=False)
    assert g64[6][0, 0] == 1.0 + 2.0 ** -10


def test_candidate_layout_and_spread():
    part = [0, 10, 22, 30]
    cand, mask = M.candidate_layout(part, 3, [8, 9, 10, 20, 23])
    assert list(cand) == [7, 8, 9, 10, 11, 12, 19, 20, 21, 22, 23, 24]
    assert list(mask) == [0, 1, 1, 1, 0, 0, 0, 1, 0, 0, 1, 0]
    v = M.to_candidates(np.array([1.0, 2.0, 3.0, 4.0, 5.0]), [8, 9, 10, 20, 23], cand)
    assert list(v) == [0, 1, 2, 3, 0, 0, 0, 4, 0, 0, 5, 0]


def test_guess_features_compose_target_round_trip():
    # compose(target(z)) returns z on c (up to the float32 rounding of T), the
    # r and z^prev parts of each feature row have max-norm 1, and a zero r
    # gives scale 1.
    rng = np.random.default_rng(11)
    t = 4
    w = 2 * t
    nif = 3
    mask = (rng.uniform(size=nif * w) > 0.3).astype(np.float64)
    gh = rng.standard_normal(nif * w) * mask * 10.0
    gh[w:2 * w] = 0.0
    zp = rng.standard_normal(nif * w)
    zh = rng.standard_normal(nif * w) * mask
    X, s = M.guess_features(gh, zp, mask, t, 0.5, -0.25, 4 * t + 5)
    assert X.shape == (nif, 4 * t + 5) and np.all(X[:, 4 * t + 2:] == 0)
    assert np.isclose(np.max(np.abs(X[0, :w])), 1.0) and s[1] == 1.0
    assert np.all(X[:, 2 * w] == np.float32(0.5)) and np.all(X[:, 2 * w + 1] == np.float32(-0.25))
    zm = zp * mask
    assert np.allclose(X[2, w:2 * w], zm[2 * w:] / np.max(np.abs(zm[2 * w:])), rtol=1e-6)
    assert np.isclose(np.max(np.abs(X[0, w:2 * w])), 1.0)
    T = M.guess_target(zh, zp, s, mask, t)
    z0 = M.guess_compose(zp, T, s, mask, t)
    assert np.allclose(z0, zh, rtol=1e-6, atol=1e-6 * np.max(np.abs(zh)))
    assert np.all(z0[mask == 0] == 0)


def _bf16_scalar(v):
    """Nearest bfloat16 of a float (ties to even), via the float32 bit
    pattern: bfloat16 is the top 16 bits of a float32."""
    import struct
    bits = struct.unpack("<I", struct.pack("<f", float(v)))[0]
    bits = (bits + 0x7FFF + ((bits >> 16) & 1)) & 0xFFFF0000
    return struct.unpack("<f", struct.pack("<I", bits))[0]


def _loop_net(params, x, t):
    """The network's bf16 mode written out element by element.  Rounding
    points, read from 'bf16 weights and activations, FP32 accumulation': the
    operands of every product are bf16 (weights as used, the input, the
    stored activations, and in the backward pass the activation gradients dy
    and dz that the backward products consume); sums, biases, the output y
    and the parameter gradients are not rounded (FP32 accumulators and FP32
    master parameters).  Sums are taken in Python floats so that only the
    rounding points, not the summation order, can differ."""
    W = [params[0], params[2], params[4], params[6]]
    bvec = [params[1], params[3], params[5], params[7]]
    B = len(x)
    act = [[[_bf16_scalar(v) for v in row] for row in x]]
    pre = []
    for l in range(4):
        a = act[-1]
        fi, fo = W[l].shape
        z = [[sum(a[r][i] * _bf16_scalar(W[l][i][j]) for i in range(fi)) + bvec[l][j] for j in range(fo)]
             for r in range(B)]
        pre.append(z)
        if l < 3:
            act.append([[_bf16_scalar(max(v, 0.0)) for v in row] for row in z])
    y = pre[3]
    N = B * len(y[0])
    dz = [[_bf16_scalar(2.0 * (y[r][j] - t[r][j]) / N) for j in range(len(y[0]))] for r in range(B)]
    grads = [None] * 8
    for l in range(3, -1, -1):
        a = act[l]
        fi, fo = W[l].shape
        grads[2 * l] = np.array([[sum(a[r][i] * dz[r][j] for r in range(B)) for j in range(fo)] for i in range(fi)])
        grads[2 * l + 1] = np.array([sum(dz[r][j] for r in range(B)) for j in range(fo)])
        if l > 0:
            zprev = pre[l - 1]
            dz = [[_bf16_scalar(sum(dz[r][j] * _bf16_scalar(W[l][i][j]) for j in range(fo))
                                * (1.0 if zprev[r][i] > 0 else 0.0)) for i in range(fi)] for r in range(B)]
    return np.array(y), grads


def test_bf16_mode_matches_elementwise_definition():
    # Random (non-representable) weights and inputs: every bf16 rounding point
    # of the vectorised oracle must sit where the element-by-element
    # definition puts it; a missing or extra rounding moves results by about
    # 2^-9 relative, far above the 1e-12 allowed here for summation order.
    rng = np.random.default_rng(21)
    dims = [5, 4, 4, 4, 3]
    params = []
    for a, b in zip(dims[:-1], dims[1:]):
        params.append(rng.uniform(-1.3, 1.3, (a, b)))
        params.append(rng.uniform(-0.2, 0.2, b))
    x = rng.uniform(-2, 2, (3, 5))
    t = rng.uniform(-1, 1, (3, 3))
    y_loop, g_loop = _loop_net(params, x, t)
    y, cache = M.forward(params, x, bf16=True)
    g = M.backward(params, cache, y, t, bf16=True)
    assert np.allclose(y, y_loop, rtol=1e-12, atol=1e-12)
    for a, b in zip(g, g_loop):
        assert np.allclose(a, b, rtol=1e-12, atol=1e-12)
    # the rounding is not a no-op on these values
    y64, c64 = M.forward(params, x, bf16=False)
    assert np.max(np.abs(y64 - y)) > 1e-4

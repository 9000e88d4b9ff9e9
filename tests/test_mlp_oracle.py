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

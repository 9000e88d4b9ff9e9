"""Full-size C2 (32 x 32 x 512 3D convection-diffusion, p = 64, band 1024) on
the GPU, in the launch configuration the benchmark times.  The oracle cannot
run the whole system in seconds, so it is checked on samples it computes one
by one (spike columns and a block solve of one block) and through properties
that hold at any size (residual, error against the known x*)."""
import numpy as np
import pytest

from tests.gpu_util import dev_vec, host, make_solver, relerr, torch_cuda
from workloads import configs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c2():
    return configs.c2()


@pytest.fixture(scope="module")
def c2_f64(c2):
    S = make_solver(c2, inner_tol=1e-12)
    S.factor()
    yield S
    S.close()


def test_c2_f64_solve(c2, c2_f64):
    A = c2["A"]
    x = dev_vec(np.zeros(A.n))
    rc, info = c2_f64.solve(dev_vec(c2["f"]), x, 1e-11)
    xs = host(x)
    r = c2["f"] - A.scipy() @ xs
    assert np.linalg.norm(r, np.inf) / np.linalg.norm(c2["f"], np.inf) <= 1e-11
    assert relerr(xs, c2["x_star"]) <= 1e-8
    assert info.outer_iters <= 2


def test_c2_sampled_spikes_and_block_solve(c2, c2_f64):
    from oracle import ddps_oracle as O
    from paper_1008_1700_amd import ddps
    torch = torch_cuda()
    S = c2["A"].scipy()
    blk, t = 5, 1024
    lo, hi = c2["part_ptr"][blk], c2["part_ptr"][blk + 1]
    fac = O.factor_block(S[lo:hi, lo:hi].tocsr(), require_no_pivot=True)
    ni = hi - lo
    buf = torch.empty(ni * 2 * t, dtype=torch.float64, device="cuda")
    ddps.ddps_get_spikes(c2_f64.h, blk, buf)
    G = host(buf).reshape(2 * t, ni).T
    cols = [0, 511, 1023, t + 0, t + 700, t + 1023]          # global: lo - t + j, hi + (j - t)
    gcols = [lo - t + j if j < t else hi + (j - t) for j in cols]
    R = S[lo:hi, :].tocsc()[:, gcols].toarray()
    exp = O.block_solve(fac, R)
    assert relerr(G[:, cols], exp) <= 1e-11
    y = np.random.default_rng(12).standard_normal(c2["A"].n)
    g = torch.empty_like(dev_vec(y))
    ddps.ddps_block_solve(c2_f64.h, 1, dev_vec(y), g)
    assert relerr(host(g)[lo:hi], O.block_solve(fac, y[lo:hi])) <= 1e-12


@pytest.mark.parametrize("dtype", ["bf16x3", "f32"])
def test_c2_mixed_precision_solve(c2, dtype):
    A = c2["A"]
    S = make_solver(c2, dtype=dtype, inner_tol=1e-7)
    try:
        S.factor()
        x = dev_vec(np.zeros(A.n))
        rc, info = S.solve(dev_vec(c2["f"]), x, 1e-11)
        xs = host(x)
        r = c2["f"] - A.scipy() @ xs
        assert np.linalg.norm(r, np.inf) / np.linalg.norm(c2["f"], np.inf) <= 1e-11
        assert relerr(xs, c2["x_star"]) <= 1e-8
    finally:
        S.close()


# bounds on the normwise backward error of the factors: a small multiple of
# the unit roundoff of the products (FP64 2^-53, FP32 and split bf16 2^-24,
# bf16 2^-9) times the growth over the band LU's tile steps
BACKWARD_BOUND = {"f64": 1e-13, "f32": 1e-5, "bf16x3": 1e-5, "bf16": 3e-2}


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16x3", "bf16"])
def test_c2_factor_backward_error(c2, dtype):
    """||A_ii - L~ U~||_F / ||A_ii||_F for block 1 (an interior block: t =
    1024, 8 tiles) from the GPU's factor tiles, per precision.  The FP64
    factors pin the measurement itself at roundoff level."""
    from bench import factor_backward_error
    S = make_solver(c2, dtype=dtype, inner_tol=1e-7)
    try:
        S.factor()
        be = factor_backward_error(S, c2, 1)
        print(f"c2 {dtype}: factor backward error {be}")
        assert be["t"] == 1024 and be["tile_rows"] == 8
        assert be["rel_fro"] <= BACKWARD_BOUND[dtype]
    finally:
        S.close()

"""GPU runs at the full sizes of the uneven-partition and large 3D workloads.

The oracle cannot factor these systems whole, so parity is checked on what
it can compute one by one (one block's band LU and sampled spike columns)
and on properties that hold at any size: the FP64 residual computed on the
host, the error against the manufactured solution, and the block shapes of
the uneven partition.

C3: 2048^2 anisotropic lognormal diffusion, 123 uneven slabs (4..28 grid
    rows each), FP32 factors and spikes, FP64 refinement.
C5: 40x40x4096 diffusion-reaction, 512 slabs, 8 right-hand sides, FP32
    factors and spikes; plain FP64 storage does not fit the device.
"""
import numpy as np
import pytest

from tests.gpu_util import host, relerr, torch_cuda
from workloads import configs

pytestmark = pytest.mark.gpu


def _spike_sample(d, blk, cols):
    """Oracle spikes of block blk for the coupling columns `cols` (indices
    into the block's [left t | right t] coupling window)."""
    from oracle import ddps_oracle as O
    A = d["A"].scipy()
    part = d["part_ptr"]
    t = d["b"]
    lo, hi = int(part[blk]), int(part[blk + 1])
    fac = O.factor_block(A[lo:hi, lo:hi].tocsr())
    gcols = [lo - t + j if j < t else hi + (j - t) for j in cols]
    R = A[lo:hi, :][:, gcols].toarray()
    return O.block_solve(fac, R)


def _check_block(S, d, blk, cols, tol):
    from paper_1008_1700_amd import ddps
    torch = torch_cuda()
    part = d["part_ptr"]
    ni = int(part[blk + 1] - part[blk])
    t = d["b"]
    G = torch.empty(2 * t * ni, dtype=torch.float64, device="cuda")
    ddps.ddps_get_spikes(S.h, blk, G)
    Gh = host(G).reshape(2 * t, ni).T
    ref = _spike_sample(d, blk, cols)
    errs = [relerr(Gh[:, j], ref[:, q]) for q, j in enumerate(cols)]
    print(f"block {blk} (n_i {ni}) sampled spike columns: max rel err {max(errs):.3e}")
    assert max(errs) <= tol


def _host_check(d, X, tol_res, tol_err):
    A = d["A"].scipy()
    F = d["f"]
    r = F - A @ X
    rel = np.max(np.abs(r), axis=0) / np.max(np.abs(F), axis=0)
    xs = d["x_star"]
    err = np.linalg.norm(X - xs, axis=0) / np.linalg.norm(xs, axis=0)
    print(f"host residual max {np.max(rel):.3e}, error vs x* max {np.max(err):.3e}")
    assert np.all(rel <= tol_res)
    assert np.all(err <= tol_err)


@pytest.fixture(scope="module")
def c3():
    return configs.c3()


def test_c3_uneven_fp32_solve_and_graph(c3):
    from paper_1008_1700_amd import ddps
    torch = torch_cuda()
    d = c3
    part = d["part_ptr"]
    p = len(part) - 1
    S = ddps.Solver(d["A"], part, dtype="f32", inner_tol=1e-6, outer="refine")
    try:
        t, tiles, pads = ddps.ddps_block_shape(S.h, p)
        ni = np.diff(part)
        assert t == 2048
        assert tiles == [int(-(-n // t)) for n in ni] and pads == [int(T * t - n) for T, n in zip(tiles, ni)]
        assert min(tiles) == 4 and max(tiles) == 28
        S.factor()
        f = torch.from_numpy(d["f"]).cuda()
        x = torch.zeros(d["A"].n, dtype=torch.float64, device="cuda")
        _, info = S.solve(f, x, 1e-10)
        print(f"c3 f32: {info.as_dict()}")
        x1 = host(x)
        # C3 is badly conditioned (coefficients over ~5 decades, anisotropy
        # 1e-3): at a residual of 1e-10 no solver is closer than ~1e-4 to x*,
        # so the forward error is held to that conditioning-consistent bound
        # and the residual carries the 1e-10 bar
        _host_check(d, x1, 1e-10, 1e-3)
        # the shortest interior block against the oracle's band LU
        blk = 1 + int(np.argmin(ni[1:-1]))
        _check_block(S, d, blk, [0, 1, 1000, 2047, 2048, 2049, 3000, 4095], 1e-3)
        # graph replay of the whole factorisation: same factors, same solution
        ddps.ddps_set_execution(S.h, 4, True, 0)
        S.factor()
        S.factor()                     # second replay of the captured graph
        x2 = torch.zeros_like(x)
        S.solve(f, x2, 1e-10)
        assert np.array_equal(host(x2), x1)
    finally:
        S.close()


@pytest.fixture(scope="module")
def c5():
    return configs.c5()


def test_c5_fp64_does_not_fit(c5):
    from paper_1008_1700_amd import ddps
    d = c5
    with pytest.raises(ddps.DDPSError) as e:
        ddps.Solver(d["A"], d["part_ptr"], dtype="f64", max_rhs=8)
    assert e.value.code == -2       # DDPS_E_NOMEM, checked before any large allocation


def test_c5_fp32_eight_rhs(c5):
    from paper_1008_1700_amd import ddps
    torch = torch_cuda()
    d = c5
    k = d["f"].shape[1]
    S = ddps.Solver(d["A"], d["part_ptr"], dtype="f32", inner_tol=1e-6, outer="refine", max_rhs=k)
    try:
        print(f"c5 memory {ddps.ddps_memory(S.h) / 1e9:.1f} GB")
        S.factor()
        F = torch.from_numpy(np.ascontiguousarray(d["f"].T)).cuda()
        X = torch.zeros(k, d["A"].n, dtype=torch.float64, device="cuda")
        _, info = ddps.ddps_solve_many(S.h, F, X, 1e-10)
        print(f"c5 f32 x{k}: {info.as_dict()}")
        _host_check(d, host(X).T, 1e-10, 1e-8)
        _check_block(S, d, 0, [1600, 1601, 2400, 3199], 1e-4)
        _check_block(S, d, 300, [0, 799, 1599, 1600, 3199], 1e-4)
    finally:
        S.close()

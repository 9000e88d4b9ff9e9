"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.  Tolerances follow from FP64 rounding of well-conditioned
M-matrix blocks (entrywise factors, spikes, block solves: 1e-11 relative;
final solutions: the 1e-8 relative-error bar at residual tolerance <= 1e-10).
"""
import numpy as np
import pytest
import scipy.sparse as sp

from tests.gpu_util import dev_vec, host, make_solver, maxrel, oracle_prec, relerr, torch_cuda
from workloads import configs, pde

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c1():
    return configs.c1()


@pytest.fixture(scope="module")
def c1_solver(c1):
    S = make_solver(c1, inner_tol=1e-14, max_rhs=4)
    S.factor()
    yield S
    S.close()


@pytest.fixture(scope="module")
def c1_oracle(c1):
    return oracle_prec(c1)


def _expected_tiles(fac, t, k):
    from oracle import ddps_oracle as O
    L, U = O.unit_lower_and_upper(fac)
    sl = slice(k * t, (k + 1) * t)
    Li = np.linalg.inv(L[sl, sl])
    Ui = np.linalg.inv(U[sl, sl])
    di = np.tril(Li, -1) + np.triu(Ui)
    lp = L[(k + 1) * t:(k + 2) * t, sl] if (k + 2) * t <= L.shape[0] else None
    up = U[sl, (k + 1) * t:(k + 2) * t] if (k + 2) * t <= U.shape[0] else None
    return di, lp, up


def test_c1_layout(c1_solver):
    from paper_1008_1700_amd import ddps
    torch = torch_cuda()
    m, t, b = ddps.ddps_reduced_layout(c1_solver.h)
    assert (m, t, b) == (384, 64, 64)
    c = torch.empty(m, dtype=torch.int64, device="cuda")
    mask = torch.empty(m, dtype=torch.float64, device="cuda")
    ddps.ddps_reduced_layout(c1_solver.h, c, mask)
    P = oracle_prec(configs.c1())
    assert np.array_equal(host(c)[host(mask) > 0], P.c)


@pytest.mark.parametrize("blk", [0, 2, 3])
def test_c1_factor_tiles(c1, c1_solver, blk):
    from oracle import ddps_oracle as O
    from paper_1008_1700_amd import ddps
    torch = torch_cuda()
    A = c1["A"].scipy()
    lo, hi = c1["part_ptr"][blk], c1["part_ptr"][blk + 1]
    fac = O.factor_block(A[lo:hi, lo:hi].tocsr(), require_no_pivot=True)
    t = 64
    buf = torch.empty(t * t, dtype=torch.float64, device="cuda")
    for k in (0, 1, 7, 15):
        di, lp, up = _expected_tiles(fac, t, k)
        ddps.ddps_get_tile(c1_solver.h, blk, k, 0, buf)
        got = host(buf).reshape(t, t).T
        # unpivoted LU is unique: entry by entry
        assert maxrel(got, di) <= 1e-12, (blk, k)
        if lp is not None:
            ddps.ddps_get_tile(c1_solver.h, blk, k, 1, buf)
            assert maxrel(host(buf).reshape(t, t).T, lp) <= 1e-12
            ddps.ddps_get_tile(c1_solver.h, blk, k, 2, buf)
            assert maxrel(host(buf).reshape(t, t).T, up) <= 1e-12


@pytest.mark.parametrize("blk", [0, 1, 3])
def test_c1_spikes(c1, c1_solver, c1_oracle, blk):
    from paper_1008_1700_amd import ddps
    torch = torch_cuda()
    t = 64
    lo, hi = c1["part_ptr"][blk], c1["part_ptr"][blk + 1]
    ni = hi - lo
    buf = torch.empty(ni * 2 * t, dtype=torch.float64, device="cuda")
    ddps.ddps_get_spikes(c1_solver.h, blk, buf)
    got = host(buf).reshape(2 * t, ni).T
    exp = np.zeros((ni, 2 * t))
    ci, Gi = c1_oracle.c_i[blk], c1_oracle.G[blk]
    for j, col in enumerate(ci):
        q = col - (lo - t) if col < lo else t + (col - hi)
        exp[:, q] = Gi[:, j]
    assert maxrel(got, exp) <= 1e-12


def test_c1_block_solve(c1, c1_solver, c1_oracle):
    from oracle import ddps_oracle as O
    from paper_1008_1700_amd import ddps
    torch = torch_cuda()
    y = np.random.default_rng(3).standard_normal(c1["A"].n)
    g = torch.empty_like(dev_vec(y))
    ddps.ddps_block_solve(c1_solver.h, 1, dev_vec(y), g)
    exp = np.concatenate([O.block_solve(f, y[b.lo:b.hi]) for f, b in zip(c1_oracle.factors, c1_oracle.blocks)])
    assert relerr(host(g), exp) <= 1e-12


def test_c1_reduced_matvec(c1_solver, c1_oracle):
    from paper_1008_1700_amd import ddps
    torch = torch_cuda()
    x = np.random.default_rng(4).standard_normal(384)
    v = torch.empty(384, dtype=torch.float64, device="cuda")
    ddps.ddps_reduced_matvec(c1_solver.h, 1, dev_vec(x), v)
    assert relerr(host(v), c1_oracle.ghat_matvec(x)) <= 1e-12


def test_c1_preconditioner(c1, c1_solver, c1_oracle):
    from paper_1008_1700_amd import ddps
    torch = torch_cuda()
    y = np.random.default_rng(5).standard_normal(c1["A"].n)
    z = torch.empty(c1["A"].n, dtype=torch.float64, device="cuda")
    gh = torch.empty(384, dtype=torch.float64, device="cuda")
    zh = torch.empty(384, dtype=torch.float64, device="cuda")
    its = ddps.ddps_apply_preconditioner(c1_solver.h, 1, dev_vec(y), z, gh, zh)
    ze, d = c1_oracle.apply(y, reduced="dense")
    assert relerr(host(gh), d["ghat"]) <= 1e-12
    assert relerr(host(zh), d["zhat"]) <= 1e-11
    assert relerr(host(z), ze) <= 1e-11
    assert 5 <= its[0] <= 100


def test_c1_locally_preconditioned_inner_solve(c1, c1_solver, c1_oracle):
    """inner_prec=1 (right preconditioning of the reduced BiCGStab by
    I - N, N the interface-local part of G(c,c)): the same preconditioner
    application z = P^{-1} y as the exact reduced solve, in fewer inner
    iterations, matching the oracle's iterate count."""
    from paper_1008_1700_amd import ddps
    torch = torch_cuda()
    S = make_solver(c1, inner_tol=1e-14, max_rhs=4, inner_prec=1)
    try:
        S.factor()
        Y = np.random.default_rng(5).standard_normal((2, c1["A"].n))
        Z = torch.empty(2, c1["A"].n, dtype=torch.float64, device="cuda")
        gh = torch.empty(2 * 384, dtype=torch.float64, device="cuda")
        zh = torch.empty(2 * 384, dtype=torch.float64, device="cuda")
        its = ddps.ddps_apply_preconditioner(S.h, 2, torch.from_numpy(Y).cuda(), Z, gh, zh)
        z0 = torch.empty(c1["A"].n, dtype=torch.float64, device="cuda")
        its0 = ddps.ddps_apply_preconditioner(c1_solver.h, 1, dev_vec(Y[0]), z0)
        for j in range(2):
            ze, d = c1_oracle.apply(Y[j], reduced="dense")
            _, dl = c1_oracle.apply(Y[j], reduced="bicgstab", inner_tol=1e-14, inner_prec="local")
            assert relerr(host(zh)[j * 384:(j + 1) * 384], d["zhat"]) <= 1e-11
            assert relerr(host(Z)[j], ze) <= 1e-11
            print(f"rhs {j}: local-preconditioned {its[j]} iterations, oracle {dl['inner'].iters}")
            assert abs(its[j] - dl["inner"].iters) <= 1.0
        print(f"unpreconditioned: {its0[0]} iterations")
        assert its[0] < its0[0]
    finally:
        S.close()


def test_c1_solve_matches_oracle(c1, c1_solver):
    from oracle import ddps_oracle as O
    A = c1["A"]
    x = dev_vec(np.zeros(A.n))
    rc, info = c1_solver.solve(dev_vec(c1["f"]), x, 1e-12)
    xo, oinfo, _ = O.solve(A.n, A.row_ptr, A.col, A.val, c1["part_ptr"], c1["f"], tol=1e-12, outer="refine",
                           reduced="bicgstab", inner_tol=1e-14)
    xg = host(x)
    assert info.relres_inf <= 1e-12
    assert relerr(xg, xo) <= 1e-8
    assert relerr(xg, c1["x_star"]) <= 1e-9
    r = c1["f"] - A.scipy() @ xg
    assert np.linalg.norm(r, np.inf) / np.linalg.norm(c1["f"], np.inf) <= 1e-12


def test_c1_solve_is_deterministic(c1, c1_solver):
    x1 = dev_vec(np.zeros(c1["A"].n))
    x2 = dev_vec(np.zeros(c1["A"].n))
    c1_solver.solve(dev_vec(c1["f"]), x1, 1e-12)
    c1_solver.solve(dev_vec(c1["f"]), x2, 1e-12)
    assert np.array_equal(host(x1), host(x2))


def test_c1_solve_many(c1, c1_solver):
    from paper_1008_1700_amd import ddps
    torch = torch_cuda()
    A = c1["A"]
    rng = np.random.default_rng(8)
    Xs = rng.uniform(-1, 1, (3, A.n))
    F = np.stack([A.scipy() @ x for x in Xs])
    Fd = dev_vec(F)
    Xd = torch.zeros_like(Fd)
    rc, info = ddps.ddps_solve_many(c1_solver.h, Fd, Xd, 1e-12)
    for j in range(3):
        assert relerr(host(Xd)[j], Xs[j]) <= 1e-9
        x1 = dev_vec(np.zeros(A.n))
        c1_solver.solve(dev_vec(F[j]), x1, 1e-12)
        assert relerr(host(Xd)[j], host(x1)) <= 1e-11


def test_zero_right_hand_side(c1, c1_solver):
    """f = 0 meets any relative tolerance on entry: x stays exactly zero and
    no preconditioner application runs.  As one column of a block of
    right-hand sides it stays zero while the other column is solved."""
    from paper_1008_1700_amd import ddps
    torch = torch_cuda()
    A = c1["A"]
    x = dev_vec(np.zeros(A.n))
    rc, info = c1_solver.solve(dev_vec(np.zeros(A.n)), x, 1e-12)
    assert rc == 0
    assert info.applications == 0
    assert not np.any(host(x))
    F = np.stack([c1["f"], np.zeros(A.n)])
    Fd = dev_vec(F)
    Xd = torch.zeros_like(Fd)
    rc, info = ddps.ddps_solve_many(c1_solver.h, Fd, Xd, 1e-12)
    assert rc == 0
    X = host(Xd)
    assert not np.any(X[1])
    assert relerr(X[0], c1["x_star"]) <= 1e-9


@pytest.mark.parametrize("sizes,b,seed", [
    ([300], 20, 1),                      # p = 1, padded single block
    ([150, 201, 170], 5, 2),             # pad 42 / 55 / 22 rows, t = 64
    ([260, 300, 257, 333, 290], 70, 3),  # t = 128 (two panels per tile), ragged
    ([128, 128], 64, 4),                 # minimum block size 2t, no padding
])
def test_ragged_systems(sizes, b, seed):
    from oracle import ddps_oracle as O
    d = configs.small_banded(len(sizes), sizes, b, seed)
    A = d["A"]
    S = make_solver(d, inner_tol=1e-14)
    try:
        S.factor()
        x = dev_vec(np.zeros(A.n))
        rc, info = S.solve(dev_vec(d["f"]), x, 1e-12)
        xo, _, _ = O.solve(A.n, A.row_ptr, A.col, A.val, d["part_ptr"], d["f"], outer="none")
        assert relerr(host(x), xo) <= 1e-10
        assert info.relres_inf <= 1e-12
    finally:
        S.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_ragged_many_rhs_unaligned_products(dtype):
    """Four right-hand sides on blocks whose padding is not a multiple of
    16 bytes: the reduced products then run on the column-major spikes at
    unaligned row offsets (the one-column-per-load GEMV), and every column
    must match the oracle's direct solution."""
    from oracle import ddps_oracle as O
    from paper_1008_1700_amd import ddps
    torch = torch_cuda()
    d = configs.small_banded(3, [150, 201, 170], 5, 2)    # t = 64, pads 42 / 55 / 22
    A = d["A"]
    rng = np.random.default_rng(11)
    Xs = rng.uniform(-1, 1, (4, A.n))
    F = np.stack([A.scipy() @ x for x in Xs])
    S = make_solver(d, dtype=dtype, inner_tol=1e-14 if dtype == "f64" else 1e-8, max_rhs=4)
    try:
        S.factor()
        Fd = dev_vec(F)
        Xd = torch.zeros_like(Fd)
        rc, info = ddps.ddps_solve_many(S.h, Fd, Xd, 1e-12)
        assert info.relres_inf <= 1e-12
        for j in range(4):
            xo, _, _ = O.solve(A.n, A.row_ptr, A.col, A.val, d["part_ptr"], F[j], outer="none")
            assert relerr(host(Xd)[j], xo) <= 1e-9
    finally:
        S.close()


def test_ragged_spikes_and_padding():
    from paper_1008_1700_amd import ddps
    torch = torch_cuda()
    d = configs.small_banded(3, [150, 201, 170], 5, 2)
    P = oracle_prec(d)
    S = make_solver(d)
    try:
        S.factor()
        t, tiles, pads = ddps.ddps_block_shape(S.h, 3)
        assert t == 64 and tiles == [3, 4, 3] and pads == [42, 55, 22]
        for blk in range(3):
            lo, hi = d["part_ptr"][blk], d["part_ptr"][blk + 1]
            ni = hi - lo
            buf = torch.empty(ni * 2 * t, dtype=torch.float64, device="cuda")
            ddps.ddps_get_spikes(S.h, blk, buf)
            got = host(buf).reshape(2 * t, ni).T
            exp = np.zeros((ni, 2 * t))
            for j, col in enumerate(P.c_i[blk]):
                q = col - (lo - t) if col < lo else t + (col - hi)
                exp[:, q] = P.G[blk][:, j]
            assert relerr(got, exp) <= 1e-11
    finally:
        S.close()


@pytest.mark.parametrize("outer", ["bicgstab", "refine"])
def test_dropping_with_outer_krylov(outer):
    from oracle import ddps_oracle as O
    from paper_1008_1700_amd import ddps
    torch = torch_cuda()
    d = configs.small_banded(4, [300, 280, 310, 290], 40, 7)
    A = d["A"]
    S = make_solver(d, delta=0.5, outer=outer, inner_tol=1e-13)
    try:
        S.factor()
        m, t, b = ddps.ddps_reduced_layout(S.h)
        c = torch.empty(m, dtype=torch.int64, device="cuda")
        mask = torch.empty(m, dtype=torch.float64, device="cuda")
        ddps.ddps_reduced_layout(S.h, c, mask)
        P = O.Preconditioner(A.n, A.row_ptr, A.col, A.val, d["part_ptr"], 0.5)
        assert np.array_equal(host(c)[host(mask) > 0], P.c)
        x = dev_vec(np.zeros(A.n))
        rc, info = S.solve(dev_vec(d["f"]), x, 1e-11)
        assert info.relres_inf <= 1e-11 and info.outer_iters >= 1
        xd = np.linalg.solve(pde.csr_to_dense(A), d["f"])
        assert relerr(host(x), xd) <= 1e-8
    finally:
        S.close()


@pytest.mark.parametrize("dtype", ["f32", "bf16x3", "bf16"])
def test_low_precision_factors_refined_to_fp64(c1, dtype):
    from oracle import ddps_oracle as O
    A = c1["A"]
    S = make_solver(c1, dtype=dtype, inner_tol=1e-10, outer="refine")
    try:
        S.factor()
        x = dev_vec(np.zeros(A.n))
        rc, info = S.solve(dev_vec(c1["f"]), x, 1e-12)
        xo, _, _ = O.solve(A.n, A.row_ptr, A.col, A.val, c1["part_ptr"], c1["f"], outer="none")
        assert info.relres_inf <= 1e-12
        assert relerr(host(x), xo) <= 1e-8
        assert info.outer_iters >= 1
    finally:
        S.close()


def test_singular_block_is_reported():
    from paper_1008_1700_amd import ddps
    d = configs.small_banded(3, [200, 220, 210], 8, 9)
    A = d["A"]
    val = A.val.copy()
    bad = 200 + 37                          # a row of block 1
    a, b = A.row_ptr[bad], A.row_ptr[bad + 1]
    cols = A.col[a:b]
    inblk = (cols >= 200) & (cols < 420)
    val[a:b][inblk] = 0.0                   # the row of A_11 vanishes: exact zero pivot
    A2 = pde.CSR(A.n, A.row_ptr, A.col, val)
    S = make_solver(dict(A=A2, part_ptr=d["part_ptr"]))
    try:
        with pytest.raises(ddps.DDPSError) as e:
            S.factor()
        assert e.value.code == -4
        assert ddps.ddps_last_singular(S.h) == (1, bad)
    finally:
        S.close()


def test_argument_and_state_errors(c1):
    from paper_1008_1700_amd import ddps
    torch = torch_cuda()
    A = c1["A"]
    rp = torch.from_numpy(A.row_ptr).cuda()
    col = torch.from_numpy(A.col).cuda()
    val = torch.from_numpy(A.val).cuda()
    with pytest.raises(ddps.DDPSError) as e:
        ddps.ddps_setup(A.n, 4, [0, 2048, 1024, 3072, 4096], rp, col, val)
    assert e.value.code == -1
    with pytest.raises(ddps.DDPSError) as e:                  # blocks of 64 rows < 2t
        ddps.ddps_setup(A.n, 64, np.arange(65) * 64, rp, col, val)
    assert e.value.code == -1
    o = ddps.ddps_default_options()
    o.mem_budget = 1 << 20
    with pytest.raises(ddps.DDPSError) as e:
        ddps.ddps_setup(A.n, 4, c1["part_ptr"], rp, col, val, o)
    assert e.value.code == -2
    bad = val.clone()
    bad[5] = float("nan")
    with pytest.raises(ddps.DDPSError) as e:
        ddps.ddps_setup(A.n, 4, c1["part_ptr"], rp, col, bad)
    assert e.value.code == -1
    h = ddps.ddps_setup(A.n, 4, c1["part_ptr"], rp, col, val)
    try:
        x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        rc, info = ddps.ddps_solve(h, dev_vec(c1["f"]), x, 1e-10, check=False)
        assert rc == -6
    finally:
        ddps.ddps_destroy(h)


def test_c1_refactor_values_and_guess(c1):
    from paper_1008_1700_amd import ddps
    torch = torch_cuda()
    A = c1["A"]
    S = make_solver(c1, inner_tol=1e-12, guess=True)
    try:
        S.factor()
        x = dev_vec(np.zeros(A.n))
        S.solve(dev_vec(c1["f"]), x, 1e-12)
        zh = torch.empty(384, dtype=torch.float64, device="cuda")
        ddps.ddps_last_reduced(S.h, None, zh)
        # scaled matrix: same pattern, values x 2 -> same solution for f x 2
        ddps.ddps_refactor_values(S.h, dev_vec(2.0 * A.val))
        S.factor()
        ddps.ddps_set_guess(S.h, zh, 1)
        x2 = dev_vec(np.zeros(A.n))
        rc, info = S.solve(dev_vec(2.0 * c1["f"]), x2, 1e-12)
        assert relerr(host(x2), host(x)) <= 1e-10
        # the exact reduced solution as guess needs (almost) no inner iterations
        assert info.inner_iters_avg <= 3
    finally:
        S.close()


@pytest.mark.parametrize("ratio", [-1.0, 0.0, 1e-300])
def test_loosened_refinement_steps(c1, ratio):
    """Refinement with bf16x3 factors on C1: each step cuts the residual by a
    ratio the factors set, so later steps may loosen their inner solve.
    ratio < 0 never loosens; 0 keeps the default guard (10 rho_f); a guard
    of 1e-300 undoes the first loosened step (x and residual restored), stops
    loosening and redoes the step.  Every form must converge to the same bar
    against the oracle's direct solve."""
    from oracle import ddps_oracle as O
    A = c1["A"]
    S = make_solver(c1, dtype="bf16x3", inner_tol=1e-12, outer="refine", loosen_ratio=ratio)
    try:
        S.factor()
        x = dev_vec(np.zeros(A.n))
        rc, info = S.solve(dev_vec(c1["f"]), x, 1e-12)
        ref = O.direct_solve(A.scipy(), c1["f"])
        print(f"loosen_ratio {ratio}: {info.as_dict()}")
        assert rc == 0 and info.relres_inf <= 1e-12
        assert relerr(host(x), ref) <= 1e-8
        if ratio < 0:
            assert info.loosened_steps == 0 and info.undone_steps == 0
        elif ratio == 1e-300:
            # the first loosened step is undone, and no later step loosens
            assert info.loosened_steps == 1 and info.undone_steps == 1
        else:
            assert info.loosened_steps >= 1 and info.undone_steps <= 1
    finally:
        S.close()


@pytest.mark.parametrize("retrieval", [0, 1])
def test_many_rhs_fp32_products_on_matrix_cores(retrieval):
    """FP32 storage with 8 right-hand sides: the reduced products (and with
    retrieval 0 the spike retrieval) run on the FP32 matrix cores with FP32
    sums (gemv_sums 0, the default) or on the vector units with FP64 sums
    (gemv_sums 1).  t = 256, so each tip block has 512 columns: the products'
    main loop and its tail both run.  The two forms agree to the FP32
    rounding of the sums, the FP64-sum form matches the oracle's reduced
    product on c to the FP32 rounding of the spikes, and full solves of both
    forms meet the 1e-12 residual and the direct solution."""
    from paper_1008_1700_amd import ddps
    torch = torch_cuda()
    d = configs.small_banded(4, [600, 652, 700, 620], 200, 5)   # row counts multiples of 4: aligned spike rows
    A = d["A"]
    P = oracle_prec(d)
    Ss = [make_solver(d, dtype="f32", inner_tol=1e-10, max_rhs=8, retrieval=retrieval, work_slots=2, gemv_sums=g)
          for g in (0, 1)]
    try:
        for S in Ss:
            S.factor()
        m, t, _ = ddps.ddps_reduced_layout(Ss[0].h)
        assert t == 256
        c = torch.empty(m, dtype=torch.int64, device="cuda")
        mask = torch.empty(m, dtype=torch.float64, device="cuda")
        ddps.ddps_reduced_layout(Ss[0].h, c, mask)
        on = host(mask) > 0
        assert np.array_equal(host(c)[on], P.c)
        X = np.random.default_rng(21).standard_normal((8, m)) * on
        V = []
        for S in Ss:
            v = torch.empty(8, m, dtype=torch.float64, device="cuda")
            ddps.ddps_reduced_matvec(S.h, 8, dev_vec(X), v)
            V.append(host(v))
        assert not np.array_equal(V[0], V[1])             # two arithmetic paths
        assert maxrel(V[0], V[1]) <= 1e-5
        for j in range(8):
            assert maxrel(V[1][j][on], P.ghat_matvec(X[j][on])) <= 1e-4
        Xs = np.random.default_rng(22).uniform(-1, 1, (8, A.n))
        F = np.stack([A.scipy() @ x for x in Xs])
        for S in Ss:
            Xd = torch.zeros(8, A.n, dtype=torch.float64, device="cuda")
            rc, info = ddps.ddps_solve_many(S.h, dev_vec(F), Xd, 1e-12)
            assert rc == 0 and info.relres_inf <= 1e-12
            assert relerr(host(Xd), Xs) <= 1e-9
    finally:
        for S in Ss:
            S.close()


@pytest.mark.parametrize("dtype,retrieval", [("bf16x3", 0), ("f64", 1)])
def test_inner_preconditioner_many_rhs(dtype, retrieval):
    """The interface-local inner preconditioner (inner_prec 1) on the two
    paths the benchmark times it on: mixed storage with 8 right-hand sides
    (the products on the FP32 matrix cores) and plain FP64 with the spike tips
    only and the re-solved retrieval.  Both forms of the inner solve reach the
    same solutions as the direct solve; the preconditioned one in no more
    inner iterations."""
    from paper_1008_1700_amd import ddps
    torch = torch_cuda()
    d = configs.small_banded(4, [600, 652, 700, 620], 200, 5)
    A = d["A"]
    Xs = np.random.default_rng(23).uniform(-1, 1, (8, A.n))
    F = np.stack([A.scipy() @ x for x in Xs])
    its = []
    for prec in (0, 1):
        S = make_solver(d, dtype=dtype, inner_tol=1e-10, max_rhs=8, retrieval=retrieval, work_slots=2,
                        inner_prec=prec)
        try:
            S.factor()
            Xd = torch.zeros(8, A.n, dtype=torch.float64, device="cuda")
            rc, info = ddps.ddps_solve_many(S.h, dev_vec(F), Xd, 1e-12)
            assert rc == 0 and info.relres_inf <= 1e-12
            assert relerr(host(Xd), Xs) <= 1e-9
            its.append(info.inner_iters_total / max(info.applications, 1))
        finally:
            S.close()
    print(f"{dtype}: inner iterations per application {its[0]:.2f} -> {its[1]:.2f}")
    assert its[1] <= its[0]

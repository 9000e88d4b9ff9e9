"""Pins for the CPU oracle: each test ties it to something other than itself
(the paper's printed worked example, dense LAPACK, brute force on tiny
inputs, closed forms, and special cases of the method)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import ddps_oracle as O
from tests.golden.fixtures import worked_example
from workloads import configs, pde


def _prec_from_dense(A, part, delta=0.0):
    S = sp.csr_matrix(A)
    return O.Preconditioner(A.shape[0], S.indptr, S.indices, S.data, part, delta)


# ---------------------------------------------------------------- worked example
@pytest.fixture(scope="module")
def we():
    return worked_example()


def test_worked_example_c(we):
    P = _prec_from_dense(we["A"], we["part_ptr"])
    assert list(P.c + 1) == list(we["c"])


def test_worked_example_g_G_zhat_x(we):
    P = _prec_from_dense(we["A"], we["part_ptr"])
    z, d = P.apply(we["f"])
    for key, got in (("g", d["g"]), ("zhat", d["zhat"]), ("x", z)):
        val, tol = we[key]
        assert np.all(np.abs(got - val) <= tol * (1 + 1e-9)), (key, got, val)
    G = np.zeros((9, 9))
    for b, ci, Gi in zip(P.blocks, P.c_i, P.G):
        G[b.lo:b.hi][:, ci] = Gi
    val, tol = we["G"]
    got = G[:, we["c"] - 1]
    assert np.all(np.abs(got - val) <= tol * (1 + 1e-9)), (got, val)


def test_worked_example_ghat(we):
    # G^ = I(c,c) + G(c,c): rows of the printed G at c, plus the identity.
    P = _prec_from_dense(we["A"], we["part_ptr"])
    val, tol = we["G"]
    c = we["c"] - 1
    expect = np.eye(4) + val[c, :]
    assert np.all(np.abs(P.ghat_dense() - expect) <= tol[c, :] * (1 + 1e-9))


def test_worked_example_delta_09(we):
    # Dropping rule by hand: block 1 has column norms {5: 0.3, 9: 0.01}, so
    # the threshold is 0.27: keep 5, drop 9.  Block 2 has {2: 0.2, 9: 1.1},
    # threshold 0.99: keep 9, drop 2.  Block 3 has {1: 1.2}: keep 1.
    # c = {1, 5, 9}.
    P = _prec_from_dense(we["A"], we["part_ptr"], delta=0.9)
    assert list(P.c + 1) == [1, 5, 9]


def test_worked_example_outer_is_half_step(we):
    # With nothing dropped, exact LU and an exact reduced solve, P = A, so
    # preconditioned BiCGStab finishes in its first half step (count 0.5).
    S = sp.csr_matrix(we["A"])
    x, info, _ = O.solve(9, S.indptr, S.indices, S.data, we["part_ptr"], we["f"],
                         outer="bicgstab", tol=1e-12)
    assert info.outer_iters == 0.5
    assert np.allclose(x, np.linalg.solve(we["A"], we["f"]), rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------- direct invariant
@pytest.mark.parametrize("sizes,b,seed", [
    ([120], 7, 1),                    # p = 1
    ([60, 61], 5, 2),                 # p = 2, uneven
    ([40, 75, 33], 9, 3),             # p = 3, uneven
    ([50, 47, 64, 29, 80], 6, 4),     # p = 5, uneven
    ([130, 140, 130], 31, 5),         # wide band
])
def test_direct_invariant_vs_dense_solve(sizes, b, seed):
    d = configs.small_banded(len(sizes), sizes, b, seed)
    A = d["A"]
    x, info, _ = O.solve(A.n, A.row_ptr, A.col, A.val, d["part_ptr"], d["f"], outer="none")
    ref = np.linalg.solve(pde.csr_to_dense(A), d["f"])
    assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)


def test_direct_invariant_bicgstab_inner():
    d = configs.small_banded(4, [70, 90, 64, 77], 8, 11)
    A = d["A"]
    x, info, _ = O.solve(A.n, A.row_ptr, A.col, A.val, d["part_ptr"], d["f"], outer="none",
                         reduced="bicgstab", inner_tol=1e-14)
    ref = np.linalg.solve(pde.csr_to_dense(A), d["f"])
    assert np.linalg.norm(x - ref) <= 1e-11 * np.linalg.norm(ref)


def test_block_jacobi_when_everything_dropped():
    d = configs.small_banded(3, [50, 60, 70], 6, 21)
    A = d["A"]
    P = O.Preconditioner(A.n, A.row_ptr, A.col, A.val, d["part_ptr"], delta=1.0)
    assert P.m == 0
    y = np.random.default_rng(0).standard_normal(A.n)
    z, _ = P.apply(y)
    Ad = pde.csr_to_dense(A)
    p = d["part_ptr"]
    for i in range(3):
        lo, hi = p[i], p[i + 1]
        assert np.allclose(z[lo:hi], np.linalg.solve(Ad[lo:hi, lo:hi], y[lo:hi]), rtol=1e-12)


def test_spikes_equal_dense_inverse_products():
    d = configs.small_banded(3, [64, 80, 72], 10, 31)
    A = d["A"]
    P = O.Preconditioner(A.n, A.row_ptr, A.col, A.val, d["part_ptr"])
    Ad = pde.csr_to_dense(A)
    for b, ci, Gi in zip(P.blocks, P.c_i, P.G):
        ref = np.linalg.inv(Ad[b.lo:b.hi, b.lo:b.hi]) @ Ad[b.lo:b.hi][:, ci]
        assert np.allclose(Gi, ref, rtol=1e-11, atol=1e-13)
    # every candidate coupling column of a banded matrix is in c
    assert P.m == 2 * 10 * 2


def test_block_lu_matches_brute_force_doolittle():
    # Tiny dense block, pure-Python Doolittle elimination without pivoting.
    d = configs.small_banded(1, [12], 3, 41)
    A = pde.csr_to_dense(d["A"])
    n = A.shape[0]
    L = [[float(i == j) for j in range(n)] for i in range(n)]
    U = [[0.0] * n for _ in range(n)]
    for i in range(n):
        for j in range(i, n):
            U[i][j] = A[i, j] - sum(L[i][k] * U[k][j] for k in range(i))
        for j in range(i + 1, n):
            L[j][i] = (A[j, i] - sum(L[j][k] * U[k][i] for k in range(i))) / U[i][i]
    S = sp.csr_matrix(A)
    fac = O.factor_block(S, require_no_pivot=True)
    Lo, Uo = O.unit_lower_and_upper(fac)
    assert np.allclose(Lo, np.array(L), rtol=1e-13, atol=1e-15)
    assert np.allclose(Uo, np.array(U), rtol=1e-13, atol=1e-15)


def test_block_lu_backward_error_on_c1_block():
    d = configs.c1()
    A = d["A"]
    S = A.scipy()
    blk = S[:1024, :1024].tocsr()
    fac = O.factor_block(blk, require_no_pivot=True)
    L, U = O.unit_lower_and_upper(fac)
    Ad = blk.toarray()
    err = np.linalg.norm(L @ U - Ad, np.inf) / np.linalg.norm(Ad, np.inf)
    assert err <= 1024 * np.finfo(float).eps


# ---------------------------------------------------------------- BiCGStab
def test_bicgstab_half_step_on_scaled_identity():
    b = np.random.default_rng(1).standard_normal(17)
    x, info = O.bicgstab(lambda v: 2.0 * v, b, tol=1e-14)
    assert info.iters == 0.5 and info.converged
    assert np.allclose(x, b / 2.0, rtol=0, atol=1e-15)


def test_bicgstab_solves_nonsymmetric_system():
    d = configs.small_banded(1, [200], 6, 51)
    Ad = pde.csr_to_dense(d["A"])
    x, info = O.bicgstab(lambda v: Ad @ v, d["f"], tol=1e-13, maxit=500)
    assert info.converged
    ref = np.linalg.solve(Ad, d["f"])
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)


def test_bicgstab_reports_breakdown():
    # Rotation: r~' A r = 0 for every r, so r~'v = 0 at once and again after
    # the restart with r~ = r.
    R = np.array([[0.0, 1.0], [-1.0, 0.0]])
    x, info = O.bicgstab(lambda v: R @ v, np.array([1.0, 0.0]), tol=1e-12, maxit=10)
    assert info.breakdown and not info.converged


# ---------------------------------------------------------------- outer layer
@pytest.mark.parametrize("outer", ["refine", "bicgstab"])
def test_outer_layer_with_dropping(outer):
    d = configs.small_banded(4, [80, 90, 70, 85], 8, 61)
    A = d["A"]
    x, info, _ = O.solve(A.n, A.row_ptr, A.col, A.val, d["part_ptr"], d["f"], delta=0.5,
                         outer=outer, tol=1e-11, reduced="bicgstab", inner_tol=1e-12)
    assert info.converged and info.relres_inf <= 1e-11
    assert info.outer_iters >= 1
    assert np.linalg.norm(x - d["x_star"]) <= 1e-8 * np.linalg.norm(d["x_star"])


def test_c1_end_to_end_against_sparse_lu():
    d = configs.c1()
    A = d["A"]
    x, info, P = O.solve(A.n, A.row_ptr, A.col, A.val, d["part_ptr"], d["f"], outer="refine",
                         tol=1e-12, reduced="bicgstab", inner_tol=1e-12)
    ref = spla.splu(A.scipy().tocsc()).solve(d["f"])
    assert info.relres_inf <= 1e-12
    assert P.m == 384
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)
    assert np.linalg.norm(x - d["x_star"]) <= 1e-9 * np.linalg.norm(d["x_star"])


# ---------------------------------------------------------------- planted mistakes
def test_planted_sign_error_in_retrieval_is_caught(we, monkeypatch):
    orig = O.Preconditioner.g_times
    monkeypatch.setattr(O.Preconditioner, "g_times", lambda self, zc: -orig(self, zc))
    P = _prec_from_dense(we["A"], we["part_ptr"])
    z, d = P.apply(we["f"])
    val, tol = we["x"]
    assert not np.all(np.abs(z - val) <= tol)


def test_planted_strict_drop_test_is_caught(monkeypatch):
    # '<' instead of '<=' keeps the largest column at delta = 1.
    def bad(Ri, delta):
        cols, norms = O.column_inf_norms(Ri)
        return np.sort(cols[~(norms < delta * norms.max())]) if cols.size else cols
    monkeypatch.setattr(O, "kept_columns", bad)
    d = configs.small_banded(3, [50, 60, 70], 6, 21)
    A = d["A"]
    P = O.Preconditioner(A.n, A.row_ptr, A.col, A.val, d["part_ptr"], delta=1.0)
    assert P.m != 0


def test_local_part_of_reduced_matrix():
    # N is a restriction of G(c,c): with one interface (p = 2) it is all of
    # it, and in general N and the rest split G^ - I entry by entry (each
    # entry of G(c,c) is either local or not).
    from oracle import ddps_oracle as O
    d = configs.small_banded(2, [150, 170], 6, 3)
    A = d["A"]
    P = O.Preconditioner(A.n, A.row_ptr, A.col, A.val, d["part_ptr"])
    rng = np.random.default_rng(4)
    z = rng.standard_normal(P.m)
    assert np.allclose(P.local_matvec(z), P.ghat_matvec(z) - z, rtol=1e-14, atol=1e-14)
    d = configs.small_banded(4, [150, 170, 160, 140], 6, 3)
    A = d["A"]
    P = O.Preconditioner(A.n, A.row_ptr, A.col, A.val, d["part_ptr"])
    Gm = P.ghat_dense() - np.eye(P.m)
    Nm = np.column_stack([P.local_matvec(e) for e in np.eye(P.m)])
    # Same-interface support, built from the partition alone: a reduced row
    # (a global row in c) and a reduced column (a global column in c) belong
    # to the interface whose boundary is nearest; N must equal G(c,c) on every
    # entry whose row and column share an interface (zero entries included)
    # and be zero on every other entry.
    part = np.asarray(d["part_ptr"])
    bnd = part[1:-1]
    iface = np.abs(P.c[:, None] - bnd[None, :]).argmin(axis=1)
    same = iface[:, None] == iface[None, :]
    assert np.array_equal(Nm[same], Gm[same])
    assert np.all(Nm[~same] == 0.0)
    assert (Gm[same] != 0).sum() > 0 and (Gm[~same] != 0).sum() > 0   # both parts are present


def test_locally_preconditioned_inner_solve_gives_same_solution():
    from oracle import ddps_oracle as O
    d = configs.small_banded(5, [150, 170, 160, 140, 155], 6, 8)
    A = d["A"]
    P = O.Preconditioner(A.n, A.row_ptr, A.col, A.val, d["part_ptr"])
    y = np.random.default_rng(1).standard_normal(A.n)
    z0, r0 = P.apply(y, reduced="dense")
    z1, r1 = P.apply(y, reduced="bicgstab", inner_tol=1e-13, inner_prec="local")
    z2, r2 = P.apply(y, reduced="bicgstab", inner_tol=1e-13)
    assert np.allclose(z1, z0, rtol=1e-10, atol=1e-11)
    assert r1["inner"].iters <= r2["inner"].iters


# ---------------------------------------------------------------- re-solve retrieval
@pytest.mark.parametrize("delta", [0.0, 0.5, 0.9, 1.0])
def test_both_retrieval_forms_solve_P_z_equals_y(delta):
    # Figure 2 solves P z = y with P = D~ + R~ (Section 3): D the block
    # diagonal of A, R~ the off-block part with the dropped columns removed.
    # Assemble P explicitly from A and the kept columns and check P z = y for
    # the printed retrieval (z = g - G z) and the re-solved one
    # (z = D~^{-1}(y - R~ z)); with delta = 0, P = A.
    d = configs.small_banded(3, [90, 110, 100], 7, 12)
    A = d["A"]
    Pc = O.Preconditioner(A.n, A.row_ptr, A.col, A.val, d["part_ptr"], delta)
    Ad = pde.csr_to_dense(A)
    part = d["part_ptr"]
    Pm = np.zeros_like(Ad)
    for i, ci in enumerate(Pc.c_i):
        lo, hi = part[i], part[i + 1]
        Pm[lo:hi, lo:hi] = Ad[lo:hi, lo:hi]
        Pm[lo:hi, ci] = Ad[lo:hi, ci]
    if delta == 0.0:
        assert np.array_equal(Pm, Ad)
    y = np.random.default_rng(5).standard_normal(A.n)
    for form in ("spikes", "resolve"):
        z, _ = Pc.apply(y, reduced="dense", retrieval=form)
        assert np.linalg.norm(Pm @ z - y) <= 1e-12 * np.linalg.norm(y), form


def test_resolve_retrieval_outer_solve_matches_direct():
    d = configs.c1()
    A = d["A"]
    x, info, _ = O.solve(A.n, A.row_ptr, A.col, A.val, d["part_ptr"], d["f"], outer="none", retrieval="resolve")
    xd = spla.spsolve(A.scipy().tocsc(), d["f"])
    assert np.linalg.norm(x - xd) <= 1e-11 * np.linalg.norm(xd)


def test_two_norm_outer_stop():
    d = configs.small_banded(3, [90, 110, 100], 7, 13)
    A = d["A"]
    x, info, _ = O.solve(A.n, A.row_ptr, A.col, A.val, d["part_ptr"], d["f"], delta=0.6, outer="refine",
                         tol=1e-9, norm="2")
    r = d["f"] - A.scipy() @ x
    assert info.converged and np.linalg.norm(r) <= 1e-9 * np.linalg.norm(d["f"])


# ---------------------------------------------------------------- condition estimates
@pytest.mark.parametrize("seed", range(8))
def test_cond1_estimate_is_a_lower_bound_within_3x(seed):
    # kappa_1 = ||A||_1 ||A^{-1}||_1 computed exactly from the dense inverse.
    # The Hager-Higham estimate is ||A^{-1} x||_1 ||A||_1 for a unit-1-norm x,
    # so it can never exceed it; on these matrices it comes within 3x.
    rng = np.random.default_rng(seed)
    n = 4 + 6 * seed
    A = rng.standard_normal((n, n)) + (seed % 3) * np.eye(n)
    A[:, 0] *= 10.0 ** (seed % 4)                  # spread the column scales
    exact = np.linalg.norm(A, 1) * np.linalg.norm(np.linalg.inv(A), 1)
    est = O.cond1_dense_estimate(A)
    assert exact / 3.0 <= est <= exact * (1.0 + 1e-10)


def test_cond1_estimate_exact_on_diagonal_and_permuted_diagonal():
    dvals = np.array([3.0, -0.25, 7.0, 1e-3, 2.0])
    exact = 7.0 / 1e-3
    assert np.isclose(O.cond1_dense_estimate(np.diag(dvals)), exact, rtol=1e-13)
    Pm = np.eye(5)[[2, 0, 4, 1, 3]]
    assert np.isclose(O.cond1_dense_estimate(Pm @ np.diag(dvals)), exact, rtol=1e-13)


def _random_m_matrix(n, seed, dominance=0.05):
    rng = np.random.default_rng(seed)
    B = sp.random(n, n, density=0.2, random_state=rng, data_rvs=lambda k: rng.uniform(0.1, 1.0, k)).tocsr()
    B.setdiag(0.0)
    B.eliminate_zeros()
    rows = np.asarray(B.sum(axis=1)).ravel()
    return (sp.diags(rows + dominance + rng.uniform(0, 0.1, n)) - B).tocsr()


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_mmatrix_bounds_bracket_exact_kinf(seed):
    A = _random_m_matrix(40, seed)
    Ad = A.toarray()
    inv = np.linalg.inv(Ad)
    assert np.all(inv >= -1e-15)                           # an M-matrix has a nonnegative inverse
    exact = np.abs(Ad).sum(axis=1).max() * np.abs(inv).sum(axis=1).max()
    y = inv @ np.ones(40)
    lo, hi = O.mmatrix_kinf_bounds(A, y)
    assert lo <= exact <= hi and hi / lo < 1.0 + 1e-10     # the exact A^{-1} 1 gives a tight bracket
    yp = inv @ (1.0 + 4.0 * np.random.default_rng(seed).uniform(0, 1, 40))
    lo2, hi2 = O.mmatrix_kinf_bounds(A, yp)
    assert lo2 <= exact <= hi2 and hi2 / lo2 > 1.5          # any positive y with A y > 0 still brackets it
    assert O.mmatrix_kinf_bounds(A, -y) is None
    Ap = A.tolil(); Ap[0, 1] = 0.5
    assert O.mmatrix_kinf_bounds(Ap.tocsr(), y) is None     # not a Z-matrix


def test_mmatrix_bounds_on_c1_match_the_dense_inverse():
    d = configs.c1()
    A = d["A"].scipy()
    Ad = A.toarray()
    inv = np.linalg.inv(Ad)
    exact = np.abs(Ad).sum(axis=1).max() * np.abs(inv).sum(axis=1).max()
    lo, hi = O.mmatrix_kinf_bounds(A, spla.spsolve(A.tocsc(), np.ones(A.shape[0])))
    assert lo <= exact <= hi and hi / lo < 1.0 + 1e-8
    # and the 1-norm estimate through the dense LU is within 3x of the exact 1-norm condition number
    exact1 = np.abs(Ad).sum(axis=0).max() * np.abs(inv).sum(axis=0).max()
    est1 = O.cond1_dense_estimate(A)
    assert exact1 / 3.0 <= est1 <= exact1 * (1.0 + 1e-10)


@pytest.mark.parametrize("seed", [0, 1])
def test_direct_solve_matches_dense_solve_and_residual(seed):
    """The sparse direct solve that stands for the exact solution of a large
    system: against LAPACK's dense solve on a small nonsymmetric banded
    system (one and several columns), and by its residual."""
    d = configs.small_banded(3, [70, 90, 80], 12, 40 + seed)
    A = d["A"].scipy()
    rng = np.random.default_rng(seed)
    F = rng.standard_normal((A.shape[0], 3))
    X = O.direct_solve(A, F)
    ref = np.linalg.solve(A.toarray(), F)
    assert np.max(np.abs(X - ref)) <= 1e-12 * np.max(np.abs(ref))
    x1 = O.direct_solve(A, F[:, 0])
    assert x1.shape == (A.shape[0],) and np.array_equal(x1, X[:, 0])
    r = F - A @ X
    assert np.max(np.abs(r)) <= 1e-13 * np.max(np.abs(F))

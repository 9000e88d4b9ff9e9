"""Pins for the oracle's incomplete block factors (ILU(0), the reading of
Section 3's L~_i U~_i): each test ties factor_block_ilu0 to something other
than its own loop (the defining property checked with a sparse product,
LAPACK's LU where zero fill is no restriction, closed forms) and the DDPS
pieces built on it to the explicit preconditioner P = D~ + R~."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import ddps_oracle as O
from workloads import configs, pde


def _csr(A):
    S = sp.csr_matrix(A.scipy() if hasattr(A, "scipy") else A)
    S.sort_indices()
    return S


def _pattern(S):
    S = sp.csr_matrix(S).copy()
    S.data = np.ones_like(S.data)
    return S


@pytest.mark.parametrize("kind", ["convdiff2d", "geometric"])
def test_ilu0_reproduces_a_on_its_pattern(kind):
    """The definition: L~ unit lower, U~ upper, both inside the pattern of A,
    and (L~ U~)(i, j) = a_ij at every stored (i, j); the product differs
    from A elsewhere (fill was dropped, so the factors are not exact)."""
    if kind == "convdiff2d":
        A = _csr(pde.convdiff2d(12, 11, (20.0, -7.0)))
    else:
        A = _csr(pde.random_geometric(400, 7, 3))
    F = O.factor_block_ilu0(A)
    L, U = F.L.tocsr(), F.U.tocsr()
    assert np.allclose(L.diagonal(), 1.0)
    assert sp.triu(L, 1).nnz == 0 and sp.tril(U, -1).nnz == 0
    P = _pattern(A)
    assert ((_pattern(sp.tril(L, -1)) + _pattern(U)) - P).max() <= 0  # inside the pattern
    LU = (L @ U).tocsr()
    on = LU.multiply(P) - A
    assert abs(on).max() <= 1e-13 * abs(A).max()
    off = LU - LU.multiply(P)
    assert abs(off).max() > 1e-6 * abs(A).max()


@pytest.mark.parametrize("case", ["tridiagonal", "full_band"])
def test_ilu0_is_the_lu_when_nothing_fills(case):
    """With a pattern that LU does not fill (tridiagonal; a band stored in
    full) ILU(0) is the exact LU: LAPACK's band LU of the same block."""
    rng = np.random.default_rng(11)
    n = 60
    if case == "tridiagonal":
        A = sp.diags([rng.uniform(-1, 0, n - 1), rng.uniform(3, 4, n), rng.uniform(-1, 0, n - 1)], [-1, 0, 1])
    else:
        bl, bu = 3, 2
        D = np.zeros((n, n))
        for i in range(n):
            for j in range(max(0, i - bl), min(n, i + bu + 1)):
                D[i, j] = rng.uniform(-1, 0) if i != j else rng.uniform(6, 7)
        A = sp.csr_matrix(D)
    A = sp.csr_matrix(A)
    F = O.factor_block_ilu0(A)
    fac = O.factor_block(A, require_no_pivot=True)
    L, U = O.unit_lower_and_upper(fac)
    assert np.max(np.abs(F.L.toarray() - L)) <= 1e-13
    assert np.max(np.abs(F.U.toarray() - U)) <= 1e-13 * np.max(np.abs(U))


def test_ilu0_of_a_diagonal_and_a_triangular_matrix():
    """Closed forms: a diagonal matrix gives L~ = I and U~ = A; an upper
    triangular one gives L~ = I, U~ = A; a lower triangular one L~ = A D^{-1}
    (D its diagonal) and U~ = D."""
    rng = np.random.default_rng(4)
    d = rng.uniform(1, 2, 30)
    F = O.factor_block_ilu0(sp.diags(d))
    assert np.array_equal(F.L.toarray(), np.eye(30)) and np.array_equal(F.U.toarray(), np.diag(d))
    Up = sp.csr_matrix(np.triu(rng.uniform(-1, 1, (30, 30))) + np.diag(d))
    F = O.factor_block_ilu0(Up)
    assert np.array_equal(F.L.toarray(), np.eye(30)) and np.allclose(F.U.toarray(), Up.toarray(), rtol=0, atol=0)
    Lo = np.tril(rng.uniform(-1, 1, (30, 30)), -1) + np.diag(d)
    F = O.factor_block_ilu0(sp.csr_matrix(Lo))
    assert np.allclose(F.L.toarray(), Lo / d[None, :], rtol=1e-15, atol=0)
    assert np.allclose(F.U.toarray(), np.diag(d), rtol=0, atol=0)


def test_ilu0_rejects_a_missing_diagonal():
    A = sp.csr_matrix(np.array([[2.0, -1.0, 0.0], [-1.0, 0.0, -1.0], [0.0, -1.0, 2.0]]))
    A.eliminate_zeros()
    with pytest.raises(np.linalg.LinAlgError):
        O.factor_block_ilu0(A)


def test_ilu_preconditioner_is_d_tilde_plus_r_tilde():
    """P z = y with D~ = blockdiag(L~_i U~_i) built explicitly from the
    factors (sparse products) and R~ = A outside the blocks: every piece of
    Figure 2 (block solve, spikes, reduced solve, both retrievals) computed
    with the incomplete factors solves it."""
    cfg = configs.small_banded(4, [150, 130, 170, 140], 9, 5)
    S, part = _csr(cfg["A"]), cfg["part_ptr"]
    P = O.Preconditioner(S.shape[0], S.indptr, S.indices, S.data, part, 0.0, block_factor="ilu0")
    n = S.shape[0]
    D = sp.lil_matrix((n, n))
    for b, F in zip(P.blocks, P.factors):
        D[b.lo:b.hi, b.lo:b.hi] = (F.L @ F.U).toarray()
    D = D.tocsr()
    Dmask = sp.lil_matrix((n, n))
    for b in P.blocks:
        Dmask[b.lo:b.hi, b.lo:b.hi] = 1.0
    Rt = S - S.multiply(Dmask.tocsr())
    Pm = (D + Rt).tocsc()
    y = np.random.default_rng(2).uniform(-1, 1, n)
    exp = spla.spsolve(Pm, y)
    for retrieval in ("spikes", "resolve"):
        z, d = P.apply(y, retrieval=retrieval)
        assert np.linalg.norm(z - exp) <= 1e-11 * np.linalg.norm(exp)
    # D~ differs from D: the preconditioner is not the exact one
    Pex = O.Preconditioner(S.shape[0], S.indptr, S.indices, S.data, part, 0.0)
    zex, _ = Pex.apply(y)
    assert np.linalg.norm(zex - exp) > 1e-6 * np.linalg.norm(exp)


def test_ilu_ddps_solves_with_the_outer_layer():
    """DDPS with incomplete block factors as the preconditioner of the outer
    BiCGStab reaches the direct solution (Section 3: approximate factors are
    won back by the outer layer), with more iterations than exact factors."""
    cfg = configs.small_banded(4, [150, 130, 170, 140], 9, 5)
    S, part = _csr(cfg["A"]), cfg["part_ptr"]
    xs = np.random.default_rng(3).uniform(-1, 1, S.shape[0])
    f = S @ xs
    x, info, _ = O.solve(S.shape[0], S.indptr, S.indices, S.data, part, f, tol=1e-12, outer="bicgstab",
                         block_factor="ilu0")
    assert info.converged
    assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)
    _, info_lu, _ = O.solve(S.shape[0], S.indptr, S.indices, S.data, part, f, tol=1e-12, outer="bicgstab")
    assert info.outer_iters > info_lu.outer_iters

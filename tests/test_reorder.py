"""Host-side preparation of general sparse matrices (reverse Cuthill-McKee,
symmetric permutation, half-bandwidth, equal-slab partition), checked on the
CPU against properties the orderings must have and against SciPy's RCM."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import reverse_cuthill_mckee

from workloads import pde


def _lib():
    from paper_1008_1700_amd import ddps
    return ddps


def _shuffled(M, seed):
    q = np.random.default_rng(seed).permutation(M.shape[0])
    return M[q][:, q].tocsr(), q


def _band(M):
    C = M.tocoo()
    return int(np.max(np.abs(C.row - C.col))) if C.nnz else 0


def test_path_graph_gets_bandwidth_one():
    ddps = _lib()
    n = 500
    P = sp.diags([np.ones(n - 1), 2 * np.ones(n), np.ones(n - 1)], [-1, 0, 1]).tocsr()
    S, _ = _shuffled(P, 1)
    perm = ddps.ddps_rcm(n, S.indptr, S.indices)
    assert np.array_equal(np.sort(perm), np.arange(n))
    assert _band(S[perm][:, perm]) == 1


@pytest.mark.parametrize("nx,ny", [(30, 50), (64, 64)])
def test_grid_bandwidth_close_to_grid_width(nx, ny):
    """A shuffled 5-point grid: RCM from a corner numbers the anti-diagonals,
    whose widths are at most min(nx, ny), so the bandwidth stays within
    twice that; and no worse than SciPy's RCM by more than a few rows."""
    ddps = _lib()
    G = pde.convdiff2d(nx, ny, (1.0, 2.0)).scipy()
    S, _ = _shuffled(G, 2)
    perm = ddps.ddps_rcm(G.shape[0], S.indptr, S.indices)
    b = _band(S[perm][:, perm])
    b_ref = _band(S[reverse_cuthill_mckee(S, symmetric_mode=False)][:, reverse_cuthill_mckee(S, symmetric_mode=False)])
    assert b <= 2 * min(nx, ny)
    assert b <= b_ref + 4
    assert ddps.ddps_bandwidth(G.shape[0], S.indptr, S.indices) > 10 * b


def test_components_nonsymmetric_pattern_and_permuted_csr():
    """Two disconnected shuffled grids plus one-sided (nonsymmetric)
    couplings: every node is numbered once, the permuted CSR equals
    P A P^T entry for entry with sorted columns, and the pattern of A + A^T
    (not A alone) decides the order."""
    ddps = _lib()
    G1 = pde.convdiff2d(20, 30, (3.0, 1.0)).scipy()
    G2 = pde.convdiff2d(25, 12, (1.0, 1.0)).scipy()
    M = sp.block_diag([G1, G2]).tolil()
    M[5, 40] = -0.3            # upper-only entries inside the first component
    M[100, 7] = -0.2
    S, q = _shuffled(M.tocsr(), 3)
    n = S.shape[0]
    perm = ddps.ddps_rcm(n, S.indptr, S.indices)
    assert np.array_equal(np.sort(perm), np.arange(n))
    rp, col, val = ddps.ddps_permute_csr(n, S.indptr, S.indices, S.data, perm)
    B = sp.csr_matrix((val, col, rp), shape=(n, n))
    ref = S[perm][:, perm].tocsr()
    ref.sort_indices()
    assert np.array_equal(B.indptr, ref.indptr) and np.array_equal(B.indices, ref.indices)
    assert np.array_equal(B.data, ref.data)
    for i in range(n):
        assert np.all(np.diff(col[rp[i]:rp[i + 1]]) > 0)
    # each component occupies one contiguous range of the new numbering:
    # new row i is shuffled row perm[i], which is original row q[perm[i]]
    comp = np.r_[np.zeros(G1.shape[0], int), np.ones(G2.shape[0], int)]
    labels = comp[q[perm]]
    assert np.count_nonzero(np.diff(labels)) == 1
    assert _band(B) <= 2 * 30 + 2


def test_partition_rows():
    ddps = _lib()
    part = ddps.ddps_partition_rows(10000, 150, 16)        # t = 192: slabs of at least 384 rows
    sizes = np.diff(part)
    assert part[0] == 0 and part[-1] == 10000 and len(sizes) == 16
    assert sizes.max() - sizes.min() <= 1 and sizes.min() >= 384
    part = ddps.ddps_partition_rows(10000, 700, 64)        # t = 704: at most 7 slabs
    sizes = np.diff(part)
    assert len(sizes) == 7 and sizes.min() >= 2 * 704
    assert len(ddps.ddps_partition_rows(100, 200, 8)) == 2  # too small to split: one block
    with pytest.raises(ddps.DDPSError):
        ddps.ddps_partition_rows(100, 10, 0)


def test_errors():
    ddps = _lib()
    with pytest.raises(ddps.DDPSError):
        ddps.ddps_rcm(3, np.array([0, 1, 2, 3]), np.array([0, 5, 2]))      # column out of range
    with pytest.raises(ddps.DDPSError):
        ddps.ddps_permute_csr(3, np.array([0, 1, 2, 3]), np.array([0, 1, 2]), None, np.array([0, 0, 2]))


def test_random_geometric_system_becomes_banded():
    """The general test system: shuffled, its bandwidth is of order n; after
    RCM it is a small fraction of n, and the permuted blocks satisfy the
    banded path's requirement."""
    ddps = _lib()
    A = pde.random_geometric(6000, 8, 5)
    b0 = ddps.ddps_bandwidth(A.n, A.row_ptr, A.col)
    gs = ddps.GeneralSystem(A.n, A.row_ptr, A.col, A.val, 8)
    assert b0 > A.n // 2 and gs.b < A.n // 20
    t = max(64, -(-gs.b // 64) * 64)
    assert len(gs.part_ptr) - 1 >= 2 and np.min(np.diff(gs.part_ptr)) >= 2 * t
    x = np.random.default_rng(1).standard_normal(A.n)
    Ap = sp.csr_matrix((gs.val, gs.col, gs.row_ptr), shape=(A.n, A.n))
    assert np.allclose(gs.from_perm(Ap @ gs.to_perm(x)), A.scipy() @ x, rtol=0, atol=1e-12)


# ------------------------------------------------------------ property tests
from hypothesis import given, settings, strategies as st


@st.composite
def sparse_patterns(draw):
    """Random square patterns (possibly nonsymmetric, with isolated rows and
    several components), stored as sorted CSR with the diagonal."""
    n = draw(st.integers(1, 60))
    density = draw(st.floats(0.0, 0.3))
    seed = draw(st.integers(0, 2**31 - 1))
    rng = np.random.default_rng(seed)
    M = sp.random(n, n, density=density, random_state=rng, format="csr")
    M = (M + sp.eye(n)).tocsr()
    M.sort_indices()
    M.data = rng.uniform(-1.0, 1.0, M.nnz)
    return M


@settings(max_examples=60, deadline=None)
@given(sparse_patterns())
def test_rcm_properties(M):
    """For any pattern: the ordering is a permutation; the permuted CSR is
    S[perm][:, perm] entry for entry; the reported bandwidth is the permuted
    matrix's; and every connected component of A + A^T occupies one
    contiguous index range (breadth-first numbering component by
    component)."""
    from scipy.sparse.csgraph import connected_components
    ddps = _lib()
    n = M.shape[0]
    perm = ddps.ddps_rcm(n, M.indptr, M.indices)
    assert np.array_equal(np.sort(perm), np.arange(n))
    rp, cl, vl = ddps.ddps_permute_csr(n, M.indptr, M.indices, M.data, perm)
    P = sp.csr_matrix((vl, cl, rp), shape=(n, n))
    E = M[perm][:, perm].tocsr()
    E.sort_indices()
    assert np.array_equal(P.indptr, E.indptr) and np.array_equal(P.indices, E.indices)
    assert np.array_equal(P.data, E.data)
    assert ddps.ddps_bandwidth(n, rp, cl) == _band(P)
    _, lab = connected_components(M + M.T, directed=False)
    lp = lab[perm]
    for c in np.unique(lp):
        idx = np.nonzero(lp == c)[0]
        assert idx[-1] - idx[0] + 1 == idx.size


@settings(max_examples=60, deadline=None)
@given(st.integers(1, 5000), st.integers(0, 600), st.integers(1, 64))
def test_partition_properties(n, b, p_max):
    """Equal slabs: they cover [0, n) in order, differ in size by at most
    one, number at most p_max, and are at least 2t rows (t = b rounded up to
    64, at least 64) whenever there is more than one."""
    ddps = _lib()
    part = ddps.ddps_partition_rows(n, b, p_max)
    p = len(part) - 1
    sizes = np.diff(part)
    t = max(64, -(-b // 64) * 64)
    assert part[0] == 0 and part[-1] == n and 1 <= p <= p_max
    assert sizes.min() >= 1 and sizes.max() - sizes.min() <= 1
    if p > 1:
        assert sizes.min() >= 2 * t

"""Seeded synthetic sparse systems for the DDPS solver.

These generators build the finite-difference / finite-volume matrices that
stand in for the paper's sparse test set (the paper solves systems from a
public sparse-matrix collection; none of those matrices is reproduced here).
They hold none of the solver's arithmetic: they only assemble CSR arrays,
row partitions and right-hand sides, and both the CPU oracle (through the
tests) and the GPU path consume their output.

Conventions (shared by every generator):
  * natural lexicographic ordering, x fastest, then y, then z;
  * homogeneous Dirichlet boundaries, eliminated (boundary nodes are not
    unknowns);
  * CSR with int64 row_ptr, int32 col (sorted ascending within a row) and
    float64 val.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "CSR", "stencil_csr", "convdiff2d", "convdiff3d", "aniso_diffusion2d",
    "vardiff_reaction3d", "implicit_euler_convdiff2d", "slab_partition",
    "uneven_partition", "random_banded", "random_geometric", "csr_matvec", "csr_to_dense",
]


class CSR:
    """Plain CSR container (n x n)."""

    def __init__(self, n, row_ptr, col, val):
        self.n = int(n)
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.val = np.ascontiguousarray(val, dtype=np.float64)

    @property
    def nnz(self):
        return int(self.row_ptr[-1])

    def bandwidth(self):
        rows = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))
        if rows.size == 0:
            return 0
        return int(np.max(np.abs(rows - self.col.astype(np.int64))))

    def scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))


def csr_matvec(A: CSR, x):
    """y = A x in float64 (x may be (n,) or (n, k))."""
    return A.scipy() @ x


def csr_to_dense(A: CSR):
    return A.scipy().toarray()


def stencil_csr(n, offsets, coeffs, valid):
    """Assemble CSR from per-row stencil coefficients.

    offsets: list of column offsets, ascending (so each row comes out sorted);
    coeffs: list of (n,) float64 arrays; valid: list of (n,) bool arrays.
    """
    order = np.argsort(offsets)
    offs = [offsets[i] for i in order]
    cs = np.stack([np.asarray(coeffs[i], dtype=np.float64) for i in order], axis=1)
    vs = np.stack([np.asarray(valid[i], dtype=bool) for i in order], axis=1)
    rows = np.arange(n, dtype=np.int64)
    cols = rows[:, None] + np.asarray(offs, dtype=np.int64)[None, :]
    counts = vs.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col = cols[vs].astype(np.int32)
    val = cs[vs]
    return CSR(n, row_ptr, col, val)


def _grid2(nx, ny):
    idx = np.arange(nx * ny, dtype=np.int64)
    return idx % nx, idx // nx


def _grid3(nx, ny, nz):
    idx = np.arange(nx * ny * nz, dtype=np.int64)
    return idx % nx, (idx // nx) % ny, idx // (nx * ny)


def _upwind(v, h, nu):
    """Coefficients (minus-neighbour, plus-neighbour, diagonal part) of
    -nu u'' + v u' on one axis, first-order upwind, rows scaled by h^2."""
    a = abs(v) * h
    lo = -nu - (a if v > 0 else 0.0)
    hi = -nu - (a if v < 0 else 0.0)
    return lo, hi, 2.0 * nu + a


def convdiff2d(nx, ny, vel, nu=1.0, h=None):
    """-nu Lap u + v . grad u on the unit square, 5-point, upwind, h^2-scaled."""
    h = 1.0 / (nx + 1) if h is None else h
    n = nx * ny
    ix, iy = _grid2(nx, ny)
    xl, xh, xd = _upwind(vel[0], h, nu)
    yl, yh, yd = _upwind(vel[1], h, nu)
    one = np.ones(n)
    offsets = [-nx, -1, 0, 1, nx]
    coeffs = [yl * one, xl * one, (xd + yd) * one, xh * one, yh * one]
    valid = [iy > 0, ix > 0, np.ones(n, bool), ix < nx - 1, iy < ny - 1]
    return stencil_csr(n, offsets, coeffs, valid)


def convdiff3d(nx, ny, nz, vel, nu=1.0, h=None):
    """-nu Lap u + v . grad u, 7-point, upwind, h^2-scaled, isotropic h."""
    h = 1.0 / (nx + 1) if h is None else h
    n = nx * ny * nz
    ix, iy, iz = _grid3(nx, ny, nz)
    xl, xh, xd = _upwind(vel[0], h, nu)
    yl, yh, yd = _upwind(vel[1], h, nu)
    zl, zh, zd = _upwind(vel[2], h, nu)
    one = np.ones(n)
    pl = nx * ny
    offsets = [-pl, -nx, -1, 0, 1, nx, pl]
    coeffs = [zl * one, yl * one, xl * one, (xd + yd + zd) * one, xh * one, yh * one, zh * one]
    valid = [iz > 0, iy > 0, ix > 0, np.ones(n, bool), ix < nx - 1, iy < ny - 1, iz < nz - 1]
    return stencil_csr(n, offsets, coeffs, valid)


def _harm(a, b):
    return 2.0 * a * b / (a + b)


def aniso_diffusion2d(nx, ny, eps_y, sigma, seed):
    """-div(a grad u) on cells, a ~ lognormal(0, sigma) per cell, harmonic face
    transmissibilities, y-faces scaled by eps_y, Dirichlet faces 2 a_cell."""
    rng = np.random.default_rng(seed)
    n = nx * ny
    a = rng.lognormal(0.0, sigma, n)
    ix, iy = _grid2(nx, ny)
    idx = np.arange(n)
    def nb(mask, off):
        j = np.where(mask, idx + off, idx)
        return a[j]
    tw = np.where(ix > 0, _harm(a, nb(ix > 0, -1)), 2.0 * a)
    te = np.where(ix < nx - 1, _harm(a, nb(ix < nx - 1, 1)), 2.0 * a)
    ts = eps_y * np.where(iy > 0, _harm(a, nb(iy > 0, -nx)), 2.0 * a)
    tn = eps_y * np.where(iy < ny - 1, _harm(a, nb(iy < ny - 1, nx)), 2.0 * a)
    diag = tw + te + ts + tn
    offsets = [-nx, -1, 0, 1, nx]
    coeffs = [-ts, -tw, diag, -te, -tn]
    valid = [iy > 0, ix > 0, np.ones(n, bool), ix < nx - 1, iy < ny - 1]
    return stencil_csr(n, offsets, coeffs, valid)


def vardiff_reaction3d(nx, ny, nz, sigma, reaction, seed, h=None):
    """-div(a grad u) + reaction u, 7-point cell scheme, a ~ lognormal(0, sigma),
    harmonic faces, Dirichlet faces 2 a_cell, rows scaled by h^2."""
    h = 1.0 / (nx + 1) if h is None else h
    rng = np.random.default_rng(seed)
    n = nx * ny * nz
    a = rng.lognormal(0.0, sigma, n)
    ix, iy, iz = _grid3(nx, ny, nz)
    idx = np.arange(n)
    pl = nx * ny
    def face(mask, off):
        j = np.where(mask, idx + off, idx)
        return np.where(mask, _harm(a, a[j]), 2.0 * a)
    t = {}
    t[-pl] = face(iz > 0, -pl)
    t[-nx] = face(iy > 0, -nx)
    t[-1] = face(ix > 0, -1)
    t[1] = face(ix < nx - 1, 1)
    t[nx] = face(iy < ny - 1, nx)
    t[pl] = face(iz < nz - 1, pl)
    diag = sum(t.values()) + reaction * h * h
    valid = {-pl: iz > 0, -nx: iy > 0, -1: ix > 0, 1: ix < nx - 1, nx: iy < ny - 1, pl: iz < nz - 1}
    offsets = [-pl, -nx, -1, 0, 1, nx, pl]
    coeffs = [(-t[o] if o != 0 else diag) for o in offsets]
    vmask = [(valid[o] if o != 0 else np.ones(n, bool)) for o in offsets]
    return stencil_csr(n, offsets, coeffs, vmask)


def implicit_euler_convdiff2d(nx, ny, dt, vel, nu=1.0):
    """A = I + dt * L_h with L_h = -nu Lap + v . grad (upwind, unscaled 1/h^2)."""
    h = 1.0 / (nx + 1)
    L = convdiff2d(nx, ny, vel, nu=nu, h=h)        # = h^2 * L_h
    val = L.val * (dt / (h * h))
    rows = np.repeat(np.arange(L.n, dtype=np.int64), np.diff(L.row_ptr))
    val = val + (rows == L.col.astype(np.int64)).astype(np.float64)
    return CSR(L.n, L.row_ptr, L.col, val)


def c4_velocity(step, magnitude=50.0, deg_per_step=1.2):
    th = np.deg2rad(deg_per_step * step)
    return (magnitude * np.cos(th), magnitude * np.sin(th)), th


def slab_partition(n_planes, planes_per_slab, plane):
    """part_ptr for equal slabs of whole grid planes (rows)."""
    assert n_planes % planes_per_slab == 0
    p = n_planes // planes_per_slab
    return (np.arange(p + 1, dtype=np.int64) * planes_per_slab * plane)


def uneven_partition(n_planes, plane, lo, hi, seed):
    """Slabs of whole planes with heights drawn from U{lo..hi}; the last slab
    takes the remaining planes so every height stays in [lo, hi]."""
    rng = np.random.default_rng(seed)
    heights = []
    rem = n_planes
    while rem > hi:
        top = min(hi, rem - lo)
        hgt = int(rng.integers(lo, top + 1))
        heights.append(hgt)
        rem -= hgt
    heights.append(rem)
    assert all(lo <= x <= hi for x in heights), heights
    ptr = np.zeros(len(heights) + 1, dtype=np.int64)
    np.cumsum(np.asarray(heights, dtype=np.int64) * plane, out=ptr[1:])
    return ptr


def random_banded(n, b, seed, density=0.6, margin=0.5, nonsym=True):
    """Random strictly row- and column-diagonally-dominant banded matrix with
    half-bandwidth exactly b (the two outermost diagonals are kept full so the
    band is attained)."""
    rng = np.random.default_rng(seed)
    offsets = [o for o in range(-b, b + 1)]
    coeffs, valid = [], []
    idx = np.arange(n)
    for o in offsets:
        ok = (idx + o >= 0) & (idx + o < n)
        if o == 0:
            coeffs.append(np.zeros(n))
        else:
            keep = ok & ((rng.random(n) < density) | (abs(o) == b))
            v = -rng.random(n) if nonsym else -np.ones(n)
            coeffs.append(np.where(keep, v, 0.0))
            ok = keep
        valid.append(ok)
    A = stencil_csr(n, offsets, coeffs, valid)
    # make it an M-matrix, dominant by rows and columns
    S = A.scipy().tocsr()
    rs = np.asarray(abs(S).sum(axis=1)).ravel()
    cs = np.asarray(abs(S).sum(axis=0)).ravel()
    d = np.maximum(rs, cs) + margin + rng.random(n)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(A.row_ptr))
    val = A.val.copy()
    dmask = rows == A.col.astype(np.int64)
    val[dmask] = d[rows[dmask]]
    return CSR(n, A.row_ptr, A.col, val)


def random_geometric(n, degree, seed, shuffle=True, sigma=None, margin=0.5, margin_rand=1.0):
    """A general (non-banded) sparse system: n points uniform in the unit
    square, each joined to the points within the radius that gives about
    `degree` neighbours on average; off-diagonal entries -(0.5 + u) with u ~
    U[0,1) (or, with sigma, -exp(sigma z) with z ~ N(0,1)) independently for
    a_ij and a_ji (nonsymmetric), diagonal = the larger of the absolute row
    and column sums + margin + margin_rand U[0,1): a strictly row- and
    column-diagonally-dominant M-matrix.  The rows come in a random order
    (shuffle) or sorted by x, then y."""
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(seed)
    pts = rng.random((n, 2))
    if not shuffle:
        pts = pts[np.lexsort((pts[:, 1], pts[:, 0]))]
    radius = np.sqrt(degree / (np.pi * n))
    pairs = cKDTree(pts).query_pairs(radius, output_type="ndarray")
    i = np.concatenate([pairs[:, 0], pairs[:, 1]])
    j = np.concatenate([pairs[:, 1], pairs[:, 0]])
    v = -(0.5 + rng.random(len(i))) if sigma is None else -np.exp(sigma * rng.standard_normal(len(i)))
    import scipy.sparse as sp
    M = sp.csr_matrix((v, (i, j)), shape=(n, n))
    rs = np.asarray(abs(M).sum(axis=1)).ravel()
    cs = np.asarray(abs(M).sum(axis=0)).ravel()
    M = (M + sp.diags(np.maximum(rs, cs) + margin + margin_rand * rng.random(n))).tocsr()
    M.sort_indices()
    return CSR(n, M.indptr, M.indices, M.data)

"""CPU oracle for DDPS (Manguoglu, "A domain-decomposing parallel sparse
linear system solver", arXiv 1008.1700).

TEST INFRASTRUCTURE ONLY.  Only the tests, the package's smoke entry point and
the benchmark's CPU-baseline leg may import this module.  It shares no code
with the GPU path and imports nothing from it: it is a plain, slow, float64
restatement of the method, written from the paper, against which the HIP
kernels are checked.

Stages (Section 3, Figures 1 and 2):
  1  split A = D + R by the given row partition              -> split()
  2  LU of every diagonal block A_ii (exact, banded LAPACK)   -> factor_block()
     or its incomplete LU with zero fill (L~_i U~_i)           -> factor_block_ilu0()
  3  drop columns of R_i with the delta rule                  -> kept_columns()
  4  spikes G_i = A_ii^{-1} R~_i(:, c_i)                      -> Preconditioner
  5  c = indices of the nonzero columns of G (ascending)      -> Preconditioner
  6  Krylov solve of Ax=f preconditioned by P = D~ + R~, where P z = y is
     6.1 g = D~^{-1} y; 6.2 G^ = I(c,c)+G(c,c), g^ = g(c); 6.3 G^ z^ = g^;
     6.4 z(c) = z^;    6.5 z = g - G z                        -> apply()

Readings of the paper taken here (each is listed in the design notes):
  * drop test: column k of R_i is dropped when ||R_i(:,k)||_inf <= delta *
    max_j ||R_i(:,j)||_inf, per block; so delta = 0 drops only all-zero
    columns and delta = 1 drops every column (block Jacobi).
  * c is kept in ascending global order (the order of the worked example).
  * 6.5 is applied to every row, including the rows in c.
  * the inner solve's tolerance is relative to ||g^||_2; the outer stopping
    test is ||f - Ax||_inf / ||f||_inf (x0 = 0, so this equals the paper's
    ||r_k||/||r_0|| form).
  * the outer Krylov method is preconditioned BiCGStab in the Templates form
    (P applied to the search directions, true-residual recurrences), with the
    convergence test also made after the first half of each iteration; an
    iteration that stops there counts as k - 0.5 (the convention of the
    paper's iteration tables).  Iterative refinement x += P^{-1}(f - Ax) is
    provided as the second outer method.
  * block factors come from LAPACK's partially pivoted band LU (an exact LU,
    as stage 2 asks).  The blocks of the PDE systems are diagonally dominant
    M-matrices, for which no row interchange happens, so there the factors
    are the unique unpivoted LU factors; factor_block(require_no_pivot=True)
    checks that before factors are compared entry by entry.
  * the incomplete factors of Section 3 (A~_ii = L~_i U~_i, the kind left
    open there) are read as ILU(0): L~_i unit lower and U~_i upper with the
    sparsity pattern of A_ii, so that (L~_i U~_i)(j,k) = a_jk wherever A_ii
    stores an entry; no pivoting, every row must store its diagonal.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
from scipy.linalg import lapack


# --------------------------------------------------------------------------
# Stage 1: A = D + R for the given partition (Section 3, Eqs. (1)-(2)).
# --------------------------------------------------------------------------
@dataclass
class Block:
    lo: int
    hi: int
    Aii: sp.csr_matrix           # n_i x n_i, local indices
    Ri: sp.csc_matrix            # n_i x n, global columns, block columns removed


def split(n, row_ptr, col, val, part_ptr):
    A = sp.csr_matrix((np.asarray(val, np.float64), np.asarray(col, np.int64),
                       np.asarray(row_ptr, np.int64)), shape=(n, n))
    blocks = []
    for i in range(len(part_ptr) - 1):
        lo, hi = int(part_ptr[i]), int(part_ptr[i + 1])
        rows = A[lo:hi, :].tocsc()
        Aii = rows[:, lo:hi].tocsr()
        Ri = rows.copy().tolil()
        Ri[:, lo:hi] = 0
        Ri = Ri.tocsc()
        Ri.eliminate_zeros()
        blocks.append(Block(lo, hi, Aii, Ri))
    return A, blocks


# --------------------------------------------------------------------------
# Stage 3: column dropping with tolerance delta (Section 3, dropping rule).
# --------------------------------------------------------------------------
def column_inf_norms(Ri):
    """||R_i(:,k)||_inf for every column k that has stored entries."""
    Ri = sp.csc_matrix(Ri)
    cols, norms = [], []
    for k in range(Ri.shape[1]):
        a, b = Ri.indptr[k], Ri.indptr[k + 1]
        if b > a:
            cols.append(k)
            norms.append(np.max(np.abs(Ri.data[a:b])))
    return np.asarray(cols, dtype=np.int64), np.asarray(norms, dtype=np.float64)


def kept_columns(Ri, delta):
    cols, norms = column_inf_norms(Ri)
    if cols.size == 0:
        return cols
    mu = norms.max()
    keep = norms > delta * mu
    return np.sort(cols[keep])


# --------------------------------------------------------------------------
# Stage 2: exact LU of each diagonal block (LAPACK band LU).
# --------------------------------------------------------------------------
@dataclass
class BandLU:
    lu: np.ndarray
    ipiv: np.ndarray
    kl: int
    ku: int
    n: int

    @property
    def pivoted(self):
        return not np.array_equal(self.ipiv, np.arange(self.n))


def block_bandwidth(Aii):
    coo = sp.coo_matrix(Aii)
    if coo.nnz == 0:
        return 0, 0
    d = coo.row.astype(np.int64) - coo.col.astype(np.int64)
    return int(max(d.max(), 0)), int(max((-d).max(), 0))


def factor_block(Aii, require_no_pivot=False):
    """Exact LU of A_ii in LAPACK band storage (partial pivoting).  With
    require_no_pivot the call fails if a row was swapped, so the factors are
    the unique unpivoted LU factors (for comparison with an unpivoted LU)."""
    n = Aii.shape[0]
    kl, ku = block_bandwidth(Aii)
    kl, ku = max(kl, 1), max(ku, 1)
    ab = np.zeros((2 * kl + ku + 1, n))
    coo = sp.coo_matrix(Aii)
    ab[kl + ku + coo.row - coo.col, coo.col] = coo.data
    lu, ipiv, info = lapack.dgbtrf(ab, kl, ku)
    if info != 0:
        raise np.linalg.LinAlgError(f"singular diagonal block (dgbtrf info={info})")
    fac = BandLU(lu, ipiv, kl, ku, n)
    if require_no_pivot and fac.pivoted:
        raise ValueError("band LU pivoted: the block is not suited to unpivoted LU")
    return fac


def block_solve(fac: BandLU, Y):
    Y = np.asarray(Y, dtype=np.float64)
    vec = Y.ndim == 1
    Y2 = Y.reshape(fac.n, -1)
    X, info = lapack.dgbtrs(fac.lu, fac.kl, fac.ku, Y2, fac.ipiv)
    assert info == 0
    return X.ravel() if vec else X


# --------------------------------------------------------------------------
# Stage 2 with incomplete factors (Section 3: D~ built from L~_i U~_i).
# --------------------------------------------------------------------------
@dataclass
class ILU0:
    L: sp.csr_matrix   # unit lower triangular (ones stored on the diagonal)
    U: sp.csr_matrix   # upper triangular, the pivots on its diagonal
    n: int


def factor_block_ilu0(Aii):
    """ILU(0) of A_ii: Gaussian elimination row by row (the IKJ order of
    Saad, Iterative Methods for Sparse Linear Systems, 2nd ed., Sec. 10.3.2)
    in which every update that would land outside the pattern of A_ii is
    discarded.  Row i, for each k < i that it stores, in increasing order:
    l_ik = a_ik / u_kk, then a_ij -= l_ik u_kj for each j > k stored in both
    row i and the finished row k.  Plain Python over the stored entries."""
    A = sp.csr_matrix(Aii, dtype=np.float64)
    A.sum_duplicates()
    A.sort_indices()
    n = A.shape[0]
    done = []                                  # finished rows: {col: value}
    for i in range(n):
        a, b = A.indptr[i], A.indptr[i + 1]
        row = {int(j): float(v) for j, v in zip(A.indices[a:b], A.data[a:b])}
        if i not in row:
            raise np.linalg.LinAlgError(f"row {i} stores no diagonal entry")
        for k in sorted(j for j in row if j < i):
            ukk = done[k][k]
            if ukk == 0.0:
                raise np.linalg.LinAlgError(f"zero pivot in row {k}")
            row[k] /= ukk
            lik = row[k]
            for j, ukj in done[k].items():
                if j > k and j in row:
                    row[j] -= lik * ukj
        if row[i] == 0.0:
            raise np.linalg.LinAlgError(f"zero pivot in row {i}")
        done.append(row)
    li, lj, lv, ui, uj, uv = [], [], [], [], [], []
    for i, row in enumerate(done):
        li.append(i); lj.append(i); lv.append(1.0)
        for j, v in row.items():
            if j < i:
                li.append(i); lj.append(j); lv.append(v)
            else:
                ui.append(i); uj.append(j); uv.append(v)
    L = sp.csr_matrix((lv, (li, lj)), shape=(n, n))
    U = sp.csr_matrix((uv, (ui, uj)), shape=(n, n))
    return ILU0(L, U, n)


def ilu0_solve(fac: ILU0, Y):
    """(L~ U~)^{-1} Y by the two sparse triangular solves."""
    import scipy.sparse.linalg as spla
    Y = np.asarray(Y, dtype=np.float64)
    W = spla.spsolve_triangular(fac.L, Y, lower=True, unit_diagonal=True)
    return spla.spsolve_triangular(fac.U, W, lower=False)


def solve_with(fac, Y):
    """D~_ii^{-1} Y for either kind of block factor."""
    return ilu0_solve(fac, Y) if isinstance(fac, ILU0) else block_solve(fac, Y)


def unit_lower_and_upper(fac: BandLU):
    """Dense L (unit lower) and U of the block, read out of the band storage."""
    n, kl, ku = fac.n, fac.kl, fac.ku
    L = np.eye(n)
    U = np.zeros((n, n))
    for j in range(n):
        for i in range(max(0, j - kl - ku), j + 1):
            U[i, j] = fac.lu[kl + ku + i - j, j]
        for i in range(j + 1, min(n, j + kl + 1)):
            L[i, j] = fac.lu[kl + ku + i - j, j]
    return L, U


# --------------------------------------------------------------------------
# BiCGStab (van der Vorst 1992; Templates, Barrett et al. 1994, Fig. 2.10).
# --------------------------------------------------------------------------
@dataclass
class KrylovInfo:
    iters: float = 0.0          # counted in half steps, as the paper's tables do
    relres: float = float("nan")
    converged: bool = False
    breakdown: bool = False
    history: list = field(default_factory=list)


def bicgstab(matvec, b, x0=None, tol=1e-10, maxit=1000, precond=None,
             norm=lambda v: np.linalg.norm(v, 2), ref=None):
    """Preconditioned BiCGStab in the Templates form; precond=None gives the
    unpreconditioned method.

    Convergence: norm(r)/ref <= tol, tested on s after the first half of an
    iteration (counted k - 0.5) and on r after the second half (counted k).
    `ref` defaults to norm(b).  On a breakdown (rho = 0, r~'v = 0 or
    omega = 0) the method restarts once with r~ = r; a second breakdown ends
    it with info.breakdown set."""
    M = (lambda v: v) if precond is None else precond
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    ref = norm(b) if ref is None else ref
    info = KrylovInfo()
    if ref == 0.0:
        info.relres, info.converged = 0.0, True
        return np.zeros_like(b), info
    r = b - matvec(x) if x0 is not None else b.copy()
    res = norm(r) / ref
    info.history.append(res)
    info.relres = res
    if res <= tol:
        info.converged = True
        return x, info
    rt = r.copy()
    restarts = 0
    fresh = True                       # next direction is p = r
    rho_old = alpha = omega = 1.0
    p = v = None

    def restart():
        nonlocal rt, fresh, restarts
        restarts += 1
        rt = r.copy()
        fresh = True
        return restarts <= 1

    i = 0
    while i < maxit:
        i += 1
        info.iters = float(i)
        rho = float(rt @ r)
        if rho == 0.0:
            if not restart():
                info.breakdown = True
                break
            rho = float(rt @ r)
        if fresh:
            p = r.copy()
            fresh = False
        else:
            beta = (rho / rho_old) * (alpha / omega)
            p = r + beta * (p - omega * v)
        ph = M(p)
        v = matvec(ph)
        rtv = float(rt @ v)
        if rtv == 0.0:
            if not restart():
                info.breakdown = True
                break
            continue
        alpha = rho / rtv
        s = r - alpha * v
        res = norm(s) / ref
        if res <= tol:
            x = x + alpha * ph
            info.iters = i - 0.5
            info.history.append(res)
            info.relres, info.converged = res, True
            return x, info
        sh = M(s)
        t = matvec(sh)
        tt = float(t @ t)
        omega = float(t @ s) / tt if tt != 0.0 else 0.0
        x = x + alpha * ph + omega * sh
        r = s - omega * t
        res = norm(r) / ref
        info.history.append(res)
        info.relres = res
        if res <= tol:
            info.converged = True
            return x, info
        if omega == 0.0 and not restart():
            info.breakdown = True
            break
        rho_old = rho
    return x, info


# --------------------------------------------------------------------------
# Stages 2-5 and the preconditioner application of Figure 2.
# --------------------------------------------------------------------------
class Preconditioner:
    """Stages 1-5 of Figure 1 (no right-hand side needed) and P z = y."""

    def __init__(self, n, row_ptr, col, val, part_ptr, delta=0.0, block_factor="lu"):
        self.n = int(n)
        self.part_ptr = np.asarray(part_ptr, dtype=np.int64)
        self.A, self.blocks = split(n, row_ptr, col, val, self.part_ptr)      # stage 1
        if block_factor not in ("lu", "ilu0"):
            raise ValueError(block_factor)
        fac = factor_block if block_factor == "lu" else factor_block_ilu0
        self.factors = [fac(b.Aii) for b in self.blocks]                       # stage 2
        self.c_i = [kept_columns(b.Ri, delta) for b in self.blocks]            # stage 3
        self.G = []                                                            # stage 4
        for b, fac, ci in zip(self.blocks, self.factors, self.c_i):
            Rt = b.Ri[:, ci].toarray() if ci.size else np.zeros((b.hi - b.lo, 0))
            self.G.append(solve_with(fac, Rt) if ci.size else Rt)
        nz = [ci[np.any(Gi != 0.0, axis=0)] if ci.size else ci                 # stage 5
              for ci, Gi in zip(self.c_i, self.G)]
        self.c = np.unique(np.concatenate(nz)) if nz else np.zeros(0, np.int64)
        self.m = int(self.c.size)
        self.pos = {int(k): j for j, k in enumerate(self.c)}
        self._Ghat = None

    # -- pieces of G^ --------------------------------------------------------
    def block_of(self, k):
        return int(np.searchsorted(self.part_ptr, k, side="right") - 1)

    def g_times(self, zc):
        """G z for z supported on c (values zc in c order): an n-vector."""
        out = np.zeros(self.n)
        for b, ci, Gi in zip(self.blocks, self.c_i, self.G):
            if ci.size:
                sel = np.array([self.pos.get(int(k), -1) for k in ci])
                zz = np.where(sel >= 0, zc[np.maximum(sel, 0)], 0.0)
                out[b.lo:b.hi] += Gi @ zz
        return out

    def ghat_matvec(self, zc):
        """G^ z^ = z^ + G(c, c) z^ (stage 6.2 operator)."""
        return zc + self.g_times(zc)[self.c]

    def local_matvec(self, zc):
        """The interface-local part N of G(c, c) applied to z^ (values on c).

        N keeps the entries of G(c, c) whose row and column lie at the same
        block boundary: rows in the upper half of block i with columns of
        block i-1, rows in the lower half of block i with columns of block
        i+1 (every block has at least twice as many rows as its coupling
        width, so the halves separate the two boundaries).  Used by the
        optional inner preconditioner z -> z - N z."""
        out = np.zeros(self.n)
        for b, ci, Gi in zip(self.blocks, self.c_i, self.G):
            if not ci.size:
                continue
            sel = np.array([self.pos.get(int(k), -1) for k in ci])
            zz = np.where(sel >= 0, zc[np.maximum(sel, 0)], 0.0)
            mid = (b.lo + b.hi) // 2
            left = ci < b.lo
            top = Gi[: mid - b.lo] @ np.where(left, zz, 0.0)
            bot = Gi[mid - b.lo:] @ np.where(~left, zz, 0.0)
            out[b.lo:mid] += top
            out[mid:b.hi] += bot
        return out[self.c]

    def ghat_dense(self):
        if self._Ghat is None:
            Gh = np.eye(self.m)
            for j in range(self.m):
                e = np.zeros(self.m); e[j] = 1.0
                Gh[:, j] = self.ghat_matvec(e)
            self._Ghat = Gh
        return self._Ghat

    # -- Figure 2 ------------------------------------------------------------
    def apply(self, y, reduced="dense", inner_tol=1e-12, inner_maxit=1000, zhat0=None, inner_prec=None,
              retrieval="spikes"):
        """Solve P z = y.  Returns z, and a dict with g, g^, z^ and the inner
        iteration record.  inner_prec="local" preconditions the inner
        BiCGStab with z -> z - N z (N = local_matvec), the first term of the
        Neumann series of the interface-local blocks of G^.

        retrieval="spikes" is step 6.5 as printed, z = g - G z with z(c) = z^.
        retrieval="resolve" is the same result written without the spikes:
        since G = D~^{-1} R~, g - G z = D~^{-1}(y - R~ z), one more block solve
        against y - R~ z (R~ has columns only in c, where z = z^)."""
        y = np.asarray(y, dtype=np.float64)
        g = np.empty(self.n)
        for b, fac in zip(self.blocks, self.factors):                         # 6.1
            g[b.lo:b.hi] = solve_with(fac, y[b.lo:b.hi])
        gh = g[self.c]                                                        # 6.2
        inner = KrylovInfo(converged=True, relres=0.0)
        if self.m == 0:
            zh = gh
        elif reduced == "dense":                                              # 6.3
            zh = np.linalg.solve(self.ghat_dense(), gh)
        else:
            M = (lambda v: v - self.local_matvec(v)) if inner_prec == "local" else None
            zh, inner = bicgstab(self.ghat_matvec, gh, x0=zhat0, tol=inner_tol,
                                 maxit=inner_maxit, precond=M)
        if retrieval == "spikes":
            z = g - self.g_times(zh)                                          # 6.4, 6.5
        elif retrieval == "resolve":
            zfull = np.zeros(self.n)                                          # 6.4
            zfull[self.c] = zh
            z = np.empty(self.n)
            for b, fac, ci in zip(self.blocks, self.factors, self.c_i):       # 6.5, re-solved
                rhs = y[b.lo:b.hi] - (b.Ri[:, ci] @ zfull[ci] if ci.size else 0.0)
                z[b.lo:b.hi] = solve_with(fac, rhs)
        else:
            raise ValueError(retrieval)
        return z, dict(g=g, ghat=gh, zhat=zh, inner=inner)


# --------------------------------------------------------------------------
# Stage 6: the outer layer.
# --------------------------------------------------------------------------
@dataclass
class SolveInfo:
    outer_iters: float = 0.0
    applications: int = 0
    inner_iters_total: float = 0.0
    relres_inf: float = float("nan")
    relres_2: float = float("nan")
    converged: bool = False


def solve(n, row_ptr, col, val, part_ptr, f, delta=0.0, tol=1e-10, outer="refine",
          outer_maxit=1000, reduced="dense", inner_tol=1e-12, inner_maxit=1000, prec=None,
          retrieval="spikes", norm="inf", block_factor="lu"):
    """DDPS for Ax = f.  outer in {'none', 'refine', 'bicgstab'}; the outer
    stopping test is ||f - Ax|| / ||f|| <= tol in the norm `norm` ('inf',
    the paper's choice in Section 4, or '2')."""
    P = prec if prec is not None else Preconditioner(n, row_ptr, col, val, part_ptr, delta, block_factor)
    A = P.A
    f = np.asarray(f, dtype=np.float64)
    info = SolveInfo()
    nrm = (lambda v: np.linalg.norm(v, np.inf)) if norm == "inf" else (lambda v: np.linalg.norm(v))
    fn = nrm(f)

    def papply(y):
        z, d = P.apply(y, reduced=reduced, inner_tol=inner_tol, inner_maxit=inner_maxit, retrieval=retrieval)
        info.applications += 1
        info.inner_iters_total += d["inner"].iters
        return z

    if outer == "none":
        x = papply(f)
    elif outer == "refine":
        x = np.zeros(n)
        r = f.copy()
        while nrm(r) > tol * fn and info.outer_iters < outer_maxit:
            x = x + papply(r)
            r = f - A @ x
            info.outer_iters += 1
    elif outer == "bicgstab":
        x, kinfo = bicgstab(lambda v: A @ v, f, tol=tol, maxit=outer_maxit, precond=papply, norm=nrm)
        info.outer_iters = kinfo.iters
    else:
        raise ValueError(outer)
    r = f - A @ x
    finf, f2 = np.linalg.norm(f, np.inf), np.linalg.norm(f)
    info.relres_inf = float(np.linalg.norm(r, np.inf) / finf) if finf else 0.0
    info.relres_2 = float(np.linalg.norm(r) / f2) if f2 else 0.0
    info.converged = (info.relres_inf if norm == "inf" else info.relres_2) <= tol
    return x, info, P


def direct_solve(A, f):
    """x = A^{-1} f by sparse LU with partial pivoting (SuperLU through
    scipy): the exact solution that every DDPS solve approaches (Section 3:
    with exact blocks and an exact reduced solve the method is a direct
    solver), for systems too large for the dense routines.  f may hold
    several columns."""
    import scipy.sparse.linalg as spla
    lu = spla.splu(sp.csc_matrix(A))
    return lu.solve(np.asarray(f, dtype=np.float64))


def hager_higham_cond1(solve, solveT, n, A1norm, iters=5):
    """Estimate of kappa_1(A) = ||A||_1 ||A^{-1}||_1 (Hager 1984; Higham 1988,
    Algorithm 2.1): a power-method style search for the column of A^{-1}
    with the largest 1-norm, from solves with A and A^T.  The estimate of
    ||A^{-1}||_1 is ||A^{-1} x||_1 for a unit-1-norm x, so it never exceeds
    the true value; it is usually exact or within a small factor.
    solve(v) = A^{-1} v, solveT(v) = A^{-T} v; A1norm = ||A||_1."""
    x = np.full(n, 1.0 / n)
    est = 0.0
    for _ in range(iters):
        y = solve(x)
        est_new = np.linalg.norm(y, 1)
        xi = np.sign(y); xi[xi == 0] = 1.0
        z = solveT(xi)
        j = int(np.argmax(np.abs(z)))
        if est_new <= est or np.abs(z[j]) <= z @ x:
            est = max(est, est_new)
            break
        est = est_new
        x = np.zeros(n); x[j] = 1.0
    return est * A1norm


def cond1_dense_estimate(A):
    """kappa_1 estimate of a (small) matrix through its dense LU: the
    Hager-Higham search above with LAPACK solves."""
    import scipy.linalg as sla
    Ad = A.toarray() if sp.issparse(A) else np.asarray(A, dtype=np.float64)
    lu = sla.lu_factor(Ad)
    n = Ad.shape[0]
    return hager_higham_cond1(lambda v: sla.lu_solve(lu, v), lambda v: sla.lu_solve(lu, v, trans=1), n,
                              np.linalg.norm(Ad, 1))


def mmatrix_kinf_bounds(A, y):
    """Two-sided bounds on kappa_inf(A) = ||A||_inf ||A^{-1}||_inf from any
    vector y > 0 (for example an approximate solution of A y = 1).

    For a Z-matrix A (off-diagonal entries <= 0), a vector y > 0 with A y > 0
    proves that A is a nonsingular M-matrix, so that A^{-1} >= 0 entrywise
    and ||A^{-1}||_inf = ||A^{-1} 1||_inf (Berman & Plemmons, Ch. 6).  With
    r = A y:  A^{-1} 1 <= y / min(r) gives the upper bound, and
    y = A^{-1} r gives ||A^{-1}||_inf >= ||y||_inf / ||r||_inf.  r is formed
    in float64 and widened by a bound on its rounding error
    (|fl(Ay) - Ay| <= gamma_k |A| |y|, k the longest row), so the bounds hold
    whatever y is.  Returns (lo, hi), or None if A is not a Z-matrix or the
    certificate fails (some entry of y or of A y not positive)."""
    A = sp.csr_matrix(A)
    y = np.asarray(y, dtype=np.float64)
    coo = A.tocoo()
    off = coo.row != coo.col
    if np.any(coo.data[off] > 0.0) or not np.all(y > 0.0):
        return None
    r = A @ y
    kmax = int(np.max(np.diff(A.indptr))) if A.nnz else 1
    u = np.finfo(np.float64).eps / 2
    gam = kmax * u / (1.0 - kmax * u)
    err = gam * (abs(A) @ np.abs(y))
    rmin = float(np.min(r - err))
    if not rmin > 0.0:
        return None
    ainf = float(np.max(abs(A) @ np.ones(A.shape[0])))
    ynorm = float(np.max(y))
    hi = ainf * ynorm / rmin
    lo = ainf * ynorm / float(np.max(np.abs(r) + err))
    return lo, hi

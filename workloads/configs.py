"""The five DDPS workloads (plus small test systems), built from pde.py.

Each builder returns a dict with:
  name, A (CSR), part_ptr (int64, p+1), x_star (n,) or (n, k), f = A x_star,
  grid (tuple), b (half-bandwidth), and workload-specific extras.

Sizes and seeds:
  c1: 64x64 2D upwind convection-diffusion, v=(20,20), p=4 slabs of 16 rows.
  c2: 32x32x512 3D upwind convection-diffusion, v=(1,1,10), h=1/33,
      p=64 slabs of 8 planes (block n 8192, band 1024).
  c3: 2048^2 anisotropic (eps_y=1e-3) lognormal(0,1.5) diffusion, uneven slabs
      of U{4..28} grid rows (seed 2), coefficients seed 1.
  c4: 1024^2 implicit-Euler convection-diffusion, dt=1e-3, |v|=50 rotating
      1.2 degrees per step, p=64; the matrix of step s is c4_matrix(s).
  c5: 40x40x4096 3D lognormal(0,1) diffusion + reaction 0.1, p=512 slabs of
      8 planes, 8 right-hand sides.
x_star ~ U[-1, 1] from default_rng(0) everywhere.
"""
from __future__ import annotations

import numpy as np

from . import pde


def _rhs(A, n, k=None, seed=0):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1.0, 1.0, n if k is None else (n, k))
    return x, pde.csr_matvec(A, x)


def c1():
    nx = ny = 64
    A = pde.convdiff2d(nx, ny, (20.0, 20.0))
    part = pde.slab_partition(ny, 16, nx)
    x, f = _rhs(A, A.n)
    return dict(name="c1", A=A, part_ptr=part, x_star=x, f=f, grid=(nx, ny), b=nx)


def c2(nz=512, planes_per_slab=8, nx=32, ny=32):
    A = pde.convdiff3d(nx, ny, nz, (1.0, 1.0, 10.0), h=1.0 / (nx + 1))
    part = pde.slab_partition(nz, planes_per_slab, nx * ny)
    x, f = _rhs(A, A.n)
    return dict(name="c2", A=A, part_ptr=part, x_star=x, f=f, grid=(nx, ny, nz), b=nx * ny)


def c3(nx=2048, ny=2048, lo=4, hi=28):
    A = pde.aniso_diffusion2d(nx, ny, 1e-3, 1.5, seed=1)
    part = pde.uneven_partition(ny, nx, lo, hi, seed=2)
    x, f = _rhs(A, A.n)
    return dict(name="c3", A=A, part_ptr=part, x_star=x, f=f, grid=(nx, ny), b=nx)


C4_DT = 1e-3
C4_STEPS = 300


def c4_matrix(step, nx=1024, ny=1024):
    """Matrix of implicit-Euler step `step` (1-based): velocity b_step."""
    vel, th = pde.c4_velocity(step)
    return pde.implicit_euler_convdiff2d(nx, ny, C4_DT, vel), th


def c4_kinds(A, nx):
    """Stencil position of every stored entry of a C4 matrix (0: -nx, 1: -1,
    2: diagonal, 3: +1, 4: +nx); the pattern is the same at every step."""
    rows = np.repeat(np.arange(A.n, dtype=np.int64), np.diff(A.row_ptr))
    off = A.col.astype(np.int64) - rows
    kinds = np.full(A.nnz, -1, dtype=np.int8)
    for k, o in enumerate([-nx, -1, 0, 1, nx]):
        kinds[off == o] = k
    assert np.all(kinds >= 0)
    return kinds


def c4_step_values(step, kinds, nx):
    """CSR values of c4_matrix(step) from the stencil positions (same result,
    without rebuilding the pattern)."""
    vel, th = pde.c4_velocity(step)
    h = 1.0 / (nx + 1)
    xl, xh, xd = pde._upwind(vel[0], h, 1.0)
    yl, yh, yd = pde._upwind(vel[1], h, 1.0)
    sc = C4_DT / (h * h)
    coef = np.array([yl * sc, xl * sc, (xd + yd) * sc + 1.0, xh * sc, yh * sc])
    return coef[kinds], th


def c4(nx=1024, ny=1024, p=64):
    A, th = c4_matrix(1, nx, ny)
    part = pde.slab_partition(ny, ny // p, nx)
    return dict(name="c4", A=A, part_ptr=part, x_star=None, f=None, grid=(nx, ny), b=nx,
                dt=C4_DT, steps=C4_STEPS, source=1.0)


def c5(nz=4096, nx=40, ny=40, planes_per_slab=8, k=8):
    A = pde.vardiff_reaction3d(nx, ny, nz, 1.0, 0.1, seed=1, h=1.0 / (nx + 1))
    part = pde.slab_partition(nz, planes_per_slab, nx * ny)
    x, f = _rhs(A, A.n, k=k)
    return dict(name="c5", A=A, part_ptr=part, x_star=x, f=f, grid=(nx, ny, nz), b=nx * ny)


def small_banded(n_blocks, block_sizes, b, seed):
    """Random diagonally dominant banded system with an explicit (possibly
    uneven) partition; used for ragged-size tests."""
    sizes = np.asarray(block_sizes, dtype=np.int64)
    assert sizes.size == n_blocks
    n = int(sizes.sum())
    A = pde.random_banded(n, b, seed)
    part = np.zeros(n_blocks + 1, dtype=np.int64)
    np.cumsum(sizes, out=part[1:])
    x, f = _rhs(A, n, seed=seed + 1000)
    return dict(name=f"banded{n}", A=A, part_ptr=part, x_star=x, f=f, b=b)


BUILDERS = {"c1": c1, "c2": c2, "c3": c3, "c4": c4, "c5": c5}

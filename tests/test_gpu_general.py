"""General (non-banded) sparse systems through the banded block path: a
shuffled random-geometric M-matrix is reordered by reverse Cuthill-McKee,
cut into equal slabs, and solved with exact coupling (delta 0, refinement)
and with dropped coupling columns (delta > 0, outer preconditioned
BiCGStab: the paper's experimental mode, Section 3 and Section 4).  Every
solution is mapped back to the original numbering and checked against the
oracle's sparse direct solve, and against the oracle's DDPS on the same
permuted matrix and partition."""
import numpy as np
import pytest

from tests.gpu_util import dev_vec, host, relerr, torch_cuda
from workloads import pde

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def system():
    from paper_1008_1700_amd import ddps
    A = pde.random_geometric(6000, 8, 5)
    gs = ddps.GeneralSystem(A.n, A.row_ptr, A.col, A.val, 8)
    xs = np.random.default_rng(6).uniform(-1, 1, A.n)
    f = A.scipy() @ xs
    return A, gs, xs, f


# The coupling entries of this matrix lie in [0.5, 1.5) in magnitude, so a
# column falls under the dropping rule only once delta exceeds 1/3.
@pytest.mark.parametrize("dtype,delta,outer", [("f64", 0.0, "refine"), ("f64", 0.4, "bicgstab"),
                                               ("f64", 0.6, "bicgstab"), ("bf16x3", 0.4, "bicgstab")])
def test_general_sparse_solve(system, dtype, delta, outer):
    from oracle import ddps_oracle as O
    from paper_1008_1700_amd import ddps
    torch_cuda()
    A, gs, xs, f = system
    p = len(gs.part_ptr) - 1
    assert p >= 4
    S = ddps.Solver(gs, gs.part_ptr, dtype=dtype, delta=delta, outer=outer, inner_tol=1e-10)
    try:
        S.factor()
        fp = gs.to_perm(f)
        x = dev_vec(np.zeros(A.n))
        rc, info = S.solve(dev_vec(fp), x, 1e-10)
        xg = gs.from_perm(host(x))
        r = f - A.scipy() @ xg
        relres = np.max(np.abs(r)) / np.max(np.abs(f))
        xd = O.direct_solve(A.scipy(), f)
        xo, oinfo, _ = O.solve(gs.n, gs.row_ptr, gs.col, gs.val, gs.part_ptr, fp, delta=delta, tol=1e-10,
                               outer=outer, inner_tol=1e-10)
        print(f"{dtype} delta {delta} {outer}: p {p}, b {gs.b}, GPU {info.as_dict()}; oracle outer "
              f"{oinfo.outer_iters}, host relres {relres:.3e}")
        assert rc == 0 and relres <= 1e-10
        assert relerr(xg, xd) <= 1e-8
        assert relerr(xg, gs.from_perm(xo)) <= 1e-8
        # the index set c of the kept coupling columns is the oracle's, and
        # dropping removes columns at these deltas
        torch = torch_cuda()
        m, t, _ = ddps.ddps_reduced_layout(S.h)
        c = torch.empty(m, dtype=torch.int64, device="cuda")
        mask = torch.empty(m, dtype=torch.float64, device="cuda")
        ddps.ddps_reduced_layout(S.h, c, mask)
        on = host(mask) > 0
        P = O.Preconditioner(gs.n, gs.row_ptr, gs.col, gs.val, gs.part_ptr, delta)
        assert np.array_equal(host(c)[on], P.c)
        if delta > 0:
            P0 = O.Preconditioner(gs.n, gs.row_ptr, gs.col, gs.val, gs.part_ptr, 0.0)
            assert len(P.c) < len(P0.c)
        print(f"kept coupling columns {len(P.c)}")
    finally:
        S.close()

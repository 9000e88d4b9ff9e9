"""Full-size time sequence on the GPU: 2D implicit-Euler upwind
convection-diffusion on 1024 x 1024 (dt = 1e-3, |v| = 50 rotating 1.2
degrees per step, source 1, u_0 = 0), p = 64 slabs of 16 grid rows, in the
precision the benchmark times (bf16x3 factors, FP64 refinement).

Every step refreshes the matrix values on the device, refactors and solves
u_n = A_n^{-1} (u_{n-1} + dt s).  At steps 1 and 200 the GPU's u_n is
compared with the exact solution of the same step's system, built from the
GPU's own u_{n-1} and solved on the host by the oracle's sparse direct
solve, and kappa_inf(A_n) is certified on the host to state the bound that
the residual implies."""
import numpy as np
import pytest

from tests.gpu_util import host, torch_cuda
from workloads import configs, pde

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(900)
def test_c4_steps_1_and_200_against_direct_solve():
    from oracle import ddps_oracle as O
    from paper_1008_1700_amd import ddps
    torch = torch_cuda()
    nx = ny = 1024
    p = 64
    A1, _ = configs.c4_matrix(1, nx, ny)
    part = pde.slab_partition(ny, ny // p, nx)
    kinds = configs.c4_kinds(A1, nx)
    S = ddps.Solver(A1, part, dtype="bf16x3", inner_tol=1e-6, outer="refine")
    checks = {1, 200}
    try:
        u = torch.zeros(A1.n, dtype=torch.float64, device="cuda")
        x = torch.zeros_like(u)
        f = torch.empty_like(u)
        for step in range(1, max(checks) + 1):
            val, _ = configs.c4_step_values(step, kinds, nx)
            S.val.copy_(torch.from_numpy(val))
            ddps.ddps_refactor_values(S.h, S.val)
            ddps.ddps_factor(S.h)
            torch.add(u, configs.C4_DT * 1.0, out=f)
            x.zero_()
            _, info = S.solve(f, x, 1e-10)
            assert info.relres_inf <= 1e-10
            if step in checks:
                A = pde.CSR(A1.n, A1.row_ptr, A1.col, val).scipy()
                fh = host(f)
                xh = host(x)
                ref = O.direct_solve(A, fh)
                err = np.max(np.abs(xh - ref)) / np.max(np.abs(ref))
                # kappa_inf(A_n) from a GPU solve of A_n y = 1, certified on the host
                ones = torch.ones_like(u)
                y = torch.zeros_like(u)
                S.solve(ones, y, 1e-10, check=False)
                kb = O.mmatrix_kinf_bounds(A, host(y))
                assert kb is not None
                relres = np.max(np.abs(fh - A @ xh)) / np.max(np.abs(fh))
                print(f"step {step}: {info.as_dict()}; kappa_inf in [{kb[0]:.4g}, {kb[1]:.4g}]; "
                      f"host relres {relres:.3e}; max error vs direct solve {err:.3e}")
                # both solutions are within kappa_inf * tol of the exact one
                assert err <= 2.0 * kb[1] * 1e-10 + 1e-14
                assert err <= 1e-8
            u, x = x, u
    finally:
        S.close()

"""Handle-free residual norms (the outer stopping test's quantities) on the
GPU against r = f - A x formed on the CPU."""
import numpy as np
import pytest

from tests.gpu_util import torch_cuda
from workloads import configs

pytestmark = pytest.mark.gpu


def _csr_dev(A):
    torch = torch_cuda()
    return (torch.from_numpy(A.row_ptr).cuda(), torch.from_numpy(A.col).cuda(),
            torch.from_numpy(A.val).cuda())


@pytest.mark.parametrize("k", [1, 3, 8])
def test_residual_norms_match_cpu(k):
    torch = torch_cuda()
    from paper_1008_1700_amd import ddps
    d = configs.c1()
    A = d["A"]
    rng = np.random.default_rng(k)
    X = rng.uniform(-1, 1, (k, A.n))
    F = rng.uniform(-1, 1, (k, A.n))
    rp, cl, vl = _csr_dev(A)
    Xd = torch.from_numpy(X).cuda()
    Fd = torch.from_numpy(F).cuda()
    Rd = torch.zeros_like(Fd)
    out = ddps.ddps_residual_norms(rp, cl, vl, Xd, Fd, Rd)
    Rc = F - (A.scipy() @ X.T).T
    assert np.allclose(Rd.cpu().numpy(), Rc, rtol=0, atol=1e-13 * np.abs(Rc).max())
    exp = np.stack([np.abs(Rc).max(axis=1), np.linalg.norm(Rc, axis=1), np.abs(F).max(axis=1),
                    np.linalg.norm(F, axis=1)], axis=1)
    assert np.allclose(out, exp, rtol=1e-12, atol=0)
    # a NULL residual output gives the same norms
    out2 = ddps.ddps_residual_norms(rp, cl, vl, Xd, Fd, None)
    assert np.array_equal(out, out2)

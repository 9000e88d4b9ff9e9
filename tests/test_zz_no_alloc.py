"""The allocation-free residual entry point against the allocating one,
through the C ABI: same kernels, so the outputs must be identical, on two
calls in a row, the second smaller than the first."""
import ctypes

import numpy as np
import pytest

from tests.gpu_util import torch_cuda
from workloads import configs

pytestmark = pytest.mark.gpu

_I64, _I32, _P, _D = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_double
_ARGS = [_I64, _I32, _P, _P, _P, _P, _I64, _P, _I64, _P, _I64, ctypes.POINTER(_D), _P]


def _fn(name):
    from paper_1008_1700_amd import ddps
    f = getattr(ddps.lib(), name)
    f.restype = _I32
    f.argtypes = _ARGS
    return f


def _call(f, A, X, F, R):
    k, n = F.shape
    out = np.full(4 * k, np.nan)
    torch = torch_cuda()
    rp = torch.from_numpy(A.row_ptr).cuda()
    cl = torch.from_numpy(A.col).cuda()
    vl = torch.from_numpy(A.val).cuda()
    torch.cuda.synchronize()
    rc = f(n, k, rp.data_ptr(), cl.data_ptr(), vl.data_ptr(), X.data_ptr(), n, F.data_ptr(), n,
           R.data_ptr(), n, out.ctypes.data_as(ctypes.POINTER(_D)), None)
    return rc, out


def test_noalloc_matches_allocating_entry_point_twice():
    torch = torch_cuda()
    alloc = _fn("ddps_residual_norms")
    noalloc = _fn("ddps_residual_norms_noalloc")
    cases = [(configs.c1()["A"], 7, 1), (configs.small_banded(3, [300, 340, 280], 40, 11)["A"], 2, 2)]
    for A, k, seed in cases:
        rng = np.random.default_rng(seed)
        X = torch.from_numpy(rng.uniform(-1, 1, (k, A.n))).cuda()
        F = torch.from_numpy(rng.uniform(-1, 1, (k, A.n))).cuda()
        R1 = torch.full_like(F, np.nan)
        R2 = torch.full_like(F, np.nan)
        rc1, n1 = _call(alloc, A, X, F, R1)
        rc2, n2 = _call(noalloc, A, X, F, R2)
        assert rc1 == 0 and rc2 == 0
        assert np.array_equal(n1, n2)
        assert torch.equal(R1, R2)
        Rc = F.cpu().numpy() - (A.scipy() @ X.cpu().numpy().T).T
        assert np.allclose(R2.cpu().numpy(), Rc, rtol=0, atol=1e-13 * np.abs(Rc).max())


def test_noalloc_rejects_more_columns_than_its_scratch_holds():
    torch = torch_cuda()
    noalloc = _fn("ddps_residual_norms_noalloc")
    A = configs.c1()["A"]
    X = torch.zeros(9, A.n, dtype=torch.float64, device="cuda")
    F = torch.zeros(9, A.n, dtype=torch.float64, device="cuda")
    R = torch.zeros(9, A.n, dtype=torch.float64, device="cuda")
    rc, _ = _call(noalloc, A, X, F, R)
    assert rc == -1

"""Helpers for GPU parity tests: build systems, run the HIP path, run the
oracle on the same inputs.  Nothing here computes the method."""
import numpy as np

from workloads import configs, pde


def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def dev_vec(x):
    torch = torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def make_solver(d, **kw):
    from paper_1008_1700_amd import ddps
    return ddps.Solver(d["A"], d["part_ptr"], **kw)


def relerr(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def oracle_prec(d, delta=0.0):
    from oracle import ddps_oracle as O
    A = d["A"]
    return O.Preconditioner(A.n, A.row_ptr, A.col, A.val, d["part_ptr"], delta)


def maxrel(a, b):
    """Element-wise bar: max |a - b| over max |b| (every entry is held to the
    largest one's scale, so a wrong small entry is not averaged away)."""
    mb = np.max(np.abs(b)) if np.size(b) else 0.0
    return float(np.max(np.abs(a - b)) / (mb if mb > 0 else 1.0)) if np.size(b) else 0.0

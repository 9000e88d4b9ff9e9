"""Python binding of the DDPS C ABI (include/ddps.h).

Argument marshalling only: every step of the solver runs in the HIP library
libddps.so.  torch supplies device memory (tensor data pointers) and the
stream; nothing here computes.  The library must have been built
(paper_1008_1700_amd.build); loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libddps.so")

F64, F32, BF16X3, BF16 = 0, 1, 2, 3
DTYPES = {"f64": F64, "f32": F32, "bf16x3": BF16X3, "bf16": BF16}
STATUS = {0: "DDPS_OK", -1: "DDPS_E_ARG", -2: "DDPS_E_NOMEM", -3: "DDPS_E_NOCONV", -4: "DDPS_E_SINGULAR",
          -5: "DDPS_E_BREAKDOWN", -6: "DDPS_E_STATE", -7: "DDPS_E_HIP"}
TIMING_KINDS = {"gemm": 0, "panel": 1, "sweep": 2, "reduced": 3, "retrieval": 4, "csr": 5, "reduced_factor": 6}


class DDPSError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {STATUS.get(code, code)}")


class ddps_options(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_int32),
        ("drop_delta", ctypes.c_double),
        ("factor_dtype", ctypes.c_int32),
        ("inner_tol", ctypes.c_double),
        ("inner_maxit", ctypes.c_int32),
        ("outer_maxit", ctypes.c_int32),
        ("outer_method", ctypes.c_int32),
        ("guess", ctypes.c_int32),
        ("use_x0", ctypes.c_int32),
        ("max_rhs", ctypes.c_int32),
        ("mem_budget", ctypes.c_size_t),
        ("stream", ctypes.c_void_p),
        ("factor_streams", ctypes.c_int32),
        ("factor_graph", ctypes.c_int32),
        ("inner_prec", ctypes.c_int32),
        ("retrieval", ctypes.c_int32),
        ("norm", ctypes.c_int32),
        ("work_slots", ctypes.c_int32),
        ("reduced_solve", ctypes.c_int32),
        ("loosen_ratio", ctypes.c_double),
        ("gemv_sums", ctypes.c_int32),
        ("block_factor", ctypes.c_int32),
    ]


class ddps_info(ctypes.Structure):
    _fields_ = [
        ("outer_iters", ctypes.c_double),
        ("inner_iters_avg", ctypes.c_double),
        ("inner_iters_total", ctypes.c_int64),
        ("applications", ctypes.c_int32),
        ("relres_inf", ctypes.c_double),
        ("relres_2", ctypes.c_double),
        ("t_setup_ms", ctypes.c_double),
        ("t_factor_ms", ctypes.c_double),
        ("t_solve_ms", ctypes.c_double),
        ("bad_block", ctypes.c_int32),
        ("bad_row", ctypes.c_int64),
        ("loosened_steps", ctypes.c_int32),
        ("undone_steps", ctypes.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_D = ctypes.c_double

_SIGS = {
    "ddps_default_options": (None, [ctypes.POINTER(ddps_options)]),
    "ddps_setup": (_I32, [ctypes.POINTER(_P), _I64, _I32, ctypes.POINTER(_I64), _P, _P, _P, _I64,
                          ctypes.POINTER(ddps_options)]),
    "ddps_factor": (_I32, [_P]),
    "ddps_refactor_values": (_I32, [_P, _P]),
    "ddps_solve": (_I32, [_P, _P, _P, _D, ctypes.POINTER(ddps_info)]),
    "ddps_solve_many": (_I32, [_P, _I32, _P, _I64, _P, _I64, _D, ctypes.POINTER(ddps_info)]),
    "ddps_set_guess": (_I32, [_P, _P, _I32]),
    "ddps_reduced_layout": (_I32, [_P, ctypes.POINTER(_I64), _P, _P, ctypes.POINTER(_I32),
                                   ctypes.POINTER(_I32)]),
    "ddps_last_reduced": (_I32, [_P, _P, _P]),
    "ddps_apply_preconditioner": (_I32, [_P, _I32, _P, _P, _P, _P, ctypes.POINTER(_D)]),
    "ddps_block_solve": (_I32, [_P, _I32, _P, _P]),
    "ddps_reduced_matvec": (_I32, [_P, _I32, _P, _P]),
    "ddps_get_tile": (_I32, [_P, _I32, _I32, _I32, _P]),
    "ddps_get_spikes": (_I32, [_P, _I32, _P]),
    "ddps_block_shape": (_I32, [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "ddps_last_singular": (_I32, [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I64)]),
    "ddps_set_execution": (_I32, [_P, _I32, _I32, _I32]),
    "ddps_autotune": (_I32, [_P, ctypes.c_char_p, _D, ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                             ctypes.POINTER(_D)]),
    "ddps_timing_enable": (_I32, [_P, _I32, _I32]),
    "ddps_timing_read": (_I32, [_P, _I32, ctypes.POINTER(_I64), ctypes.POINTER(_D), ctypes.POINTER(_D),
                                ctypes.POINTER(_D)]),
    "ddps_reduced_rhs": (_I32, [_P, _I32, _P, _P]),
    "ddps_reduced_restrict": (_I32, [_P, _I32, _P, _P]),
    "ddps_reduced_residual": (_I32, [_P, _I32, _P, _P, ctypes.POINTER(_D), _P]),
    "ddps_guess_features": (_I32, [_P, _I32, _P, _P, _D, _D, _I32, _P, _P]),
    "ddps_guess_compose": (_I32, [_P, _I32, _P, _P, _P, _P]),
    "ddps_guess_target": (_I32, [_P, _I32, _P, _P, _P, _P]),
    "ddps_mlp_create": (_I32, [ctypes.POINTER(_P), _I32, _I32, _I32, _I32, ctypes.c_uint64, _P]),
    "ddps_mlp_param_count": (_I64, [_P]),
    "ddps_mlp_set_params": (_I32, [_P, _P]),
    "ddps_mlp_get_params": (_I32, [_P, _P]),
    "ddps_mlp_forward": (_I32, [_P, _I32, _P, _P]),
    "ddps_mlp_train_step": (_I32, [_P, _I32, _P, _P, ctypes.c_float, ctypes.POINTER(_D)]),
    "ddps_mlp_gradients": (_I32, [_P, _I32, _P, _P, _P, ctypes.POINTER(_D)]),
    "ddps_mlp_destroy": (None, [_P]),
    "ddps_memory": (_I32, [_P, ctypes.POINTER(ctypes.c_size_t)]),
    "ddps_set_guess_model": (_I32, [_P, _P]),
    "ddps_guess_counts": (_I32, [_P, ctypes.POINTER(_I64)]),
    "ddps_guess_trial": (_I32, [_P, ctypes.POINTER(_I64), ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I32)]),
    "ddps_rcm": (_I32, [_I64, _P, _P, _P]),
    "ddps_last_hip_error": (ctypes.c_char_p, []),
    "ddps_bandwidth": (_I32, [_I64, _P, _P, ctypes.POINTER(_I64)]),
    "ddps_permute_csr": (_I32, [_I64, _P, _P, _P, _P, _P, _P, _P]),
    "ddps_partition_rows": (_I32, [_I64, _I64, _I32, _P, ctypes.POINTER(_I32)]),
    "ddps_residual_norms": (_I32, [_I64, _I32, _P, _P, _P, _P, _I64, _P, _I64, _P, _I64, ctypes.POINTER(_D), _P]),
    "ddps_residual_norms_noalloc": (_I32, [_I64, _I32, _P, _P, _P, _P, _I64, _P, _I64, _P, _I64, ctypes.POINTER(_D),
                                           _P]),
    "ddps_destroy": (None, [_P]),
    "ddps_status_string": (ctypes.c_char_p, [_I32]),
}


def lib():
    """Load libddps.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_1008_1700_amd.build")
        # torch first: the library then binds to the HIP runtime torch has
        # loaded, so that one runtime (one device context) serves both, in
        # whatever order the caller touches them
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def _chk(code, where):
    if code != 0:
        if STATUS.get(code) == "DDPS_E_HIP":
            where = f"{where} ({lib().ddps_last_hip_error().decode()})"
        raise DDPSError(code, where)


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _need_cuda(t, dtype, name):
    import torch
    if t is None:
        return
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor")


# ------------------------------------------------------------------ C names
def ddps_default_options():
    o = ddps_options()
    lib().ddps_default_options(ctypes.byref(o))
    return o


def ddps_setup(n, p, part_ptr, row_ptr, col, val, opt=None):
    import torch
    part = np.ascontiguousarray(np.asarray(part_ptr, dtype=np.int64))
    _need_cuda(row_ptr, torch.int64, "row_ptr")
    _need_cuda(col, torch.int32, "col")
    _need_cuda(val, torch.float64, "val")
    h = ctypes.c_void_p()
    o = opt if opt is not None else ddps_default_options()
    rc = lib().ddps_setup(ctypes.byref(h), int(n), int(p),
                          part.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                          _ptr(row_ptr), _ptr(col), _ptr(val), int(val.numel()), ctypes.byref(o))
    _chk(rc, "ddps_setup")
    return h


def ddps_factor(h):
    rc = lib().ddps_factor(h)
    _chk(rc, "ddps_factor")


def ddps_refactor_values(h, val):
    _chk(lib().ddps_refactor_values(h, _ptr(val)), "ddps_refactor_values")


def ddps_solve(h, f, x, tol, check=True):
    info = ddps_info()
    rc = lib().ddps_solve(h, _ptr(f), _ptr(x), float(tol), ctypes.byref(info))
    if check:
        _chk(rc, "ddps_solve")
    return rc, info


def ddps_solve_many(h, F, X, tol, check=True):
    """F, X: (k, n) contiguous float64 CUDA tensors (row j = right-hand side j)."""
    k, n = F.shape
    info = ddps_info()
    rc = lib().ddps_solve_many(h, int(k), _ptr(F), int(n), _ptr(X), int(n), float(tol), ctypes.byref(info))
    if check:
        _chk(rc, "ddps_solve_many")
    return rc, info


def ddps_set_guess(h, zhat0, k=1):
    _chk(lib().ddps_set_guess(h, _ptr(zhat0), int(k if zhat0 is not None else 0)), "ddps_set_guess")


def ddps_reduced_layout(h, c=None, mask=None):
    m = ctypes.c_int64()
    t = ctypes.c_int32()
    b = ctypes.c_int32()
    _chk(lib().ddps_reduced_layout(h, ctypes.byref(m), _ptr(c), _ptr(mask), ctypes.byref(t), ctypes.byref(b)),
         "ddps_reduced_layout")
    return m.value, t.value, b.value


def ddps_last_reduced(h, ghat=None, zhat=None):
    _chk(lib().ddps_last_reduced(h, _ptr(ghat), _ptr(zhat)), "ddps_last_reduced")


def ddps_apply_preconditioner(h, k, y, z, ghat=None, zhat=None):
    its = (ctypes.c_double * 8)()
    rc = lib().ddps_apply_preconditioner(h, int(k), _ptr(y), _ptr(z), _ptr(ghat), _ptr(zhat), its)
    _chk(rc, "ddps_apply_preconditioner")
    return [its[j] for j in range(k)]


def ddps_block_solve(h, k, y, g):
    _chk(lib().ddps_block_solve(h, int(k), _ptr(y), _ptr(g)), "ddps_block_solve")


def ddps_reduced_matvec(h, k, x, v):
    _chk(lib().ddps_reduced_matvec(h, int(k), _ptr(x), _ptr(v)), "ddps_reduced_matvec")


def ddps_get_tile(h, blk, k, which, dst):
    _chk(lib().ddps_get_tile(h, int(blk), int(k), int(which), _ptr(dst)), "ddps_get_tile")


def ddps_get_spikes(h, blk, dst):
    _chk(lib().ddps_get_spikes(h, int(blk), _ptr(dst)), "ddps_get_spikes")


def ddps_block_shape(h, p):
    t = ctypes.c_int32()
    tiles = (ctypes.c_int32 * p)()
    pads = (ctypes.c_int32 * p)()
    _chk(lib().ddps_block_shape(h, ctypes.byref(t), tiles, pads), "ddps_block_shape")
    return t.value, list(tiles), list(pads)


def ddps_last_singular(h):
    b = ctypes.c_int32()
    r = ctypes.c_int64()
    _chk(lib().ddps_last_singular(h, ctypes.byref(b), ctypes.byref(r)), "ddps_last_singular")
    return b.value, r.value


def ddps_set_execution(h, streams=0, graph=False, tile_policy=0):
    _chk(lib().ddps_set_execution(h, int(streams), 1 if graph else 0, int(tile_policy)), "ddps_set_execution")


def ddps_autotune(h, cache_path=None, budget_s=0.0):
    s = ctypes.c_int32()
    q = ctypes.c_int32()
    ms = ctypes.c_double()
    path = None if cache_path is None else os.fsencode(cache_path)
    _chk(lib().ddps_autotune(h, path, float(budget_s), ctypes.byref(s), ctypes.byref(q), ctypes.byref(ms)),
         "ddps_autotune")
    return dict(streams=s.value, tile_policy=q.value, factor_ms=ms.value)


def ddps_timing_enable(h, kind, on=True):
    _chk(lib().ddps_timing_enable(h, TIMING_KINDS.get(kind, kind), 1 if on else 0), "ddps_timing_enable")


def ddps_timing_read(h, kind):
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    fl = ctypes.c_double()
    by = ctypes.c_double()
    _chk(lib().ddps_timing_read(h, TIMING_KINDS.get(kind, kind), ctypes.byref(n), ctypes.byref(ms),
                                ctypes.byref(fl), ctypes.byref(by)), "ddps_timing_read")
    return dict(launches=n.value, ms=ms.value, flops=fl.value, bytes=by.value)


def ddps_reduced_rhs(h, k, y, ghat):
    _chk(lib().ddps_reduced_rhs(h, int(k), _ptr(y), _ptr(ghat)), "ddps_reduced_rhs")


def ddps_reduced_restrict(h, k, x, z):
    _chk(lib().ddps_reduced_restrict(h, int(k), _ptr(x), _ptr(z)), "ddps_reduced_restrict")


def ddps_reduced_residual(h, k, ghat, z, rvec=None):
    res = (ctypes.c_double * max(1, k))()
    _chk(lib().ddps_reduced_residual(h, int(k), _ptr(ghat), _ptr(z), res, _ptr(rvec)), "ddps_reduced_residual")
    return [res[j] for j in range(k)]


def ddps_guess_features(h, k, r, zprev, cos_t, sin_t, d_in, X, scale):
    _chk(lib().ddps_guess_features(h, int(k), _ptr(r), _ptr(zprev), float(cos_t), float(sin_t), int(d_in),
                                   _ptr(X), _ptr(scale)), "ddps_guess_features")


def ddps_guess_compose(h, k, zprev, Y, scale, zhat0):
    _chk(lib().ddps_guess_compose(h, int(k), _ptr(zprev), _ptr(Y), _ptr(scale), _ptr(zhat0)),
         "ddps_guess_compose")


def ddps_guess_target(h, k, zhat, zprev, scale, T):
    _chk(lib().ddps_guess_target(h, int(k), _ptr(zhat), _ptr(zprev), _ptr(scale), _ptr(T)), "ddps_guess_target")


def ddps_mlp_create(d_in, hidden, d_out, max_batch, seed=0, stream=None):
    m = ctypes.c_void_p()
    _chk(lib().ddps_mlp_create(ctypes.byref(m), int(d_in), int(hidden), int(d_out), int(max_batch),
                               ctypes.c_uint64(seed), ctypes.c_void_p(stream or 0)), "ddps_mlp_create")
    return m


def ddps_mlp_param_count(m):
    return int(lib().ddps_mlp_param_count(m))


def ddps_mlp_set_params(m, params):
    a = np.ascontiguousarray(params, dtype=np.float32)
    _chk(lib().ddps_mlp_set_params(m, a.ctypes.data_as(ctypes.c_void_p)), "ddps_mlp_set_params")


def ddps_mlp_get_params(m):
    a = np.empty(ddps_mlp_param_count(m), dtype=np.float32)
    _chk(lib().ddps_mlp_get_params(m, a.ctypes.data_as(ctypes.c_void_p)), "ddps_mlp_get_params")
    return a


def ddps_mlp_forward(m, batch, X, Y):
    _chk(lib().ddps_mlp_forward(m, int(batch), _ptr(X), _ptr(Y)), "ddps_mlp_forward")


def ddps_mlp_train_step(m, batch, X, T, lr, want_loss=True):
    loss = ctypes.c_double()
    _chk(lib().ddps_mlp_train_step(m, int(batch), _ptr(X), _ptr(T), ctypes.c_float(lr),
                                   ctypes.byref(loss) if want_loss else None), "ddps_mlp_train_step")
    return loss.value if want_loss else None


def ddps_mlp_gradients(m, batch, X, T):
    g = np.empty(ddps_mlp_param_count(m), dtype=np.float32)
    loss = ctypes.c_double()
    _chk(lib().ddps_mlp_gradients(m, int(batch), _ptr(X), _ptr(T), g.ctypes.data_as(ctypes.c_void_p),
                                  ctypes.byref(loss)), "ddps_mlp_gradients")
    return g, loss.value


def ddps_mlp_destroy(m):
    if m:
        lib().ddps_mlp_destroy(m)


def ddps_residual_norms(row_ptr, col, val, X, F, R=None, stream=None):
    """X, F (and R): (k, n) contiguous float64 CUDA tensors (row j = column j).
    Returns a (k, 4) array: ||r||_inf, ||r||_2, ||f||_inf, ||f||_2."""
    k, n = F.shape
    out = np.zeros(4 * k)
    rc = lib().ddps_residual_norms(int(n), int(k), _ptr(row_ptr), _ptr(col), _ptr(val), _ptr(X), int(n), _ptr(F),
                                   int(n), _ptr(R), int(n), out.ctypes.data_as(ctypes.POINTER(_D)),
                                   ctypes.c_void_p(stream))
    _chk(rc, "ddps_residual_norms")
    return out.reshape(k, 4)


def ddps_set_guess_model(h, net):
    _chk(lib().ddps_set_guess_model(h, net), "ddps_set_guess_model")


def ddps_guess_counts(h):
    c = (_I64 * 4)()
    _chk(lib().ddps_guess_counts(h, c), "ddps_guess_counts")
    return dict(zero=c[0], ghat=c[1], learned=c[2], retired=c[3])


def ddps_guess_trial(h):
    n = (_I64 * 2)()
    mean = (ctypes.c_double * 2)()
    st = _I32()
    _chk(lib().ddps_guess_trial(h, n, mean, ctypes.byref(st)), "ddps_guess_trial")
    return dict(solves_without=n[0], solves_with=n[1], mean_iters_without=mean[0], mean_iters_with=mean[1],
                state={0: "running", 1: "kept", 2: "retired"}[st.value])


def _host(a, dtype):
    import numpy as np
    return np.ascontiguousarray(a, dtype=dtype)


def ddps_rcm(n, row_ptr, col):
    """Reverse Cuthill-McKee permutation (host arrays): new row i = old row perm[i]."""
    import numpy as np
    rp, c = _host(row_ptr, np.int64), _host(col, np.int32)
    perm = np.empty(n, dtype=np.int64)
    _chk(lib().ddps_rcm(int(n), rp.ctypes.data, c.ctypes.data, perm.ctypes.data), "ddps_rcm")
    return perm


def ddps_bandwidth(n, row_ptr, col):
    import numpy as np
    rp, c = _host(row_ptr, np.int64), _host(col, np.int32)
    b = _I64()
    _chk(lib().ddps_bandwidth(int(n), rp.ctypes.data, c.ctypes.data, ctypes.byref(b)), "ddps_bandwidth")
    return b.value


def ddps_permute_csr(n, row_ptr, col, val, perm):
    """B = P A P^T (host arrays); returns (row_ptr, col, val) of B."""
    import numpy as np
    rp, c, p = _host(row_ptr, np.int64), _host(col, np.int32), _host(perm, np.int64)
    v = None if val is None else _host(val, np.float64)
    orp = np.empty(n + 1, dtype=np.int64)
    oc = np.empty(len(c), dtype=np.int32)
    ov = None if v is None else np.empty(len(v), dtype=np.float64)
    _chk(lib().ddps_permute_csr(int(n), rp.ctypes.data, c.ctypes.data, None if v is None else v.ctypes.data,
                                p.ctypes.data, orp.ctypes.data, oc.ctypes.data, None if ov is None else ov.ctypes.data),
         "ddps_permute_csr")
    return orp, oc, ov


def ddps_partition_rows(n, b, p_max):
    import numpy as np
    part = np.empty(int(p_max) + 1, dtype=np.int64)
    p = _I32()
    _chk(lib().ddps_partition_rows(int(n), int(b), int(p_max), part.ctypes.data, ctypes.byref(p)),
         "ddps_partition_rows")
    return part[:p.value + 1].copy()


class GeneralSystem:
    """A general sparse matrix prepared for the banded block path: reverse
    Cuthill-McKee order, the permuted CSR (attributes n, row_ptr, col, val,
    as Solver takes them), its half-bandwidth and an equal-slab partition
    into at most p_max blocks.  to_perm / from_perm move vectors between the
    original and the permuted numbering."""

    def __init__(self, n, row_ptr, col, val, p_max):
        self.perm = ddps_rcm(n, row_ptr, col)
        self.n = int(n)
        self.row_ptr, self.col, self.val = ddps_permute_csr(n, row_ptr, col, val, self.perm)
        self.b = ddps_bandwidth(n, self.row_ptr, self.col)
        self.part_ptr = ddps_partition_rows(n, self.b, p_max)

    def to_perm(self, x):
        return x[self.perm]

    def from_perm(self, y):
        import numpy as np
        out = np.empty_like(y)
        out[self.perm] = y
        return out


def ddps_memory(h):
    b = ctypes.c_size_t()
    _chk(lib().ddps_memory(h, ctypes.byref(b)), "ddps_memory")
    return b.value


def ddps_destroy(h):
    if h:
        lib().ddps_destroy(h)


def ddps_status_string(code):
    return lib().ddps_status_string(int(code)).decode()


# ------------------------------------------------------------------ helper
class Solver:
    """Owns one handle: setup on construction, destroy on close()."""

    def __init__(self, A, part_ptr, dtype="f64", delta=0.0, inner_tol=1e-12, inner_maxit=1000,
                 outer_maxit=1000, outer="refine", max_rhs=1, guess=False, device="cuda", stream=None,
                 mem_budget=0, streams=0, graph=False, inner_prec=0, retrieval=0, norm=0, work_slots=0,
                 reduced="bicgstab", loosen_ratio=0.0, gemv_sums=0, block_factor="lu"):
        import torch
        self.n = A.n
        self.p = len(part_ptr) - 1
        o = ddps_default_options()
        o.drop_delta = float(delta)
        o.factor_dtype = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
        o.inner_tol = float(inner_tol)
        o.inner_maxit = int(inner_maxit)
        o.outer_maxit = int(outer_maxit)
        o.outer_method = 1 if outer == "refine" else 0
        o.max_rhs = int(max_rhs)
        o.guess = 1 if guess else 0
        o.mem_budget = int(mem_budget)
        o.factor_streams = int(streams)
        o.factor_graph = 1 if graph else 0
        o.inner_prec = int(inner_prec)
        o.retrieval = int(retrieval)
        o.norm = int(norm)
        o.work_slots = int(work_slots)
        o.reduced_solve = 1 if reduced == "direct" else 0
        o.loosen_ratio = float(loosen_ratio)
        o.gemv_sums = int(gemv_sums)
        o.block_factor = {"lu": 0, "ilu0": 1}[block_factor]
        st = stream if stream is not None else torch.cuda.current_stream(device)
        o.stream = ctypes.c_void_p(st.cuda_stream)
        self.opt = o
        self.stream = st
        self.row_ptr = torch.from_numpy(A.row_ptr).to(device)
        self.col = torch.from_numpy(A.col).to(device)
        self.val = torch.from_numpy(A.val).to(device)
        self.h = ddps_setup(A.n, self.p, part_ptr, self.row_ptr, self.col, self.val, o)

    def factor(self):
        ddps_factor(self.h)

    def solve(self, f, x, tol, check=True):
        return ddps_solve(self.h, f, x, tol, check=check)

    def close(self):
        if self.h:
            ddps_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

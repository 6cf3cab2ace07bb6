"""ctypes declarations of librcp's C interface (include/rcp.h).

Argument marshalling only.  Loading fails loudly when the HIP library has
not been built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librcp.so")

RCP_MAX_NDIM = 8
RCP_MAX_L = 64
RCP_MAX_RANK = 64
RCP_NOALLOC_SCRATCH_BYTES = 32 << 20

RCP_OK = 0
RCP_ERR_INVALID_ARG = 1
RCP_ERR_WORKSPACE = 2
RCP_ERR_HIP = 3
RCP_ERR_NUMERIC = 4
RCP_ERR_UNSUPPORTED = 5

RCP_INFO_PINV_FALLBACK = 1
RCP_INFO_NONFINITE = 2
RCP_INFO_EIG_NOT_CONVERGED = 4
RCP_INFO_QR_HOUSEHOLDER = 8

PRECISIONS = {"fp32": 0, "bf16": 1, "fp16": 2}
KERNEL_CLASSES = ["sketch", "power", "contract_in", "contract_out", "reduce", "qr", "als",
                  "expand", "other", "bcd", "mttkrp", "cp_update"]
SCHEMES = {"sequential": 0, "independent": 1}
SOLVERS = {"als": 0, "bcd": 1, "cp_als": 2}
TEST_MATRICES = {"gaussian": 0, "uniform": 1, "halton": 2, "columns": 3}


class Problem(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("k", ctypes.c_int32),
        ("p", ctypes.c_int32),
        ("q", ctypes.c_int32),
        ("dims", ctypes.c_int64 * RCP_MAX_NDIM),
        ("max_iters", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("scheme", ctypes.c_int32),
        ("solver", ctypes.c_int32),
        ("tol", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("test_matrix", ctypes.c_int32),
        ("compress_mask", ctypes.c_uint32),
        ("per_mode_p", ctypes.c_int32),
        ("mode_p", ctypes.c_int32 * RCP_MAX_NDIM),
    ]


class AlsInfo(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("rho", ctypes.c_double),
        ("rel_err", ctypes.c_double),
        ("normX2", ctypes.c_double),
    ]


_vp = ctypes.c_void_p
_st = ctypes.c_int
_i64p = ctypes.POINTER(ctypes.c_int64)

# name -> (restype, argtypes)
SIGNATURES = {
    "rcp_workspace_size": (_st, [ctypes.POINTER(Problem), ctypes.POINTER(ctypes.c_size_t)]),
    "rcp_init": (_st, [ctypes.POINTER(_vp), ctypes.POINTER(Problem), _vp, ctypes.c_size_t, _vp]),
    "rcp_destroy": (_st, [_vp]),
    "rcp_sketch": (_st, [_vp, _vp, _i64p, ctypes.c_int32, _vp]),
    "rcp_compress": (_st, [_vp, _vp, _i64p, ctypes.c_int32, _vp, _vp]),
    "rcp_norm2": (_st, [_vp, _vp, ctypes.c_int64, _vp]),
    "rcp_als": (_st, [_vp, _vp, ctypes.POINTER(_vp), _vp, _vp, _vp, ctypes.c_int32]),
    "rcp_read_status": (_st, [_vp, ctypes.POINTER(ctypes.c_int32)]),
    "rcp_bcd": (_st, [_vp, _vp, ctypes.POINTER(_vp), _vp, _vp, _vp, ctypes.c_int32]),
    "rcp_expand": (_st, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp, ctypes.POINTER(_vp), _vp]),
    "rcp_decompose": (_st, [_vp, _vp, ctypes.POINTER(_vp), _vp, _vp]),
    "rcp_cp_als": (_st, [_vp, _vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp, _vp]),
    "rcp_decompose_noalloc": (_st, [ctypes.POINTER(Problem), _vp, ctypes.POINTER(_vp), _vp, _vp, _vp]),
    "rcp_get_bases": (_st, [_vp, ctypes.POINTER(_vp)]),
    "rcp_get_core": (_st, [_vp, ctypes.POINTER(_vp), _i64p]),
    "rcp_debug_omega": (_st, [_vp, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, _vp]),
    "rcp_debug_philox": (_st, [_vp, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, _vp]),
    "rcp_debug_columns": (_st, [_vp, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, _vp]),
    "rcp_profile": (_st, [_vp, ctypes.c_int32]),
    "rcp_profile_read": (_st, [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                               ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                               ctypes.POINTER(ctypes.c_double)]),
    "rcp_batch_workspace_size": (_st, [ctypes.POINTER(Problem), ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_size_t)]),
    "rcp_batch_init": (_st, [ctypes.POINTER(_vp), ctypes.POINTER(Problem), ctypes.c_int32, _vp,
                             ctypes.c_size_t, _vp]),
    "rcp_batch_decompose": (_st, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(ctypes.POINTER(_vp)),
                                  ctypes.POINTER(_vp), _vp]),
    "rcp_batch_read_status": (_st, [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "rcp_batch_get_core": (_st, [_vp, ctypes.c_int32, ctypes.POINTER(_vp), ctypes.POINTER(ctypes.c_int64)]),
    "rcp_batch_autotune": (_st, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(ctypes.POINTER(_vp)),
                                 ctypes.POINTER(_vp), _vp, ctypes.POINTER(ctypes.c_int32),
                                 ctypes.POINTER(ctypes.c_double)]),
    "rcp_batch_destroy": (_st, [_vp]),
    "rcp_status_string": (ctypes.c_char_p, [_st]),
    "rcp_version": (ctypes.c_char_p, []),
}

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load librcp.so (once) and declare every entry point."""
    global _lib
    if _lib is not None:
        return _lib
    try:  # share PyTorch's HIP runtime (same SONAME) when PyTorch is present
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(path):
        raise RuntimeError(
            f"librcp is not built ({path} missing); run `python -m paper_1703_09074_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class RcpError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = load().rcp_status_string(status).decode()
        super().__init__(f"{where}: {msg}")
        self.status = status


def check(status: int, where: str) -> None:
    if status != RCP_OK:
        raise RcpError(status, where)


def ptr_array(ptrs):
    arr = (_vp * len(ptrs))()
    for i, p in enumerate(ptrs):
        arr[i] = p
    return arr


def dims_array(dims):
    arr = (ctypes.c_int64 * RCP_MAX_NDIM)()
    for i, d in enumerate(dims):
        arr[i] = int(d)
    return arr


def make_problem(dims, k, p, q, max_iters, tol, seed, precision="fp32", scheme="sequential",
                 solver="als", test_matrix="gaussian", modes=None, p_modes=None):
    prob = Problem()
    prob.ndim = len(dims)
    prob.k = int(k)
    prob.p = int(p)
    prob.q = int(q)
    for i, d in enumerate(dims):
        prob.dims[i] = int(d)
    prob.max_iters = int(max_iters)
    prob.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    prob.scheme = SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)
    prob.solver = SOLVERS[solver] if isinstance(solver, str) else int(solver)
    prob.tol = float(tol)
    prob.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    prob.test_matrix = TEST_MATRICES[test_matrix] if isinstance(test_matrix, str) else int(test_matrix)
    if modes is not None and not list(modes):
        raise ValueError("at least one mode must be compressed")
    prob.compress_mask = 0 if modes is None else sum(1 << int(m) for m in modes)
    prob.per_mode_p = 0 if p_modes is None else 1
    if p_modes is not None:
        for i, v in enumerate(p_modes):
            prob.mode_p[i] = int(v)
    return prob

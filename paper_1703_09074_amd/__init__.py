"""Randomized CP decomposition on AMD MI355X (gfx950).

Python front end of librcp (include/rcp.h).  PyTorch supplies device memory
and the HIP stream; every step of the computation runs in the library's HIP
kernels.  There is no CPU fallback: without the built library (or without a
GPU) these functions raise.

    lam, factors, info = decompose(X, k=20, p=10, q=2, iters=100)

X is a C-order float32 CUDA tensor; factors[n] is I_n x k, lam has k
entries sorted descending (Algorithm 2 of Erichson et al., "Randomized CP
Tensor Decomposition": randomized compression, CP-ALS on the core,
back-projection).
"""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence

from . import _lib

__all__ = ["Plan", "decompose", "sketch_width", "library_path"]

library_path = _lib.LIB_PATH


def sketch_width(k: int, p: int, I: int) -> int:
    return min(int(k) + int(p), int(I))


def _torch():
    import torch
    return torch


def _stream_handle(torch, device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _f32(t, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float32 tensor")
    return t


class Plan:
    """A plan: the problem, its device workspace and the stream it runs on.

    All methods enqueue on the current HIP stream of ``device`` at plan
    creation and return without synchronising.
    """

    def __init__(self, dims: Sequence[int], k: int, p: int = 10, q: int = 2,
                 max_iters: int = 50, tol: float = 0.0, seed: int = 0,
                 scheme: str = "sequential", precision: str = "fp32", device="cuda",
                 solver: str = "als", test_matrix: str = "gaussian",
                 modes: Optional[Sequence[int]] = None, p_modes: Optional[Sequence[int]] = None):
        """``test_matrix``: "gaussian", "uniform", "halton" or "columns";
        ``modes``: the modes Algorithm 1 compresses (default all; the others
        keep Q_n = I); ``p_modes``: oversampling per mode in place of ``p``."""
        torch = _torch()
        self.lib = _lib.load()
        self.dims = [int(d) for d in dims]
        self.N = len(self.dims)
        self.k = int(k)
        self.R = int(k)
        self.p = int(p)
        self.q = int(q)
        self.p_modes = [int(p)] * self.N if p_modes is None else [int(v) for v in p_modes]
        if len(self.p_modes) != self.N:
            raise ValueError(f"p_modes needs {self.N} entries")
        self.modes = list(range(self.N)) if modes is None else sorted({int(m) for m in modes})
        self.l = [sketch_width(k, self.p_modes[n], d) if n in self.modes else d
                  for n, d in enumerate(self.dims)]
        self.device = torch.device(device)
        self.problem = _lib.make_problem(self.dims, k, p, q, max_iters, tol, seed, precision, scheme,
                                         solver, test_matrix, modes, p_modes)
        nbytes = ctypes.c_size_t(0)
        _lib.check(self.lib.rcp_workspace_size(ctypes.byref(self.problem), ctypes.byref(nbytes)),
                   "rcp_workspace_size")
        self.workspace = torch.empty(max(256, nbytes.value), dtype=torch.uint8, device=self.device)
        self.stream = _stream_handle(torch, self.device)
        handle = ctypes.c_void_p(0)
        _lib.check(self.lib.rcp_init(ctypes.byref(handle), ctypes.byref(self.problem),
                                     ctypes.c_void_p(self.workspace.data_ptr()),
                                     ctypes.c_size_t(self.workspace.numel()), self.stream),
                   "rcp_init")
        self.handle = handle

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.lib.rcp_destroy(h)
            self.handle = None

    # -- helpers ---------------------------------------------------------------
    def _empty(self, shape, dtype=None):
        torch = _torch()
        return torch.empty(shape, dtype=dtype or torch.float32, device=self.device)

    def _info_buffer(self):
        torch = _torch()
        return torch.zeros(ctypes.sizeof(_lib.AlsInfo), dtype=torch.uint8, device=self.device)

    @staticmethod
    def read_info(buf) -> dict:
        raw = bytes(buf.cpu().numpy().tobytes())
        info = _lib.AlsInfo.from_buffer_copy(raw)
        return dict(iters=info.iters, status=info.status, rho=info.rho, rel_err=info.rel_err,
                    normX2=info.normX2)

    # -- entry points ------------------------------------------------------------
    def sketch(self, T, mode: int, cur_dims: Optional[Sequence[int]] = None):
        """Orthonormal basis Q_n (I_n x l) of mode ``mode`` (Algorithm 1's range finder)."""
        _f32(T, "T")
        cur = list(T.shape) if cur_dims is None else [int(d) for d in cur_dims]
        l = sketch_width(self.k, self.p_modes[mode], cur[mode])
        Q = self._empty((cur[mode], l))
        _lib.check(self.lib.rcp_sketch(self.handle, ctypes.c_void_p(T.data_ptr()),
                                       _lib.dims_array(cur), int(mode),
                                       ctypes.c_void_p(Q.data_ptr())), "rcp_sketch")
        return Q

    def compress(self, T, mode: int, Q):
        """T x_mode Q^T (Algorithm 1's projection)."""
        _f32(T, "T")
        _f32(Q, "Q")
        cur = list(T.shape)
        out_shape = list(cur)
        out_shape[mode] = Q.shape[1]
        out = self._empty(out_shape)
        _lib.check(self.lib.rcp_compress(self.handle, ctypes.c_void_p(T.data_ptr()),
                                         _lib.dims_array(cur), int(mode),
                                         ctypes.c_void_p(Q.data_ptr()),
                                         ctypes.c_void_p(out.data_ptr())), "rcp_compress")
        return out

    def norm2(self, X):
        torch = _torch()
        _f32(X, "X")
        out = torch.empty(1, dtype=torch.float64, device=self.device)
        _lib.check(self.lib.rcp_norm2(self.handle, ctypes.c_void_p(X.data_ptr()), X.numel(),
                                      ctypes.c_void_p(out.data_ptr())), "rcp_norm2")
        return out

    def als(self, core, normX2=None, init: Optional[List] = None):
        """CP-ALS on the core (Algorithm 2): (factors, lambda, info buffer).

        init: starting factors (l_n x R float32 CUDA tensors, one per mode; the
        first is not read) instead of the eigenvector start (warm start)."""
        return self._core_solver(self.lib.rcp_als, "rcp_als", core, normX2, init)

    def _core_solver(self, fn, name, core, normX2, init):
        _f32(core, "core")
        if list(core.shape) != self.l:
            raise ValueError(f"core has shape {list(core.shape)}, plan expects {self.l}")
        At = [self._empty((self.l[n], self.R)) for n in range(self.N)]
        if init is not None:
            if len(init) != self.N:
                raise ValueError(f"init needs {self.N} factors")
            for n in range(1, self.N):
                _f32(init[n], f"init[{n}]")
                if list(init[n].shape) != [self.l[n], self.R]:
                    raise ValueError(f"init[{n}] has shape {list(init[n].shape)}, "
                                     f"expected {[self.l[n], self.R]}")
                At[n].copy_(init[n])
        lam = self._empty((self.R,))
        info = self._info_buffer()
        if normX2 is not None and (normX2.dtype != _torch().float64 or not normX2.is_cuda):
            raise TypeError("normX2 must be a float64 CUDA tensor")
        nptr = ctypes.c_void_p(normX2.data_ptr()) if normX2 is not None else ctypes.c_void_p(0)
        _lib.check(fn(self.handle, ctypes.c_void_p(core.data_ptr()),
                      _lib.ptr_array([a.data_ptr() for a in At]),
                      ctypes.c_void_p(lam.data_ptr()), nptr,
                      ctypes.c_void_p(info.data_ptr()), 1 if init is not None else 0), name)
        return At, lam, info

    def bcd(self, core, normX2=None, init: Optional[List] = None):
        """Block coordinate descent on the core (Algorithm 3):
        (factors, lambda, info buffer); arguments as ``als``."""
        return self._core_solver(self.lib.rcp_bcd, "rcp_bcd", core, normX2, init)

    def cp_als(self, X, init: Optional[List] = None):
        """Deterministic CP-ALS on the full tensor X (rcp_cp_als; the plan's
        solver must be "cp_als"): (lambda, [A_n], info buffer).  init: N
        float32 CUDA tensors (I_n x R; init[0] is not read) to start from,
        else the eigenvector start by subspace iteration."""
        _f32(X, "X")
        if list(X.shape) != self.dims:
            raise ValueError(f"X has shape {list(X.shape)}, plan expects {self.dims}")
        init_arg = None
        if init is not None:
            if len(init) != self.N:
                raise ValueError(f"init needs {self.N} factors")
            for n in range(1, self.N):
                _f32(init[n], f"init[{n}]")
                if list(init[n].shape) != [self.dims[n], self.R]:
                    raise ValueError(f"init[{n}] has shape {list(init[n].shape)}, "
                                     f"expected {[self.dims[n], self.R]}")
            init_arg = _lib.ptr_array([init[0].data_ptr() if init[0] is not None else 0] +
                                      [t.data_ptr() for t in init[1:]])
        A = [self._empty((self.dims[n], self.R)) for n in range(self.N)]
        lam = self._empty((self.R,))
        info = self._info_buffer()
        _lib.check(self.lib.rcp_cp_als(self.handle, ctypes.c_void_p(X.data_ptr()), init_arg,
                                       _lib.ptr_array([a.data_ptr() for a in A]),
                                       ctypes.c_void_p(lam.data_ptr()),
                                       ctypes.c_void_p(info.data_ptr())), "rcp_cp_als")
        return lam, A, info

    def read_status(self) -> int:
        """The plan's device status word (RCP_INFO_* bits raised since the last
        read), cleared by the read; waits for the plan's stream."""
        v = ctypes.c_int32(0)
        _lib.check(self.lib.rcp_read_status(self.handle, ctypes.byref(v)), "rcp_read_status")
        return int(v.value)

    def expand(self, Q: List, At: List, lam):
        """A_n = Q_n Ã_n and the final renormalisation (eq. qbs, Algorithm 2's factor recovery and renormalisation)."""
        A = [self._empty((self.dims[n], self.R)) for n in range(self.N)]
        lam_out = self._empty((self.R,))
        _lib.check(self.lib.rcp_expand(self.handle, _lib.ptr_array([q.data_ptr() for q in Q]),
                                       _lib.ptr_array([a.data_ptr() for a in At]),
                                       ctypes.c_void_p(lam.data_ptr()),
                                       _lib.ptr_array([a.data_ptr() for a in A]),
                                       ctypes.c_void_p(lam_out.data_ptr())), "rcp_expand")
        return A, lam_out

    def decompose_into(self, X, A: List, lam, info) -> None:
        """The whole path into preallocated outputs (no allocation)."""
        _f32(X, "X")
        if list(X.shape) != self.dims:
            raise ValueError(f"X has shape {list(X.shape)}, plan expects {self.dims}")
        if len(A) != self.N:
            raise ValueError(f"expected {self.N} factor outputs, got {len(A)}")
        for n, a in enumerate(A):
            _f32(a, f"A[{n}]")
            if list(a.shape) != [self.dims[n], self.R]:
                raise ValueError(f"A[{n}] has shape {list(a.shape)}, expected {[self.dims[n], self.R]}")
        _f32(lam, "lam")
        if lam.numel() < self.R:
            raise ValueError("lam is too small")
        if not info.is_cuda or not info.is_contiguous() or \
                info.numel() * info.element_size() < ctypes.sizeof(_lib.AlsInfo):
            raise ValueError("info must be a contiguous CUDA buffer of at least "
                             f"{ctypes.sizeof(_lib.AlsInfo)} bytes")
        _lib.check(self.lib.rcp_decompose(self.handle, ctypes.c_void_p(X.data_ptr()),
                                          _lib.ptr_array([a.data_ptr() for a in A]),
                                          ctypes.c_void_p(lam.data_ptr()),
                                          ctypes.c_void_p(info.data_ptr())), "rcp_decompose")

    def decompose(self, X):
        """(lambda, [A_n], info buffer) for the float32 CUDA tensor X."""
        _f32(X, "X")
        if list(X.shape) != self.dims:
            raise ValueError(f"X has shape {list(X.shape)}, plan expects {self.dims}")
        A = [self._empty((self.dims[n], self.R)) for n in range(self.N)]
        lam = self._empty((self.R,))
        info = self._info_buffer()
        self.decompose_into(X, A, lam, info)
        return lam, A, info

    def _workspace_view(self, ptr, shape):
        """float32 view of a region of the plan's workspace."""
        n = 1
        for s in shape:
            n *= int(s)
        off = int(ptr) - self.workspace.data_ptr()
        if off < 0 or off % 4 or off + 4 * n > self.workspace.numel():
            raise RuntimeError("library returned a pointer outside the workspace")
        return self.workspace[off:off + 4 * n].view(_torch().float32).view(*shape)

    def bases(self):
        """Views of the bases Q_n from the last decompose (valid until the next call)."""
        arr = (ctypes.c_void_p * self.N)()
        _lib.check(self.lib.rcp_get_bases(self.handle, arr), "rcp_get_bases")
        return [self._workspace_view(arr[n], (self.dims[n], self.l[n])) for n in range(self.N)]

    def core(self):
        """View of the core from the last decompose (valid until the next call)."""
        p = ctypes.c_void_p(0)
        dims = (ctypes.c_int64 * _lib.RCP_MAX_NDIM)()
        _lib.check(self.lib.rcp_get_core(self.handle, ctypes.byref(p), dims), "rcp_get_core")
        return self._workspace_view(p.value, tuple(dims[n] for n in range(self.N)))

    def profile(self, enable: bool) -> None:
        """Start (and clear) or stop per-kernel event timing of this plan's launches."""
        _lib.check(self.lib.rcp_profile(self.handle, 1 if enable else 0), "rcp_profile")

    def profile_read(self) -> dict:
        """{kernel class: dict(launches, ms, bytes, flops)} of the recorded launches."""
        out = {}
        for cls, name in enumerate(_lib.KERNEL_CLASSES):
            n = ctypes.c_int64(0)
            ms = ctypes.c_double(0)
            b = ctypes.c_double(0)
            f = ctypes.c_double(0)
            _lib.check(self.lib.rcp_profile_read(self.handle, cls, ctypes.byref(n), ctypes.byref(ms),
                                                 ctypes.byref(b), ctypes.byref(f)),
                       "rcp_profile_read")
            if n.value:
                out[name] = dict(launches=n.value, ms=ms.value, bytes=b.value, flops=f.value)
        return out

    def omega(self, mode: int, row0: int, nrows: int, l: int):
        out = self._empty((nrows, l))
        _lib.check(self.lib.rcp_debug_omega(self.handle, int(mode), int(row0), int(nrows), int(l),
                                            ctypes.c_void_p(out.data_ptr())), "rcp_debug_omega")
        return out

    def columns(self, mode: int, J: int, l: int):
        """The l unfolding columns (ascending, int64) that the column-selection
        sketch of mode ``mode`` takes out of J."""
        out = self._empty((l,), dtype=_torch().int64)
        _lib.check(self.lib.rcp_debug_columns(self.handle, int(mode), int(J), int(l),
                                              ctypes.c_void_p(out.data_ptr())), "rcp_debug_columns")
        return out

    def philox_words(self, mode: int, row0: int, nrows: int, ngroups: int):
        """Raw Philox4x32-10 words (nrows x ngroups x 4, int32 bit patterns of
        the uint32 words) behind rows [row0, row0 + nrows) of Omega_mode."""
        out = self._empty((nrows, ngroups, 4), dtype=_torch().int32)
        _lib.check(self.lib.rcp_debug_philox(self.handle, int(mode), int(row0), int(nrows),
                                             int(ngroups), ctypes.c_void_p(out.data_ptr())),
                   "rcp_debug_philox")
        return out


class Batch:
    """Independent problems decomposed as one unit (rcp_batch_*).  The outputs
    (factors, lambda, info) are allocated here and passed on every call; the
    batch runs on the current HIP stream of ``device`` at creation (a
    non-default stream records the work in a HIP graph on the first call).

    problems: sequence of dicts with keys dims, k and optionally p, q,
    max_iters, tol, seed, precision, scheme, test_matrix, modes, p_modes.
    """

    def __init__(self, problems, device="cuda"):
        torch = _torch()
        self.lib = _lib.load()
        self.device = torch.device(device)
        self.count = len(problems)
        arr = (_lib.Problem * self.count)()
        self.dims = []
        self.k = []
        for i, pr in enumerate(problems):
            dims = [int(d) for d in pr["dims"]]
            arr[i] = _lib.make_problem(dims, pr["k"], pr.get("p", 10), pr.get("q", 2),
                                       pr.get("max_iters", 50), pr.get("tol", 0.0),
                                       pr.get("seed", 0), pr.get("precision", "fp32"),
                                       pr.get("scheme", "sequential"), "als",
                                       pr.get("test_matrix", "gaussian"), pr.get("modes"),
                                       pr.get("p_modes"))
            self.dims.append(dims)
            self.k.append(int(pr["k"]))
        self._problems = arr
        nbytes = ctypes.c_size_t(0)
        _lib.check(self.lib.rcp_batch_workspace_size(arr, self.count, ctypes.byref(nbytes)),
                   "rcp_batch_workspace_size")
        self.workspace = torch.empty(max(256, nbytes.value), dtype=torch.uint8, device=self.device)
        self.A = [[torch.empty((d, k), dtype=torch.float32, device=self.device) for d in dims]
                  for dims, k in zip(self.dims, self.k)]
        self.lam = [torch.empty((k,), dtype=torch.float32, device=self.device) for k in self.k]
        self.info = torch.zeros(self.count * ctypes.sizeof(_lib.AlsInfo), dtype=torch.uint8,
                                device=self.device)
        self.stream = _stream_handle(torch, self.device)
        handle = ctypes.c_void_p(0)
        _lib.check(self.lib.rcp_batch_init(ctypes.byref(handle), arr, self.count,
                                           ctypes.c_void_p(self.workspace.data_ptr()),
                                           ctypes.c_size_t(self.workspace.numel()), self.stream),
                   "rcp_batch_init")
        self.handle = handle

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.lib.rcp_batch_destroy(h)
            self.handle = None

    def _io(self, Xs):
        if len(Xs) != self.count:
            raise ValueError(f"expected {self.count} tensors, got {len(Xs)}")
        for X, dims in zip(Xs, self.dims):
            _f32(X, "X")
            if list(X.shape) != dims:
                raise ValueError(f"tensor of shape {list(X.shape)} where {dims} was planned")
        self._X = list(Xs)
        rows = [_lib.ptr_array([a.data_ptr() for a in As]) for As in self.A]
        self._rows = rows
        A_arg = (ctypes.POINTER(ctypes.c_void_p) * self.count)(
            *[ctypes.cast(r, ctypes.POINTER(ctypes.c_void_p)) for r in rows])
        lam_arg = _lib.ptr_array([t.data_ptr() for t in self.lam])
        return (_lib.ptr_array([X.data_ptr() for X in Xs]), A_arg, lam_arg,
                ctypes.c_void_p(self.info.data_ptr()))

    def decompose(self, Xs) -> None:
        """Enqueue the decomposition of every tensor (float32 CUDA, shapes as
        given at creation); results land in .A, .lam and .info."""
        X_arg, A_arg, lam_arg, info_arg = self._io(Xs)
        _lib.check(self.lib.rcp_batch_decompose(self.handle, X_arg, A_arg, lam_arg, info_arg),
                   "rcp_batch_decompose")

    def autotune(self, Xs) -> dict:
        """Time the batch over candidate launch shapes (rcp_batch_autotune)
        and keep the fastest; blocks.  Returns the chosen shape and its time."""
        X_arg, A_arg, lam_arg, info_arg = self._io(Xs)
        shape = (ctypes.c_int32 * 3)()
        ms = ctypes.c_double(0.0)
        _lib.check(self.lib.rcp_batch_autotune(self.handle, X_arg, A_arg, lam_arg, info_arg,
                                               shape, ctypes.byref(ms)), "rcp_batch_autotune")
        return {"streams": shape[0], "workgroups": shape[1], "row_block_rows": 64 * shape[2],
                "ms_per_batch": ms.value}

    def core(self, index: int):
        """View of problem ``index``'s core from the last decompose
        (rcp_batch_get_core; valid until the next decompose)."""
        p = ctypes.c_void_p(0)
        dims = (ctypes.c_int64 * _lib.RCP_MAX_NDIM)()
        _lib.check(self.lib.rcp_batch_get_core(self.handle, int(index), ctypes.byref(p), dims),
                   "rcp_batch_get_core")
        shape = tuple(dims[n] for n in range(len(self.dims[index])))
        n = 1
        for d in shape:
            n *= int(d)
        off = int(p.value) - self.workspace.data_ptr()
        if off < 0 or off % 4 or off + 4 * n > self.workspace.numel():
            raise RuntimeError("library returned a pointer outside the workspace")
        return self.workspace[off:off + 4 * n].view(_torch().float32).view(*shape)

    def read_status(self, index: int) -> int:
        """Status word of problem ``index`` (rcp_batch_read_status); blocks."""
        v = ctypes.c_int32(0)
        _lib.check(self.lib.rcp_batch_read_status(self.handle, int(index), ctypes.byref(v)),
                   "rcp_batch_read_status")
        return int(v.value)

    def read_info(self):
        raw = bytes(self.info.cpu().numpy().tobytes())
        sz = ctypes.sizeof(_lib.AlsInfo)
        out = []
        for i in range(self.count):
            info = _lib.AlsInfo.from_buffer_copy(raw[i * sz:(i + 1) * sz])
            out.append(dict(iters=info.iters, status=info.status, rho=info.rho,
                            rel_err=info.rel_err, normX2=info.normX2))
        return out


def decompose(X, k: int, p: int = 10, q: int = 2, iters: int = 50, tol: float = 0.0,
              seed: int = 0, scheme: str = "sequential", precision: str = "fp32",
              solver: str = "als", test_matrix: str = "gaussian",
              modes: Optional[Sequence[int]] = None, p_modes: Optional[Sequence[int]] = None):
    """Randomized CP of X (Algorithm 2, or Algorithm 3 with solver="bcd").
    Returns (lambda, [A_n], info dict)."""
    plan = Plan(list(X.shape), k, p, q, iters, tol, seed, scheme, precision, device=X.device,
                solver=solver, test_matrix=test_matrix, modes=modes, p_modes=p_modes)
    lam, A, info = plan.decompose(X)
    return lam, A, Plan.read_info(info)

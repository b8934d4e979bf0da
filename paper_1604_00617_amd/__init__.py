"""Python binding of the MI355X Accelerated Cyclic Reduction library (libacr.so).

Thin ctypes marshalling over the C ABI declared in ``include/acr.h``: the
functions below have the same names as the C entry points and only convert
torch tensors to device pointers and the current HIP stream.  Every step of
factorisation and solve runs in the library's HIP kernels; there is no
fallback path, and ``load()`` raises if the built library is missing.

Vectors: torch float64 tensors on the GPU, shape (N,) or (N, nrhs), unknown
index i*nx + j (block i = grid row).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libacr.so")

ACR_FP64 = 0
ACR_MIXED_FP32 = 1
PRECISIONS = {"fp64": ACR_FP64, "mixed": ACR_MIXED_FP32, "fp32": ACR_MIXED_FP32}

STATUS = {0: "ACR_OK", 1: "ACR_ERR_INVALID_ARG", 2: "ACR_ERR_OOM", 3: "ACR_ERR_SINGULAR",
          4: "ACR_ERR_NOT_CONVERGED", 5: "ACR_ERR_DEVICE", 6: "ACR_ERR_INTERNAL"}


class ACRError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.name = STATUS.get(code, str(code))


class _Operator(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("diag", ctypes.c_void_p), ("west", ctypes.c_void_p), ("east", ctypes.c_void_p),
                ("south", ctypes.c_void_p), ("north", ctypes.c_void_p)]


class _Options(ctypes.Structure):
    _fields_ = [("leaf", ctypes.c_int32), ("eps", ctypes.c_double), ("precision", ctypes.c_int32),
                ("max_rank", ctypes.c_int32), ("inner_eps", ctypes.c_double), ("stop_blocks", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("leaf", ctypes.c_int32),
                ("depth", ctypes.c_int32), ("levels", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("eps", ctypes.c_double), ("factor_bytes", ctypes.c_int64), ("max_rank", ctypes.c_int32),
                ("level_max_rank", ctypes.c_int32 * 40), ("factor_flops", ctypes.c_double),
                ("solve_bytes", ctypes.c_double), ("solve_flops_per_rhs", ctypes.c_double),
                ("factor_bytes_ranked", ctypes.c_double), ("solve_bytes_ranked", ctypes.c_double),
                ("level_mean_rank", ctypes.c_double * 40), ("factor_launches", ctypes.c_int64),
                ("stop_blocks", ctypes.c_int32)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libacr.so (raises if it has not been built: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1604_00617_amd.build`")
    lib = ctypes.CDLL(path)
    P, I32, D, S = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_int
    lib.acr_factor.argtypes = [ctypes.POINTER(_Operator), ctypes.POINTER(_Options), P, ctypes.POINTER(P)]
    lib.acr_solve.argtypes = [P, P, P, I32, P]
    lib.acr_solve_refined.argtypes = [P, ctypes.POINTER(_Operator), P, P, I32, D, I32,
                                      ctypes.POINTER(I32), ctypes.POINTER(D), P]
    lib.acr_solve_krylov.argtypes = [P, ctypes.POINTER(_Operator), P, P, I32, D, I32, I32,
                                     ctypes.POINTER(I32), ctypes.POINTER(D), P]
    lib.acr_residual.argtypes = [ctypes.POINTER(_Operator), P, P, P, I32, P]
    lib.acr_get_info.argtypes = [P, ctypes.POINTER(_Info)]
    lib.acr_get_block.argtypes = [P, I32, I32, I32, P, P]
    lib.acr_destroy.argtypes = [P]
    lib.acr_status_string.argtypes = [S]
    lib.acr_status_string.restype = ctypes.c_char_p
    lib.acr_last_error.restype = ctypes.c_char_p
    for name in ("acr_factor", "acr_solve", "acr_solve_refined", "acr_solve_krylov", "acr_residual",
                 "acr_get_info", "acr_get_block", "acr_destroy", "acr_trim_pool"):
        getattr(lib, name).restype = S
    _lib = lib
    return lib


def _check(code: int):
    if code != 0:
        raise ACRError(code, load().acr_last_error().decode())


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


@dataclass
class Operator:
    """5-point stencil operator on the device (FP64 arrays of length nx*ny)."""
    nx: int
    ny: int
    diag: "object"
    west: "object"
    east: "object"
    south: "object"
    north: "object"

    @classmethod
    def from_arrays(cls, nx, ny, diag, west, east, south, north, device="cuda"):
        import torch
        conv = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).to(device)
        return cls(nx, ny, conv(diag), conv(west), conv(east), conv(south), conv(north))

    def _c(self) -> _Operator:
        return _Operator(self.nx, self.ny, self.diag.data_ptr(), self.west.data_ptr(),
                         self.east.data_ptr(), self.south.data_ptr(), self.north.data_ptr())

    @property
    def n(self):
        return self.nx * self.ny


class _Operator3d(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32)] + [
        (f, ctypes.c_void_p) for f in ("diag", "west", "east", "south", "north", "down", "up")]


@dataclass
class Operator3d:
    """7-point stencil operator on the device (FP64 arrays of length nx*ny*nz); as a
    block-tridiagonal system one block per plane (block size nx*ny, nz blocks)."""
    nx: int
    ny: int
    nz: int
    diag: "object"
    west: "object"
    east: "object"
    south: "object"
    north: "object"
    down: "object"
    up: "object"

    @classmethod
    def from_arrays(cls, nx, ny, nz, diag, west, east, south, north, down, up, device="cuda"):
        import torch
        conv = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).to(device)
        return cls(nx, ny, nz, *[conv(a) for a in (diag, west, east, south, north, down, up)])

    def _c(self) -> _Operator3d:
        return _Operator3d(self.nx, self.ny, self.nz, *[a.data_ptr() for a in (
            self.diag, self.west, self.east, self.south, self.north, self.down, self.up)])

    @property
    def n(self):
        return self.nx * self.ny * self.nz


class _DenseOperator(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("D", ctypes.c_void_p), ("E", ctypes.c_void_p), ("F", ctypes.c_void_p)]


@dataclass
class DenseOperator:
    """Block-tridiagonal operator of dense blocks: D, E, F float64 device tensors of shape
    (ny, nx, nx) holding column-major blocks (block i is D[i].T in row-major terms)."""
    nx: int
    ny: int
    D: "object"
    E: "object"
    F: "object"

    @classmethod
    def from_blocks(cls, D, E, F, device="cuda"):
        """D, E, F: lists of ny (nx x nx) numpy arrays."""
        import torch
        conv = lambda bl: torch.as_tensor(np.ascontiguousarray(np.stack([b.T for b in bl]))).to(device)
        return cls(D[0].shape[0], len(D), conv(D), conv(E), conv(F))

    def _c(self) -> _DenseOperator:
        return _DenseOperator(self.nx, self.ny, self.D.data_ptr(), self.E.data_ptr(), self.F.data_ptr())

    @property
    def n(self):
        return self.nx * self.ny


class Handle:
    def __init__(self, ptr: int, op: Operator, precision: int):
        self.ptr = ptr
        if isinstance(op, Operator3d):   # block = plane
            self.nx, self.ny = op.nx * op.ny, op.nz
        else:
            self.nx, self.ny = op.nx, op.ny
        self.precision = precision

    def __del__(self):
        if getattr(self, "ptr", None) and _lib is not None:
            _lib.acr_destroy(self.ptr)
            self.ptr = None


def _as_colmajor(B, n):
    """(N,) or (N, nrhs) float64 CUDA tensor -> contiguous (nrhs, N) tensor (= column-major N x nrhs)."""
    import torch
    if B.dtype != torch.float64 or not B.is_cuda:
        raise TypeError("vectors must be float64 CUDA tensors")
    if B.dim() == 1:
        B = B.reshape(n, 1)
    if B.shape[0] != n:
        raise ValueError(f"vector has {B.shape[0]} rows, operator has {n} unknowns")
    return B.t().contiguous()


def acr_factor(op: Operator, leaf: int, eps: float, precision="fp64", max_rank: int = 0,
               inner_eps: float = 0.0, stop_blocks: int = 1, stream=None) -> Handle:
    lib = load()
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    opt = _Options(int(leaf), float(eps), prec, int(max_rank), float(inner_eps), int(stop_blocks))
    out = ctypes.c_void_p()
    _check(lib.acr_factor(ctypes.byref(op._c()), ctypes.byref(opt), _stream(stream), ctypes.byref(out)))
    return Handle(out.value, op, prec)


def acr_factor_3d(op: Operator3d, leaf: int, eps: float, precision="fp64", max_rank: int = 0,
                  inner_eps: float = 0.0, stop_blocks: int = 1, stream=None) -> Handle:
    """Factor a 3-D operator (block = plane, exact HODLR plane operators at level 0)."""
    lib = load()
    lib.acr_factor_3d.argtypes = [ctypes.POINTER(_Operator3d), ctypes.POINTER(_Options), ctypes.c_void_p,
                                  ctypes.POINTER(ctypes.c_void_p)]
    lib.acr_factor_3d.restype = ctypes.c_int
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    opt = _Options(int(leaf), float(eps), prec, int(max_rank), float(inner_eps), int(stop_blocks))
    out = ctypes.c_void_p()
    _check(lib.acr_factor_3d(ctypes.byref(op._c()), ctypes.byref(opt), _stream(stream), ctypes.byref(out)))
    return Handle(out.value, op, prec)


def acr_factor_dense(op: "DenseOperator", leaf: int, eps: float, precision="fp64", max_rank: int = 0,
                     stop_blocks: int = 1, stream=None) -> Handle:
    """Factor an operator given by dense blocks (each block compressed to eps first)."""
    lib = load()
    lib.acr_factor_dense.argtypes = [ctypes.POINTER(_DenseOperator), ctypes.POINTER(_Options), ctypes.c_void_p,
                                     ctypes.POINTER(ctypes.c_void_p)]
    lib.acr_factor_dense.restype = ctypes.c_int
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    opt = _Options(int(leaf), float(eps), prec, int(max_rank), 0.0, int(stop_blocks))
    out = ctypes.c_void_p()
    _check(lib.acr_factor_dense(ctypes.byref(op._c()), ctypes.byref(opt), _stream(stream), ctypes.byref(out)))
    return Handle(out.value, op, prec)


def acr_factor_batched(ops, leaf: int, eps: float, precision="fp64", max_rank: int = 0,
                       inner_eps: float = 0.0, stop_blocks: int = 1, stream=None):
    """Factor several independent problems in one lockstep pass; returns one Handle per operator."""
    lib = load()
    lib.acr_factor_batched.argtypes = [ctypes.POINTER(_Operator), ctypes.POINTER(_Options), ctypes.c_int32,
                                       ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
    lib.acr_factor_batched.restype = ctypes.c_int
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    opt = _Options(int(leaf), float(eps), prec, int(max_rank), float(inner_eps), int(stop_blocks))
    n = len(ops)
    arr = (_Operator * n)(*[o._c() for o in ops])
    out = (ctypes.c_void_p * n)()
    _check(lib.acr_factor_batched(arr, ctypes.byref(opt), n, _stream(stream), out))
    return [Handle(out[i], ops[i], prec) for i in range(n)]


def acr_solve_batched(handles, Bs, stream=None):
    """X_p = M_p^{-1} B_p for several handles at once (shared launches); returns the list of X."""
    import torch
    lib = load()
    lib.acr_solve_batched.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                      ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int32),
                                      ctypes.c_int32, ctypes.c_void_p]
    lib.acr_solve_batched.restype = ctypes.c_int
    n = len(handles)
    cols = [_as_colmajor(B, h.nx * h.ny) for h, B in zip(handles, Bs)]
    outs = [torch.empty_like(c) for c in cols]
    hp = (ctypes.c_void_p * n)(*[h.ptr for h in handles])
    bp = (ctypes.c_void_p * n)(*[c.data_ptr() for c in cols])
    xp = (ctypes.c_void_p * n)(*[x.data_ptr() for x in outs])
    nr = (ctypes.c_int32 * n)(*[c.shape[0] for c in cols])
    _check(lib.acr_solve_batched(hp, bp, xp, nr, n, _stream(stream)))
    res = []
    for B, X in zip(Bs, outs):
        X = X.t()
        res.append(X.reshape(B.shape) if B.dim() == 1 else X)
    return res


def acr_solve(h: Handle, B, stream=None):
    import torch
    lib = load()
    n = h.nx * h.ny
    Bc = _as_colmajor(B, n)
    X = torch.empty_like(Bc)
    _check(lib.acr_solve(h.ptr, Bc.data_ptr(), X.data_ptr(), Bc.shape[0], _stream(stream)))
    X = X.t()
    return X.reshape(B.shape) if B.dim() == 1 else X


def acr_solve_refined(h: Handle, op: Operator, B, tol: float = 1e-10, maxit: int = 50, stream=None,
                      raise_on_fail: bool = True):
    import torch
    lib = load()
    n = h.nx * h.ny
    Bc = _as_colmajor(B, n)
    X = torch.empty_like(Bc)
    its = ctypes.c_int32(0)
    rel = ctypes.c_double(0.0)
    fn = lib.acr_solve_refined
    if isinstance(op, Operator3d):
        fn = lib.acr_solve_refined_3d
        fn.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Operator3d)] + lib.acr_solve_refined.argtypes[2:]
        fn.restype = ctypes.c_int
    code = fn(h.ptr, ctypes.byref(op._c()), Bc.data_ptr(), X.data_ptr(), Bc.shape[0],
              float(tol), int(maxit), ctypes.byref(its), ctypes.byref(rel), _stream(stream))
    if code != 0 and (raise_on_fail or code != 4):
        _check(code)
    X = X.t()
    return (X.reshape(B.shape) if B.dim() == 1 else X), its.value, rel.value


def acr_solve_krylov(h: Handle, op: Operator, B, tol: float = 1e-10, maxit: int = 100, restart: int = 20,
                     stream=None, raise_on_fail: bool = True):
    """Restarted FGMRES right-preconditioned by the ACR factor; returns (X, preconditioner
    applications, relative residual)."""
    import torch
    lib = load()
    n = h.nx * h.ny
    Bc = _as_colmajor(B, n)
    X = torch.empty_like(Bc)
    its = ctypes.c_int32(0)
    rel = ctypes.c_double(0.0)
    fn = lib.acr_solve_krylov
    if isinstance(op, Operator3d):
        fn = lib.acr_solve_krylov_3d
        fn.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Operator3d)] + lib.acr_solve_krylov.argtypes[2:]
        fn.restype = ctypes.c_int
    code = fn(h.ptr, ctypes.byref(op._c()), Bc.data_ptr(), X.data_ptr(), Bc.shape[0],
              float(tol), int(maxit), int(restart), ctypes.byref(its), ctypes.byref(rel), _stream(stream))
    if code != 0 and (raise_on_fail or code != 4):
        _check(code)
    X = X.t()
    return (X.reshape(B.shape) if B.dim() == 1 else X), its.value, rel.value


def acr_residual(op: Operator, X, B, stream=None):
    import torch
    lib = load()
    Xc = _as_colmajor(X, op.n)
    Bc = _as_colmajor(B, op.n)
    R = torch.empty_like(Bc)
    fn = lib.acr_residual
    if isinstance(op, Operator3d):
        fn = lib.acr_residual_3d
        fn.argtypes = [ctypes.POINTER(_Operator3d)] + lib.acr_residual.argtypes[1:]
        fn.restype = ctypes.c_int
    _check(fn(ctypes.byref(op._c()), Xc.data_ptr(), Bc.data_ptr(), R.data_ptr(), Bc.shape[0], _stream(stream)))
    R = R.t()
    return R.reshape(B.shape) if B.dim() == 1 else R


def acr_get_info(h: Handle) -> dict:
    lib = load()
    inf = _Info()
    _check(lib.acr_get_info(h.ptr, ctypes.byref(inf)))
    d = {f: getattr(inf, f) for f, _ in _Info._fields_ if f not in ("level_max_rank", "level_mean_rank")}
    d["level_max_rank"] = list(inf.level_max_rank)[: inf.levels]
    d["level_mean_rank"] = list(inf.level_mean_rank)[: inf.levels]
    return d


def acr_launch_count() -> int:
    """Kernel launches the calling thread has issued through the library so far."""
    lib = load()
    lib.acr_launch_count.restype = ctypes.c_int64
    return int(lib.acr_launch_count())


def acr_set_solve_mode(mode: int = 0, wait_limit: int = 0):
    """Solve passes: 0 = grouped launches per step from descriptors kept on
    the device (default), 1 = the levels of at most 16 blocks as one
    persistent launch, 2 = the whole pass as one persistent launch, 3 =
    grouped launches planned on every call (all give the same bits);
    wait_limit > 0 polls per wait, 0 the default, < 0 every dependent task
    gives up (the pass then returns NaN)."""
    lib = load()
    lib.acr_set_solve_mode.argtypes = [ctypes.c_int32, ctypes.c_int64]
    lib.acr_set_solve_mode.restype = ctypes.c_int
    _check(lib.acr_set_solve_mode(int(mode), int(wait_limit)))


def acr_get_block(h: Handle, level: int, which: int, k: int, stream=None) -> np.ndarray:
    lib = load()
    out = np.zeros(h.nx * h.nx, dtype=np.float64)
    _check(lib.acr_get_block(h.ptr, level, which, k, out.ctypes.data, _stream(stream)))
    return out.reshape(h.nx, h.nx, order="F")


def acr_destroy(h: Handle):
    if h.ptr:
        _check(load().acr_destroy(h.ptr))
        h.ptr = None


def acr_trim_pool():
    _check(load().acr_trim_pool())


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
_allocator_refs = None   # keeps the installed ctypes callbacks alive


def acr_set_allocator(alloc=None, free=None):
    """Install Python callables alloc(nbytes, stream_handle) -> device pointer (int) and
    free(ptr, stream_handle) as the library's device-memory source (None, None restores
    hipMalloc).  Fails with ACR_ERR_INVALID_ARG while a handle is alive."""
    global _allocator_refs
    lib = load()
    lib.acr_set_allocator.argtypes = [_ALLOC_FN, _FREE_FN]
    lib.acr_set_allocator.restype = ctypes.c_int
    if alloc is None and free is None:
        _check(lib.acr_set_allocator(ctypes.cast(None, _ALLOC_FN), ctypes.cast(None, _FREE_FN)))
        _allocator_refs = None
        return

    def _a(nbytes, stream):
        try:
            return int(alloc(int(nbytes), stream or 0))
        except Exception:
            return None

    def _f(ptr, stream):
        try:
            free(int(ptr), stream or 0)
        except Exception:
            pass

    refs = (_ALLOC_FN(_a), _FREE_FN(_f))
    _check(lib.acr_set_allocator(refs[0], refs[1]))
    _allocator_refs = refs


def use_torch_allocator():
    """Take every device allocation of the library from PyTorch's caching allocator
    (torch.cuda.caching_allocator_alloc / _delete on the library's stream)."""
    import torch

    def alloc(nbytes, stream):
        return torch.cuda.caching_allocator_alloc(nbytes, stream=int(stream))

    def free(ptr, stream):
        torch.cuda.caching_allocator_delete(ptr)

    acr_set_allocator(alloc, free)


KERNEL_CLASSES = ["gemm", "inverse", "qr", "applyq", "svd", "matvec", "copy", "other"]


def acr_profile_start(classes=None):
    """Time every launch of the given kernel classes (names or indices; None = all)."""
    lib = load()
    lib.acr_profile_start.argtypes = [ctypes.c_uint32]
    lib.acr_profile_start.restype = ctypes.c_int
    if classes is None:
        mask = (1 << len(KERNEL_CLASSES)) - 1
    else:
        mask = 0
        for c in classes:
            mask |= 1 << (KERNEL_CLASSES.index(c) if isinstance(c, str) else int(c))
    _check(lib.acr_profile_start(mask))


def acr_profile_read(cls) -> dict:
    lib = load()
    lib.acr_profile_read.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    lib.acr_profile_read.restype = ctypes.c_int
    idx = KERNEL_CLASSES.index(cls) if isinstance(cls, str) else int(cls)
    n, ms, fl, by = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib.acr_profile_read(idx, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(fl), ctypes.byref(by)))
    return {"class": KERNEL_CLASSES[idx], "launches": n.value, "total_ms": ms.value, "flops": fl.value,
            "bytes": by.value}


def acr_profile_report() -> dict:
    """Timing of the launches recorded since acr_profile_start:
    {"stages": [(stage, level, class, launches, ms, flops, bytes)],
     "kernels": [(name, class, launches, ms, flops, bytes)],
     "paths": {kernel path: batched problems planned on it}}."""
    lib = load()
    lib.acr_profile_report.argtypes = [ctypes.c_char_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
    lib.acr_profile_report.restype = ctypes.c_int
    need = ctypes.c_int64(0)
    _check(lib.acr_profile_report(None, 0, ctypes.byref(need)))
    buf = ctypes.create_string_buffer(int(need.value) + 1)
    _check(lib.acr_profile_report(buf, len(buf), ctypes.byref(need)))
    out = {"stages": [], "kernels": []}
    for line in buf.value.decode().splitlines():
        f = line.split("\t")
        if f[0] == "stage":
            out["stages"].append((f[1], int(f[2]), f[3], int(f[4]), float(f[5]), float(f[6]), float(f[7])))
        elif f[0] == "kernel":
            out["kernels"].append((f[1], f[2], int(f[3]), float(f[4]), float(f[5]), float(f[6])))
        elif f[0] == "path":
            out.setdefault("paths", {})[f[1]] = int(f[2])
        elif f[0] == "stagekernel":
            out.setdefault("stage_kernels", []).append((f[1], f[2], int(f[3]), float(f[4]), float(f[5]),
                                                        float(f[6])))
    return out


class _ServerConfig(ctypes.Structure):
    _fields_ = [("memory_budget", ctypes.c_int64), ("tol", ctypes.c_double), ("maxit", ctypes.c_int32)]


class _ServerInfo(ctypes.Structure):
    _fields_ = [("requests", ctypes.c_int64), ("rhs", ctypes.c_int64), ("steps", ctypes.c_int64),
                ("factorizations", ctypes.c_int64), ("evictions", ctypes.c_int64),
                ("resident_bytes", ctypes.c_int64), ("peak_resident_bytes", ctypes.c_int64),
                ("seconds", ctypes.c_double), ("requests_per_s", ctypes.c_double), ("rhs_per_s", ctypes.c_double),
                ("latency_p50_ms", ctypes.c_double), ("latency_p99_ms", ctypes.c_double),
                ("latency_max_ms", ctypes.c_double), ("busy_s", ctypes.c_double)]


class Server:
    """The library's serving loop (acr_server_*): resident factors under a memory budget,
    requests refined to `tol` with continuous batching of their refinement steps."""

    def __init__(self, memory_budget: int, tol: float = 1e-10, maxit: int = 50):
        lib = load()
        P = ctypes.c_void_p
        lib.acr_server_create.argtypes = [ctypes.POINTER(_ServerConfig), ctypes.POINTER(P)]
        lib.acr_server_add_operator.argtypes = [P, ctypes.POINTER(_Operator), ctypes.POINTER(_Options),
                                                ctypes.POINTER(ctypes.c_int32)]
        lib.acr_server_submit.argtypes = [P, ctypes.c_int32, P, P, ctypes.c_int32, P, ctypes.POINTER(ctypes.c_int64)]
        lib.acr_server_wait.argtypes = [P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        lib.acr_server_stats.argtypes = [P, ctypes.c_int32, ctypes.POINTER(_ServerInfo)]
        lib.acr_server_destroy.argtypes = [P]
        for n in ("acr_server_create", "acr_server_add_operator", "acr_server_submit", "acr_server_wait",
                  "acr_server_stats", "acr_server_destroy"):
            getattr(lib, n).restype = ctypes.c_int
        self._lib = lib
        self._ptr = P()
        cfg = _ServerConfig(int(memory_budget), float(tol), int(maxit))
        _check(lib.acr_server_create(ctypes.byref(cfg), ctypes.byref(self._ptr)))
        self._ops = []
        self._live = {}   # request id -> (B, X) kept alive until waited for

    def add_operator(self, op: Operator, leaf: int, eps: float, precision="mixed", max_rank: int = 0) -> int:
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        opt = _Options(int(leaf), float(eps), prec, int(max_rank), 0.0, 1)
        oid = ctypes.c_int32(0)
        _check(self._lib.acr_server_add_operator(self._ptr, ctypes.byref(op._c()), ctypes.byref(opt), ctypes.byref(oid)))
        self._ops.append(op.n)
        return oid.value

    def submit(self, op_id: int, B, stream=None) -> int:
        import torch
        if not 0 <= int(op_id) < len(self._ops):
            raise ACRError(1, "unknown operator id")
        n = self._ops[op_id]
        Bc = _as_colmajor(B, n)
        X = torch.empty_like(Bc)
        rid = ctypes.c_int64(0)
        _check(self._lib.acr_server_submit(self._ptr, int(op_id), Bc.data_ptr(), X.data_ptr(), Bc.shape[0],
                                           _stream(stream), ctypes.byref(rid)))
        self._live[rid.value] = (B, Bc, X)
        return rid.value

    def wait(self, rid: int, raise_on_fail: bool = True):
        """Returns (X shaped like B, refinement corrections, relative residual, latency in ms)."""
        its, rel, lat = ctypes.c_int32(0), ctypes.c_double(0.0), ctypes.c_double(0.0)
        code = self._lib.acr_server_wait(self._ptr, int(rid), ctypes.byref(its), ctypes.byref(rel), ctypes.byref(lat))
        B, Bc, X = self._live.pop(rid)
        if code != 0 and (raise_on_fail or code != 4):
            _check(code)
        X = X.t()
        return (X.reshape(B.shape) if B.dim() == 1 else X), its.value, rel.value, lat.value

    def stats(self, reset: bool = False) -> dict:
        inf = _ServerInfo()
        _check(self._lib.acr_server_stats(self._ptr, 1 if reset else 0, ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in _ServerInfo._fields_}

    def close(self):
        if self._ptr:
            _check(self._lib.acr_server_destroy(self._ptr))
            self._ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _tune_lib():
    lib = load()
    lib.acr_tune_record.argtypes = [ctypes.c_int32]
    lib.acr_tune_run.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]
    lib.acr_tune_enable.argtypes = [ctypes.c_int32]
    lib.acr_tune_save.argtypes = [ctypes.c_char_p]
    lib.acr_tune_load.argtypes = [ctypes.c_char_p]
    for n in ("acr_tune_record", "acr_tune_run", "acr_tune_enable", "acr_tune_save", "acr_tune_load",
              "acr_tune_clear"):
        getattr(lib, n).restype = ctypes.c_int
    return lib


def acr_tune_record(on: bool = True):
    """Start or stop noting the shape keys the library meets (autotuner)."""
    _check(_tune_lib().acr_tune_record(1 if on else 0))


def acr_tune_run(stream=None) -> int:
    """Measure every noted key without a table entry; returns the entries added."""
    n = ctypes.c_int32(0)
    _check(_tune_lib().acr_tune_run(_stream(stream), ctypes.byref(n)))
    return n.value


def acr_tune_enable(on: bool = True):
    _check(_tune_lib().acr_tune_enable(1 if on else 0))


def acr_tune_save(path):
    _check(_tune_lib().acr_tune_save(os.fsencode(str(path))))


def acr_tune_load(path):
    _check(_tune_lib().acr_tune_load(os.fsencode(str(path))))


def acr_tune_clear():
    _check(_tune_lib().acr_tune_clear())

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
                ("max_rank", ctypes.c_int32), ("inner_eps", ctypes.c_double)]


class _Info(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("leaf", ctypes.c_int32),
                ("depth", ctypes.c_int32), ("levels", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("eps", ctypes.c_double), ("factor_bytes", ctypes.c_int64), ("max_rank", ctypes.c_int32),
                ("level_max_rank", ctypes.c_int32 * 40), ("factor_flops", ctypes.c_double),
                ("solve_bytes", ctypes.c_double), ("solve_flops_per_rhs", ctypes.c_double)]


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


class Handle:
    def __init__(self, ptr: int, op: Operator, precision: int):
        self.ptr = ptr
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
               inner_eps: float = 0.0, stream=None) -> Handle:
    lib = load()
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    opt = _Options(int(leaf), float(eps), prec, int(max_rank), float(inner_eps))
    out = ctypes.c_void_p()
    _check(lib.acr_factor(ctypes.byref(op._c()), ctypes.byref(opt), _stream(stream), ctypes.byref(out)))
    return Handle(out.value, op, prec)


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
    code = lib.acr_solve_refined(h.ptr, ctypes.byref(op._c()), Bc.data_ptr(), X.data_ptr(), Bc.shape[0],
                                 float(tol), int(maxit), ctypes.byref(its), ctypes.byref(rel),
                                 _stream(stream))
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
    code = lib.acr_solve_krylov(h.ptr, ctypes.byref(op._c()), Bc.data_ptr(), X.data_ptr(), Bc.shape[0],
                                float(tol), int(maxit), int(restart), ctypes.byref(its), ctypes.byref(rel),
                                _stream(stream))
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
    _check(lib.acr_residual(ctypes.byref(op._c()), Xc.data_ptr(), Bc.data_ptr(), R.data_ptr(),
                            Bc.shape[0], _stream(stream)))
    R = R.t()
    return R.reshape(B.shape) if B.dim() == 1 else R


def acr_get_info(h: Handle) -> dict:
    lib = load()
    inf = _Info()
    _check(lib.acr_get_info(h.ptr, ctypes.byref(inf)))
    d = {f: getattr(inf, f) for f, _ in _Info._fields_ if f != "level_max_rank"}
    d["level_max_rank"] = list(inf.level_max_rank)[: inf.levels]
    return d


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
     "kernels": [(name, class, launches, ms, flops, bytes)]}."""
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
        elif f[0] == "stagekernel":
            out.setdefault("stage_kernels", []).append((f[1], f[2], int(f[3]), float(f[4]), float(f[5]),
                                                        float(f[6])))
    return out

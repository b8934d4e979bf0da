"""acr_solve_noalloc: the allocation-free variant of acr_solve (scratch array
inside the library) gives the same bits as acr_solve, on two calls in a row
(the second with a smaller problem), takes no device memory from the
allocator, and rejects a solve larger than its scratch before doing any work."""
import ctypes
import gc

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _op(acr, st):
    return acr.Operator.from_arrays(st.nx, st.ny, *st.arrays())


def _noalloc(acr, h, B):
    import torch
    lib = acr.load()
    lib.acr_solve_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                      ctypes.c_void_p]
    lib.acr_solve_noalloc.restype = ctypes.c_int
    n = h.nx * h.ny
    Bc = B.reshape(n, -1).t().contiguous()
    X = torch.empty_like(Bc)
    code = lib.acr_solve_noalloc(h.ptr, Bc.data_ptr(), X.data_ptr(), Bc.shape[0], acr._stream())
    return code, X.t().reshape(B.shape)


def test_noalloc_matches_solve_two_calls(gpu):
    import torch
    cases = [(W.varkappa(256), 64, "mixed", 4), (W.convdiff(96, 40), 24, "fp64", 2)]   # second call smaller
    hs = []
    for st, leaf, prec, nrhs in cases:
        h = gpu.acr_factor(_op(gpu, st), leaf, 1e-8, prec)
        B = torch.from_numpy(W.rhs(st.n, nrhs, seed=31)).cuda()
        ref = gpu.acr_solve(h, B).cpu().numpy()
        code, X = _noalloc(gpu, h, B)
        assert gpu.STATUS[code] == "ACR_OK", gpu.load().acr_last_error()
        assert np.array_equal(X.cpu().numpy(), ref), f"{st.name} {st.nx}: differs from acr_solve"
        hs.append(h)
    # the first problem again after the smaller one (the scratch holds the last call's contents)
    st, leaf, prec, nrhs = cases[0]
    B = torch.from_numpy(W.rhs(st.n, nrhs, seed=32)).cuda()
    code, X = _noalloc(gpu, hs[0], B)
    assert gpu.STATUS[code] == "ACR_OK"
    assert np.array_equal(X.cpu().numpy(), gpu.acr_solve(hs[0], B).cpu().numpy())


def test_noalloc_takes_no_device_memory(gpu):
    import torch
    calls = {"alloc": 0}

    def alloc(nbytes, stream):
        calls["alloc"] += 1
        return torch.cuda.caching_allocator_alloc(nbytes, stream=int(stream))

    def free(ptr, stream):
        torch.cuda.caching_allocator_delete(ptr)

    gc.collect()
    gpu.acr_set_allocator(alloc, free)
    try:
        st = W.varkappa(128)
        h = gpu.acr_factor(_op(gpu, st), 32, 1e-8, "fp64")
        B = torch.from_numpy(W.rhs(st.n, 3, seed=33)).cuda()
        X0 = torch.empty_like(B.t().contiguous())   # output allocated before counting
        torch.cuda.synchronize()
        before = calls["alloc"]
        code, X = _noalloc(gpu, h, B)
        torch.cuda.synchronize()
        assert gpu.STATUS[code] == "ACR_OK"
        assert calls["alloc"] == before
        del X0
        gpu.acr_destroy(h)
    finally:
        gc.collect()
        gpu.acr_set_allocator(None, None)


def test_noalloc_rejects_oversized_solve(gpu):
    import torch
    st = W.varkappa(512)
    h = gpu.acr_factor(_op(gpu, st), 64, 1e-6, "fp64")
    B = torch.from_numpy(W.rhs(st.n, 8, seed=34)).cuda()
    code, X = _noalloc(gpu, h, B)
    assert gpu.STATUS[code] == "ACR_ERR_INVALID_ARG"
    assert "maximum" in gpu.load().acr_last_error().decode()

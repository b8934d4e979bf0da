"""Runtime behaviour of the library on the GPU: streams, threads and the
allocator hook of the boundary.  Results are compared bitwise (FP64)."""
import gc
import threading

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _op(acr, st):
    return acr.Operator.from_arrays(st.nx, st.ny, *st.arrays())


def test_two_streams_match_sequential(gpu):
    """Two handles solved on two streams at once give the same bits as the
    same solves one after the other on the default stream (no workspace is
    shared between the streams while in use)."""
    import torch
    sa, sb = W.varkappa(128), W.convdiff(96, 40)
    ha = gpu.acr_factor(_op(gpu, sa), 32, 1e-8, "fp64")
    hb = gpu.acr_factor(_op(gpu, sb), 24, 1e-8, "fp64")
    ba = torch.from_numpy(W.rhs(sa.n, 3, seed=1)).cuda()
    bb = torch.from_numpy(W.rhs(sb.n, 3, seed=2)).cuda()
    xa0 = gpu.acr_solve(ha, ba).cpu().numpy()
    xb0 = gpu.acr_solve(hb, bb).cpu().numpy()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    outs = []
    for _ in range(4):
        with torch.cuda.stream(s1):
            xa = gpu.acr_solve(ha, ba, stream=s1)
        with torch.cuda.stream(s2):
            xb = gpu.acr_solve(hb, bb, stream=s2)
        outs.append((xa, xb))
    torch.cuda.synchronize()
    for xa, xb in outs:
        assert np.array_equal(xa.cpu().numpy(), xa0)
        assert np.array_equal(xb.cpu().numpy(), xb0)


def test_two_threads_match_sequential(gpu):
    """Two host threads factor and solve different problems at the same time."""
    import torch
    probs = [(W.varkappa(64), 16), (W.poisson(96), 24)]
    ref = []
    for st, leaf in probs:
        h = gpu.acr_factor(_op(gpu, st), leaf, 1e-9, "fp64")
        ref.append(gpu.acr_solve(h, torch.from_numpy(W.rhs(st.n, 2, seed=5)).cuda()).cpu().numpy())
        gpu.acr_destroy(h)
    got = [None, None]
    errs = []

    def work(i):
        try:
            st, leaf = probs[i]
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                for _ in range(3):
                    h = gpu.acr_factor(_op(gpu, st), leaf, 1e-9, "fp64", stream=s)
                    x = gpu.acr_solve(h, torch.from_numpy(W.rhs(st.n, 2, seed=5)).cuda(), stream=s)
                    s.synchronize()
                    got[i] = x.cpu().numpy()
                    gpu.acr_destroy(h)
        except Exception as e:   # reported by the main thread
            errs.append(e)

    th = [threading.Thread(target=work, args=(i,)) for i in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errs, errs
    for i in range(2):
        assert np.array_equal(got[i], ref[i])


def test_torch_allocator_hook(gpu):
    """With acr_set_allocator pointing at PyTorch's caching allocator the
    library takes its device memory from torch, and results are unchanged."""
    import torch
    st = W.varkappa(128)
    b = torch.from_numpy(W.rhs(st.n, 1, seed=3)).cuda()
    h = gpu.acr_factor(_op(gpu, st), 32, 1e-8, "fp64")
    x0 = gpu.acr_solve(h, b).cpu().numpy()
    # a live handle blocks switching the memory source
    with pytest.raises(gpu.ACRError) as ei:
        gpu.use_torch_allocator()
    assert ei.value.name == "ACR_ERR_INVALID_ARG"
    gpu.acr_destroy(h)
    gc.collect()
    before = torch.cuda.memory_allocated()
    gpu.use_torch_allocator()
    try:
        h = gpu.acr_factor(_op(gpu, st), 32, 1e-8, "fp64")
        during = torch.cuda.memory_allocated()
        x1 = gpu.acr_solve(h, b).cpu().numpy()
        info = gpu.acr_get_info(h)
        assert during - before >= info["factor_bytes"]
        assert np.array_equal(x0, x1)
        gpu.acr_destroy(h)
    finally:
        gc.collect()
        gpu.acr_set_allocator(None, None)
    assert torch.cuda.memory_allocated() <= before


def test_poisoned_memory_batched(gpu):
    """Every fresh device block the library takes is filled with NaN bytes
    (0xFF) by the allocator hook: a factorisation that read memory it had not
    written (a zero fill that never ran, a dummy matrix left unset) would carry
    NaN into its result.  A batch of mixed sizes, factored and solved twice
    with the pool trimmed in between, gives the same bits as without poison,
    in FP64 and in the mixed form."""
    import torch
    rng = np.random.default_rng(W.seed_for(3, 950))
    sides = rng.choice([64, 96, 128], size=40)
    probs = [W.poisson(int(s)) if i % 2 else W.varkappa(int(s), seed=W.seed_for(3, 960 + i))
             for i, s in enumerate(sides)]
    ops = [_op(gpu, st) for st in probs]
    Bs = [torch.from_numpy(W.rhs(st.n, 3, seed=W.seed_for(3, 990 + i))).cuda() for i, st in enumerate(probs)]

    def run(prec):
        hs = gpu.acr_factor_batched(ops, 32, 1e-8, prec)
        xs = [x.cpu().numpy() for x in gpu.acr_solve_batched(hs, Bs)]
        for h in hs:
            gpu.acr_destroy(h)
        return xs

    ref = {p: run(p) for p in ("fp64", "mixed")}
    gc.collect()
    gpu.acr_trim_pool()
    live = {}

    def alloc(nbytes, stream):
        t = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        t.fill_(255)
        live[t.data_ptr()] = t
        return t.data_ptr()

    def free(ptr, stream):
        live.pop(ptr, None)

    gpu.acr_set_allocator(alloc, free)
    try:
        for rep in range(2):
            for p in ("fp64", "mixed"):
                xs = run(p)
                for i, (a, b) in enumerate(zip(xs, ref[p])):
                    assert np.all(np.isfinite(a)), f"{p} rep {rep}: problem {i} has non-finite values"
                    assert np.array_equal(a, b), f"{p} rep {rep}: problem {i} differs under poisoned memory"
            gc.collect()
            gpu.acr_trim_pool()
    finally:
        gc.collect()
        gpu.acr_trim_pool()
        gpu.acr_set_allocator(None, None)


def _poisoned(gpu, torch):
    """Allocator hook handing out NaN-filled (0xFF) device blocks."""
    live = {}

    def alloc(nbytes, stream):
        t = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        t.fill_(255)
        live[t.data_ptr()] = t
        return t.data_ptr()

    def free(ptr, stream):
        live.pop(ptr, None)

    return alloc, free


def test_poisoned_memory_entry_points(gpu):
    """The same check for the other factor and solve paths: solo factors of both
    precisions with refinement and FGMRES, early stop, dense-block and 3-D
    operators.  Every result equals the one computed on ordinary memory."""
    import torch
    st = W.varkappa(256)
    op = _op(gpu, st)
    b = torch.from_numpy(W.rhs(st.n, 2, seed=5)).cuda()
    s3 = W.varkappa3d(16)
    op3 = gpu.Operator3d.from_arrays(s3.nx, s3.ny, s3.nz, *s3.arrays())
    b3 = torch.from_numpy(W.rhs(s3.n, 1, seed=6)).cuda()
    sd = W.varkappa(64)
    from oracle import direct
    D, E, F = direct.blocks(sd)
    dop = gpu.DenseOperator.from_blocks(D, E, F)
    bd = torch.from_numpy(W.rhs(sd.n, 1, seed=7)).cuda()

    def run():
        out = []
        for prec in ("fp64", "mixed"):
            h = gpu.acr_factor(op, 64, 1e-6, prec)
            out.append(gpu.acr_solve(h, b).cpu().numpy())
            out.append(gpu.acr_solve_refined(h, op, b, tol=1e-10)[0].cpu().numpy())
            out.append(gpu.acr_solve_krylov(h, op, b, tol=1e-10)[0].cpu().numpy())
            gpu.acr_destroy(h)
            h = gpu.acr_factor(op, 64, 1e-6, prec, stop_blocks=4)
            out.append(gpu.acr_solve(h, b).cpu().numpy())
            gpu.acr_destroy(h)
            h = gpu.acr_factor_3d(op3, 32, 1e-4, prec)
            out.append(gpu.acr_solve_krylov(h, op3, b3, tol=1e-10)[0].cpu().numpy())
            gpu.acr_destroy(h)
            h = gpu.acr_factor_dense(dop, 16, 1e-8, prec)
            out.append(gpu.acr_solve(h, bd).cpu().numpy())
            gpu.acr_destroy(h)
        return out

    ref = run()
    gc.collect()
    gpu.acr_trim_pool()
    alloc, free = _poisoned(gpu, torch)
    gpu.acr_set_allocator(alloc, free)
    try:
        got = run()
    finally:
        gc.collect()
        gpu.acr_trim_pool()
        gpu.acr_set_allocator(None, None)
    for i, (a, r) in enumerate(zip(got, ref)):
        assert np.all(np.isfinite(a)), f"result {i} has non-finite values under poisoned memory"
        assert np.array_equal(a, r), f"result {i} differs under poisoned memory"

"""The execution modes of a solve pass against the default (grouped launches
from descriptors kept on the device): the persistent pass (tasks with
bounded dependency waits in one launch: the whole pass, or the levels of at
most 16 blocks) and the grouped launches planned on every call.  All run the
same device arithmetic in the same order, so every solution must agree bit
for bit, alone and batched, in FP64 and in the mixed form.  The forced
failure path (every dependent task gives up) must end every kernel normally
and return NaN, and the next pass must be correct again."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _op(acr, st):
    return acr.Operator.from_arrays(st.nx, st.ny, *st.arrays())


def _solve_both(gpu, h, B, mode):
    gpu.acr_set_solve_mode(0)
    xg = gpu.acr_solve(h, B).cpu().numpy()
    gpu.acr_set_solve_mode(mode)
    try:
        c0 = gpu.acr_launch_count()
        xp = gpu.acr_solve(h, B).cpu().numpy()
        n = gpu.acr_launch_count() - c0
        xp2 = gpu.acr_solve(h, B).cpu().numpy()   # the cached task list again
    finally:
        gpu.acr_set_solve_mode(0)
    return xg, xp, xp2, n


CASES = [
    # (workload, side, block rows, leaf, eps, nrhs)
    ("poisson", 64, 64, 16, 1e-10, 1),
    ("varkappa", 128, 77, 32, 1e-8, 3),      # odd block count, leaf < 64
    ("varkappa", 256, 40, 64, 1e-6, 8),      # leaf of 64: whole-wave rows
    ("convdiff", 128, 128, 64, 1e-7, 2),     # non-symmetric, one leaf per block
    ("varkappa", 96, 96, 24, 1e-8, 5),       # leaf 24, depth 2
]


@pytest.mark.parametrize("mode", [1, 2, 3])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}{c[1]}x{c[2]}-leaf{c[3]}-rhs{c[5]}")
def test_persistent_equals_grouped(gpu, case, prec, mode):
    import torch
    kind, n, rows, leaf, eps, nrhs = case
    st = {"poisson": W.poisson, "varkappa": W.varkappa, "convdiff": W.convdiff}[kind](n)
    if rows < n:
        st = W.strip(st, rows)
    print(f"[case] {kind} {n}x{rows} leaf {leaf} eps {eps} nrhs {nrhs} {prec} mode {mode}", flush=True)
    h = gpu.acr_factor(_op(gpu, st), leaf, eps, prec)
    B = torch.from_numpy(W.rhs(st.n, nrhs, seed=W.seed_for(2, 700 + rows))).cuda()
    xg, xp, xp2, launches = _solve_both(gpu, h, B, mode)
    assert np.isfinite(xp).all()
    assert np.array_equal(xg, xp), f"max diff {np.abs(xg - xp).max():.3e}"
    assert np.array_equal(xp, xp2)
    # mode 1: levels of more than 16 blocks run as two grouped launches per
    # step (two steps per level and direction); the rest of the pass is one
    # persistent launch next to the fill, the layout copies and the check
    wide, m = 0, rows
    while mode == 1 and m > 16:
        wide += 1
        m //= 2
    if mode in (1, 2):
        assert launches <= 6 + 8 * wide, launches
    # the kept pass: the same launches as planning on every call, nothing more
    c0 = gpu.acr_launch_count()
    gpu.acr_solve(h, B)
    kept = gpu.acr_launch_count() - c0
    if mode == 3:
        assert kept == launches, (kept, launches)
    gpu.acr_destroy(h)


def test_persistent_batched_equals_solo(gpu):
    """Several factors of different sizes, leaves and right-hand-side counts
    in one solve call (launch groups by projection slots and row form)."""
    import torch
    probs = [(W.poisson(64), 16, 1), (W.strip(W.varkappa(128), 33), 32, 4), (W.strip(W.varkappa(256), 20), 64, 8),
             (W.poisson(96), 24, 2), (W.strip(W.convdiff(128), 50), 64, 1)]
    hs, Bs = [], []
    for i, (st, leaf, nrhs) in enumerate(probs):
        hs.append(gpu.acr_factor(_op(gpu, st), leaf, 1e-8, "mixed"))
        Bs.append(torch.from_numpy(W.rhs(st.n, nrhs, seed=W.seed_for(2, 800 + i))).cuda())
    xs = [gpu.acr_solve(h, B).cpu().numpy() for h, B in zip(hs, Bs)]
    try:
        for mode in (1, 2, 3):
            gpu.acr_set_solve_mode(mode)
            xb = [x.cpu().numpy() for x in gpu.acr_solve_batched(hs, Bs)]
            for i in range(len(hs)):
                assert np.array_equal(xs[i], xb[i]), f"mode {mode}, problem {i}"
    finally:
        gpu.acr_set_solve_mode(0)
        for h in hs:
            gpu.acr_destroy(h)


def test_persistent_forced_give_up_returns_nan(gpu):
    """wait_limit < 0: every task that reads another task's output gives up
    at once; all workgroups still reach the end of the task list, the pass
    returns NaN, and the next pass with the default limit is correct."""
    import torch
    st = W.strip(W.varkappa(128), 40)
    h = gpu.acr_factor(_op(gpu, st), 32, 1e-8, "fp64")
    B = torch.from_numpy(W.rhs(st.n, 2, seed=W.seed_for(2, 901))).cuda()
    ref = gpu.acr_solve(h, B).cpu().numpy()
    try:
        gpu.acr_set_solve_mode(2, -1)
        x = gpu.acr_solve(h, B).cpu().numpy()
        assert np.isnan(x).all()
        # the refinement loop sees the NaN and reports it instead of a value
        op = _op(gpu, st)
        with pytest.raises(gpu.ACRError):
            gpu.acr_solve_refined(h, op, B, tol=1e-10, maxit=3)
    finally:
        gpu.acr_set_solve_mode(2, 0)
    try:
        x2 = gpu.acr_solve(h, B).cpu().numpy()
        assert np.array_equal(x2, ref)
    finally:
        gpu.acr_set_solve_mode(0, 0)
    gpu.acr_destroy(h)


def test_set_solve_mode_rejects_unknown_mode(gpu):
    with pytest.raises(gpu.ACRError):
        gpu.acr_set_solve_mode(7)

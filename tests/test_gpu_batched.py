"""Batched factorisation and solve of independent problems of different sizes
(the mixed-size workload: sides 64..256, leaf 32, eps 1e-8, 8 right-hand
sides).  Every problem's batched factor and solution must equal, bit for bit,
the ones it gets alone (kernel variants depend on a problem's own shapes
only), the FP64 solutions must match the oracle at 10 eps, and the batch must
take far fewer launches than the problems one by one."""
import numpy as np
import pytest

import workloads as W
from oracle import acr as OA

pytestmark = pytest.mark.gpu


def _op(acr, st):
    return acr.Operator.from_arrays(st.nx, st.ny, *st.arrays())


def _problems(count, seed=W.seed_for(3, 900)):
    rng = np.random.default_rng(seed)
    sides = rng.choice([64, 96, 128, 192, 256], size=count)
    kinds = rng.integers(0, 2, size=count)
    out = []
    for i, (s, k) in enumerate(zip(sides, kinds)):
        st = W.poisson(int(s)) if k == 0 else W.varkappa(int(s), seed=W.seed_for(3, 100 + i))
        out.append(st)
    return out


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batched_equals_solo(gpu, prec):
    import torch
    probs = _problems(10)
    probs.append(W.poisson(96, 37))       # odd block count
    probs.append(W.strip(W.varkappa(64), 5))
    leaf, eps, nrhs = 32, 1e-8, 8
    print(f"[case] batch of {len(probs)}: sides {[p.nx for p in probs]} {prec}", flush=True)
    ops = [_op(gpu, st) for st in probs]
    Bs = [torch.from_numpy(W.rhs(st.n, nrhs, seed=W.seed_for(3, 200 + i))).cuda() for i, st in enumerate(probs)]
    c0 = gpu.acr_launch_count()
    hb = gpu.acr_factor_batched(ops, leaf, eps, prec)
    c1 = gpu.acr_launch_count()
    xb = [x.cpu().numpy() for x in gpu.acr_solve_batched(hb, Bs)]
    c2 = gpu.acr_launch_count()
    solo_f, solo_s = 0, 0
    for i, (op, B) in enumerate(zip(ops, Bs)):
        a = gpu.acr_launch_count()
        h = gpu.acr_factor(op, leaf, eps, prec)
        b = gpu.acr_launch_count()
        x = gpu.acr_solve(h, B).cpu().numpy()
        c = gpu.acr_launch_count()
        solo_f += b - a
        solo_s += c - b
        assert np.array_equal(x, xb[i]), f"problem {i} (side {probs[i].nx}): batched solution differs"
        ib, isolo = gpu.acr_get_info(hb[i]), gpu.acr_get_info(h)
        assert ib["level_max_rank"] == isolo["level_max_rank"]
        assert ib["factor_bytes"] == isolo["factor_bytes"]
        if i in (0, 3):   # stored blocks of the first levels, bit for bit
            for lev in range(min(2, isolo["levels"])):
                for which, k in ((0, 0), (1, 1), (2, 1)):
                    assert np.array_equal(gpu.acr_get_block(h, lev, which, k),
                                          gpu.acr_get_block(hb[i], lev, which, k))
        gpu.acr_destroy(h)
    print(f"launches: batched factor {c1 - c0} vs {solo_f} one by one; batched solve {c2 - c1} vs {solo_s}")
    assert (c1 - c0) * 3 < solo_f
    assert (c2 - c1) * 3 < solo_s
    if prec == "fp64":
        for i, st in enumerate(probs):
            if st.nx > 96:
                continue
            xo = OA.solve(OA.factor(st, leaf, eps), st, Bs[i].cpu().numpy())
            e = float(np.linalg.norm(xb[i] - xo) / np.linalg.norm(xo))
            assert e <= 10 * eps, f"problem {i}: {e:.2e}"


def test_batched_refined_residuals(gpu):
    """Mixed batched factors as preconditioners: each problem refined to 1e-10."""
    import torch
    from oracle import direct
    probs = _problems(6, seed=W.seed_for(3, 901))
    ops = [_op(gpu, st) for st in probs]
    hs = gpu.acr_factor_batched(ops, 32, 1e-8, "mixed")
    for i, (st, op, h) in enumerate(zip(probs, ops, hs)):
        b = W.rhs(st.n, 8, seed=W.seed_for(3, 300 + i))
        x, its, rel = gpu.acr_solve_refined(h, op, torch.from_numpy(b).cuda(), tol=1e-10, maxit=30)
        r = direct.residual(st, x.cpu().numpy(), b)
        assert r <= 1e-10, f"problem {i}: {r:.2e}"


def test_batched_errors(gpu):
    import torch
    st = W.poisson(64)
    bad = W.poisson(50)                     # 50 -> 25: odd cluster above the leaf
    with pytest.raises(gpu.ACRError) as ei:
        gpu.acr_factor_batched([_op(gpu, st), _op(gpu, bad)], 16, 1e-8)
    assert ei.value.name == "ACR_ERR_INVALID_ARG" and "problem 1" in str(ei.value)
    z = np.zeros(32 * 32)
    zop = gpu.Operator.from_arrays(32, 32, z, z, z, z, z)
    with pytest.raises(gpu.ACRError) as ei:
        gpu.acr_factor_batched([_op(gpu, W.poisson(32)), zop], 16, 1e-8)
    assert ei.value.name == "ACR_ERR_SINGULAR" and "problem 1" in str(ei.value)
    # outputs must not overlap
    hs = gpu.acr_factor_batched([_op(gpu, st), _op(gpu, st)], 16, 1e-8)
    import ctypes
    lib = gpu.load()
    B = torch.from_numpy(W.rhs(st.n, 1)).cuda().reshape(-1)
    X = torch.empty_like(B)
    hp = (ctypes.c_void_p * 2)(hs[0].ptr, hs[1].ptr)
    bp = (ctypes.c_void_p * 2)(B.data_ptr(), B.data_ptr())
    xp = (ctypes.c_void_p * 2)(X.data_ptr(), X.data_ptr())
    nr = (ctypes.c_int32 * 2)(1, 1)
    assert gpu.STATUS[lib.acr_solve_batched(hp, bp, xp, nr, 2, gpu._stream())] == "ACR_ERR_INVALID_ARG"

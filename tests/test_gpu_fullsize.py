"""GPU parity at the full block size of the large workloads.

The oracle cannot factor the whole 1024 x 1024 (or 512 x 512) operator in a
test's time, but it can factor a strip of its first block rows: the same
block size, leaf, eps and coefficients, so every HODLR depth, panel height
(up to 512 rows) and core size of the real workload appears.  On the strip
every stored X_k, E_k, F_k of every level is compared element-wise with the
oracle's (|gpu - oracle| <= 10 eps max|oracle| per block), the solution is
compared at 10 eps, and the profiler's path counts show that the panels of
more than 128 rows went through the large-panel QR and Q application and that
the register SVD ran.  The mixed form's forward error before refinement is
printed next to its bound.
"""
import numpy as np
import pytest

import workloads as W
from oracle import acr as OA
from oracle import hodlr

pytestmark = pytest.mark.gpu

# bound of the mixed (FP32) form's forward error before refinement
from bounds import mixed_forward_bound  # noqa: E402

_CACHE = {}


def _full(kind):
    if kind not in _CACHE:
        _CACHE[kind] = W.varkappa(1024) if kind == "varkappa" else W.convdiff(512)
    return _CACHE[kind]


def _op(acr, st):
    return acr.Operator.from_arrays(st.nx, st.ny, *st.arrays())


def _relerr(x, y):
    return float(np.linalg.norm(x - y) / np.linalg.norm(y))


def _compare_blocks(acr, h, fac, eps):
    """Every stored block of every level; returns the worst scaled error."""
    worst = 0.0
    nblk = 0
    for lev, (X, E, F) in enumerate(fac.levels):
        for k, Xk in X.items():
            ref = hodlr.densify(Xk)
            got = acr.acr_get_block(h, lev, 0, k)
            e = np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300)
            assert e <= 10 * eps, f"level {lev} X_{k}: {e:.3e}"
            worst, nblk = max(worst, e), nblk + 1
        for which, L in ((1, E), (2, F)):
            for k in range(len(L)):
                ref = hodlr.densify(L[k])
                got = acr.acr_get_block(h, lev, which, k)
                scale = np.abs(ref).max()
                if scale == 0.0:
                    assert np.abs(got).max() == 0.0
                    continue
                e = np.abs(got - ref).max() / scale
                assert e <= 10 * eps, f"level {lev} {'EF'[which - 1]}_{k}: {e:.3e}"
                worst, nblk = max(worst, e), nblk + 1
    ref = hodlr.densify(fac.Xlast)
    got = acr.acr_get_block(h, len(fac.levels), 0, 0)
    e = np.abs(got - ref).max() / np.abs(ref).max()
    assert e <= 10 * eps, f"last inverse: {e:.3e}"
    return max(worst, e), nblk + 1


STRIPS = [
    # (workload, block rows, leaf, eps, nrhs); eps 1e-9 raises the ranks so that the
    # accumulated Schur-update cores reach 48..64 columns (the register SVD)
    ("varkappa", 16, 64, 1e-6, 1),
    ("varkappa", 33, 64, 1e-6, 1),
    ("convdiff", 16, 64, 1e-7, 64),
    ("varkappa", 33, 64, 1e-9, 1),
]


@pytest.mark.parametrize("case", range(len(STRIPS)), ids=[f"{k}-{r}rows-eps{e:g}" for k, r, _, e, _ in STRIPS])
def test_strip_fp64_every_block(gpu, case):
    import torch
    kind, rows, leaf, eps, nrhs = STRIPS[case]
    st = W.strip(_full(kind), rows)
    print(f"[case] {st.name} {st.nx}x{st.ny} leaf {leaf} eps {eps} nrhs {nrhs}", flush=True)
    gpu.acr_profile_start(None)
    h = gpu.acr_factor(_op(gpu, st), leaf, eps, "fp64")
    b = W.rhs(st.n, nrhs, seed=W.seed_for(2, 40 + rows))
    x = gpu.acr_solve(h, torch.from_numpy(b).cuda()).cpu().numpy()
    paths = gpu.acr_profile_report().get("paths", {})
    gpu.acr_profile_start([])
    fac = OA.factor(st, leaf, eps)
    worst, nblk = _compare_blocks(gpu, h, fac, eps)
    xo = OA.solve(fac, st, b)
    e = _relerr(x, xo)
    print(f"{st.name}: {nblk} stored blocks, worst block error {worst:.2e} (10 eps = {10 * eps:.0e}); "
          f"solution vs oracle {e:.2e}; ranks GPU {gpu.acr_get_info(h)['level_max_rank']} "
          f"oracle {OA.level_ranks(fac)}")
    print("paths:", {k: v for k, v in sorted(paths.items())})
    assert e <= 10 * eps
    # the panels of more than 128 rows (HODLR depth 1 and 2 at block size 512 / 1024)
    # went through the large-panel QR and Q application
    assert any(k.startswith("qr.") and k.endswith("p>128") for k in paths), paths
    assert any(k.startswith("applyq.") and k.endswith("p>128") for k in paths), paths
    assert any(k.startswith("gemm.") and k.endswith("M>128") for k in paths), paths
    if eps <= 1e-9:
        # cores of 48..64 columns arise (accumulated D' ranks): the register SVD ran
        assert paths.get("svd.reg", 0) > 0, paths


@pytest.mark.parametrize("kind,rows,leaf,eps", [("varkappa", 16, 64, 1e-6), ("convdiff", 16, 64, 1e-7)])
def test_strip_mixed_forward_error(gpu, kind, rows, leaf, eps):
    """FP32 factor and solve before refinement against the FP64 oracle on the
    same strip: reported next to 10 eps and gated by the FP32 bound."""
    import torch
    st = W.strip(_full(kind), rows)
    print(f"[case] mixed {st.name} leaf {leaf} eps {eps}", flush=True)
    h = gpu.acr_factor(_op(gpu, st), leaf, eps, "mixed")
    b = W.rhs(st.n, 1, seed=W.seed_for(2, 70 + rows))
    x = gpu.acr_solve(h, torch.from_numpy(b).cuda()).cpu().numpy()
    xo = OA.solve(OA.factor(st, leaf, eps), st, b)
    e = _relerr(x, xo)
    bound = mixed_forward_bound(eps)
    print(f"mixed {st.name}: forward error before refinement {e:.2e}; 10 eps = {10 * eps:.0e}; "
          f"FP32 bound {bound:.1e}")
    assert e <= bound

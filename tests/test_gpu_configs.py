"""GPU checks at the sizes of the benchmark workloads.

- Poisson 64x64, leaf 16, eps 1e-10, FP64: against sparse LU and exact BCR.
- Poisson / variable-kappa problems of sides 64..256, leaf 32, eps 1e-8,
  8 right-hand sides: FP64 against the oracle ACR where it is fast, refined
  residual everywhere.
- Upwind convection-diffusion 512x512, leaf 64, eps 1e-7, 64 right-hand
  sides (the many-RHS solve path): refined residual.
- Variable kappa 1024x1024, leaf 64, eps 1e-6 (the benchmark workload): the
  first-level stored blocks the oracle can compute one by one (X_k is the
  truncated inverse of the tridiagonal D_k, E'_j a scaled block of X), and
  the refined residual of the mixed and the FP64 forms.
- Option paths: inner truncation, rank cap, many RHS versus one at a time.
"""
import numpy as np
import pytest

import workloads as W
from oracle import acr as OA
from oracle import bcr, direct

pytestmark = pytest.mark.gpu


def _op(acr, st):
    return acr.Operator.from_arrays(st.nx, st.ny, *st.arrays())


def _relerr(x, y):
    return float(np.linalg.norm(x - y) / np.linalg.norm(y))


_VK1024 = []


def _varkappa1024():
    if not _VK1024:
        _VK1024.append(W.varkappa(1024))
    return _VK1024[0]


def _refined(acr, st, leaf, eps, prec, nrhs, seed, maxit=40, **kw):
    import torch
    op = _op(acr, st)
    h = acr.acr_factor(op, leaf, eps, prec, **kw)
    b = W.rhs(st.n, nrhs, seed=seed)
    x, its, rel = acr.acr_solve_refined(h, op, torch.from_numpy(b).cuda(), tol=1e-10, maxit=maxit)
    r = direct.residual(st, x.cpu().numpy(), b)
    return h, its, rel, r


def test_poisson64_against_lu_and_bcr(gpu):
    import torch
    st = W.poisson(64)
    h = gpu.acr_factor(_op(gpu, st), 16, 1e-10, "fp64")
    b = W.rhs(st.n, 1)
    x = gpu.acr_solve(h, torch.from_numpy(b).cuda()).cpu().numpy()
    e_lu = _relerr(x, direct.solve(st, b))
    e_bcr = _relerr(x, bcr.bcr_solve(st, b))
    print(f"poisson 64: vs LU {e_lu:.2e}, vs BCR {e_bcr:.2e}")
    assert e_lu <= 1e-8 and e_bcr <= 1e-8


@pytest.mark.parametrize("side", [64, 96, 128, 192, 256])
def test_mixed_sizes_leaf32(gpu, side):
    kind = "poisson" if side in (64, 128, 256) else "varkappa"
    st = W.poisson(side) if kind == "poisson" else W.varkappa(side, seed=W.seed_for(3, side))
    if side <= 96:   # FP64 form against the oracle ACR at the same eps
        import torch
        h = gpu.acr_factor(_op(gpu, st), 32, 1e-8, "fp64")
        b = W.rhs(st.n, 8, seed=W.seed_for(3, 50 + side))
        x = gpu.acr_solve(h, torch.from_numpy(b).cuda()).cpu().numpy()
        xo = OA.solve(OA.factor(st, 32, 1e-8), st, b)
        e = _relerr(x, xo)
        print(f"{kind} {side}: FP64 vs oracle {e:.2e}")
        assert e <= 10 * 1e-8
    h, its, rel, r = _refined(gpu, st, 32, 1e-8, "mixed", 8, W.seed_for(3, 60 + side))
    print(f"{kind} {side}: mixed + refinement, {its} iterations, relres {r:.2e}")
    assert r <= 1e-10


def test_convdiff512_64rhs(gpu):
    st = W.convdiff(512)
    h, its, rel, r = _refined(gpu, st, 64, 1e-7, "mixed", 64, W.seed_for(4, 1))
    print(f"convdiff 512, 64 RHS: {its} iterations, relres {r:.2e}")
    assert r <= 1e-10


def test_varkappa1024_first_level_blocks(gpu):
    """X_k = T_eps(D_k^{-1}) and E'_j = T_eps(-E_i T_eps(X_(i-1) E_(i-1))) at
    level 0 of the full-size FP64 factorisation, against dense inverses."""
    st = _varkappa1024()
    eps = 1e-6
    h = gpu.acr_factor(_op(gpu, st), 64, eps, "fp64")
    for k in (0, 512, 1022):
        Xd = np.linalg.inv(direct.block(st, k)[0])
        got = gpu.acr_get_block(h, 0, 0, k)
        err = np.abs(got - Xd).max() / np.abs(Xd).max()
        print(f"X_{k}: max error {err:.2e}")
        assert err <= 10 * eps
    i = 511                                   # odd: E'_(255) = -E_511 X_510 E_510
    Di1, Ei1, _ = direct.block(st, i - 1)
    ref = -direct.block(st, i)[1] @ np.linalg.inv(Di1) @ Ei1
    got = gpu.acr_get_block(h, 1, 1, (i - 1) // 2)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"E'_{(i - 1) // 2}: max error {err:.2e}")
    assert err <= 10 * eps


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_varkappa1024_refined(gpu, prec):
    st = _varkappa1024()
    h, its, rel, r = _refined(gpu, st, 64, 1e-6, prec, 1, W.seed_for(1, 9))
    info = gpu.acr_get_info(h)
    print(f"varkappa 1024 {prec}: {its} iterations, relres {r:.2e}, factor {info['factor_bytes'] / 1e9:.2f} GB, "
          f"max rank {info['max_rank']}")
    assert r <= 1e-10
    assert info["levels"] == 10


def test_inner_truncation_path(gpu):
    import torch
    st = W.varkappa(64)
    eps = 1e-8
    h = gpu.acr_factor(_op(gpu, st), 16, eps, "fp64", inner_eps=eps / 10)
    b = W.rhs(st.n, 1, seed=11)
    x = gpu.acr_solve(h, torch.from_numpy(b).cuda()).cpu().numpy()
    xo = OA.solve(OA.factor(st, 16, eps), st, b)
    e = _relerr(x, xo)
    print(f"inner truncation: vs oracle {e:.2e}")
    assert e <= 10 * eps


def test_rank_cap(gpu):
    st = W.varkappa(128)
    h, its, rel, r = _refined(gpu, st, 32, 1e-12, "fp64", 1, 13, maxit=50, max_rank=4)
    print(f"rank cap 4: {its} iterations, relres {r:.2e}")
    assert gpu.acr_get_info(h)["max_rank"] <= 4
    assert r <= 1e-10


def test_many_rhs_matches_one_at_a_time(gpu):
    """12 right-hand sides (the GEMM solve path) against the same columns
    solved one by one (the fused matvec path)."""
    import torch
    st = W.convdiff(96, 40)
    h = gpu.acr_factor(_op(gpu, st), 24, 1e-9, "fp64")
    b = W.rhs(st.n, 12, seed=17)
    xb = gpu.acr_solve(h, torch.from_numpy(b).cuda()).cpu().numpy()
    for q in (0, 5, 11):
        xq = gpu.acr_solve(h, torch.from_numpy(np.ascontiguousarray(b[:, q])).cuda()).cpu().numpy()
        assert _relerr(xb[:, q], xq) <= 1e-12

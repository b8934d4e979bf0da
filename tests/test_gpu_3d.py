"""GPU parity for 3-D operators (one block per plane, Section 4's closing
remarks): the HIP path through the C ABI against the CPU oracle on the dense
plane blocks, and ACR as an FGMRES preconditioner against sparse LU."""
import numpy as np
import pytest

import workloads as W
from oracle import acr as OA
from oracle import direct, hodlr

pytestmark = pytest.mark.gpu


def _op3(acr, st):
    return acr.Operator3d.from_arrays(st.nx, st.ny, st.nz, *st.arrays())


def _relerr(x, y):
    return float(np.linalg.norm(x - y) / np.linalg.norm(y))


def _scaled_poisson(nx, ny, nz, seed=5):
    """A 7-point operator with rows of unequal length and random symmetric
    couplings (every coefficient different, diagonally dominant)."""
    st = W.poisson3d(nx, ny, nz)
    rng = np.random.default_rng(seed)
    for fwd, bwd, off in ((st.east, st.west, 1), (st.north, st.south, nx), (st.up, st.down, nx * ny)):
        w = rng.uniform(0.5, 2.0, fwd.size) * (fwd != 0)
        fwd *= w
        bwd[off:] = fwd[:-off]     # symmetric: A[i, i+off] = A[i+off, i]
    st.diag = -(st.west + st.east + st.south + st.north + st.down + st.up) + 0.3
    st.name = "scaled3d"
    return st


CASES = [
    # (operator, leaf, eps): square and oblong planes, splits on rows and inside rows
    (lambda: W.varkappa3d(8), 16, 1e-9),             # s = 64, ranks 8/8/1 by depth
    (lambda: W.varkappa3d(16), 32, 1e-8),            # s = 256
    (lambda: _scaled_poisson(16, 8, 12), 32, 1e-8),  # s = 128, 12 planes
    (lambda: _scaled_poisson(32, 4, 9), 16, 1e-8),   # s = 128, splits inside a row at depth 3
    (lambda: _scaled_poisson(4, 4, 5), 16, 1e-9),    # one leaf per plane: exact BCR
]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_3d_vs_oracle(gpu, case, prec):
    import torch
    from bounds import mixed_forward_bound
    build, leaf, eps = CASES[case]
    st = build()
    h = gpu.acr_factor_3d(_op3(gpu, st), leaf, eps, prec)
    b = W.rhs(st.n, 3, seed=41)
    x = gpu.acr_solve(h, torch.from_numpy(b).cuda()).cpu().numpy()
    D, E, F = direct.blocks3d(st)
    s = st.s
    fac = OA.factor_blocks(D, E, F, leaf, eps)
    xo = np.concatenate(OA.solve_blocks(fac, [b[k * s:(k + 1) * s] for k in range(st.nz)]), axis=0)
    e = _relerr(x, xo)
    bound = 10 * eps if prec == "fp64" else mixed_forward_bound(eps)
    info = gpu.acr_get_info(h)
    print(f"{st.name} {st.nx}x{st.ny}x{st.nz} leaf {leaf} eps {eps} {prec}: vs oracle {e:.2e} "
          f"(bound {bound:.1e}); ranks {info['level_max_rank']}")
    assert e <= bound
    assert info["levels"] == len(fac.levels)
    if prec != "fp64":
        return
    # every stored block of the first levels, element-wise
    for lev in range(min(3, len(fac.levels))):
        X, El, Fl = fac.levels[lev]
        for k in sorted(X):
            ref = hodlr.densify(X[k])
            got = gpu.acr_get_block(h, lev, 0, k)
            assert np.abs(got - ref).max() <= 10 * eps * np.abs(ref).max(), (lev, k)
        for k in range(1, len(El), 2):
            for which, Lst in ((1, El), (2, Fl)):
                ref = hodlr.densify(Lst[k])
                got = gpu.acr_get_block(h, lev, which, k)
                assert np.abs(got - ref).max() <= 10 * eps * max(np.abs(ref).max(), 1e-300), (lev, which, k)


def test_3d_level0_inverse_is_plane_inverse(gpu):
    """X_0 of level 0 is T(D_0^{-1}) with D_0 the plane operator: against the
    dense inverse at eps (the ingest of the plane operator and the general
    H-inverse, not the tridiagonal closed form)."""
    st = W.varkappa3d(16)
    eps = 1e-10
    h = gpu.acr_factor_3d(_op3(gpu, st), 32, eps, "fp64")
    D, _, _ = direct.blocks3d(st)
    for k in (0, 2, 14):
        ref = np.linalg.inv(D[k])
        got = gpu.acr_get_block(h, 0, 0, k)
        assert np.abs(got - ref).max() <= 100 * eps * np.abs(ref).max()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_3d_krylov_preconditioner(gpu, prec):
    """ACR at coarse eps as the FGMRES preconditioner of a 3-D operator
    (32^3 unknowns, plane 1024, leaf 64) reaches 1e-10; the solution matches
    sparse LU and the true residual is recomputed on the CPU."""
    import torch
    st = W.varkappa3d(32)
    op = _op3(gpu, st)
    b = W.rhs(st.n, 2, seed=43)
    A = direct.assemble3d(st)
    xd = direct.solve3d(st, b)
    for eps in (1e-2, 1e-4):
        h = gpu.acr_factor_3d(op, 64, eps, prec)
        x, its, rel = gpu.acr_solve_krylov(h, op, torch.from_numpy(b).cuda(), tol=1e-10, maxit=80)
        x = x.cpu().numpy()
        r = np.linalg.norm(b - A @ x, axis=0) / np.linalg.norm(b, axis=0)
        info = gpu.acr_get_info(h)
        print(f"3-D 32^3 {prec} eps {eps}: {its} applications, relres {rel:.2e} (CPU {r.max():.2e}), "
              f"ranks {info['level_max_rank']}")
        assert r.max() <= 2e-10
        assert _relerr(x, xd) <= 1e-7
    # refinement and the residual entry point on the same operator
    h = gpu.acr_factor_3d(op, 64, 1e-6, prec)
    x, its, rel = gpu.acr_solve_refined(h, op, torch.from_numpy(b).cuda(), tol=1e-10, maxit=40)
    R = gpu.acr_residual(op, x, torch.from_numpy(b).cuda()).cpu().numpy()
    assert np.abs(R - (b - A @ x.cpu().numpy())).max() <= 1e-12 * np.abs(b).max()
    assert rel <= 1e-10


def test_3d_errors(gpu):
    import torch
    st = _scaled_poisson(6, 4, 3)             # s = 24: leaf 6 after two halvings, split 12 = 2 rows of 6
    h = gpu.acr_factor_3d(_op3(gpu, st), 6, 1e-8, "fp64")
    assert gpu.acr_get_info(h)["levels"] >= 1
    bad = _scaled_poisson(8, 3, 3)
    with pytest.raises(gpu.ACRError) as ei:   # s = 24: the top split at 12 cuts a row of 8
        gpu.acr_factor_3d(_op3(gpu, bad), 6, 1e-8, "fp64")
    assert ei.value.code == 1
    other = _scaled_poisson(6, 2, 6)          # same N, planes of 12 instead of 24
    with pytest.raises(gpu.ACRError):          # operator shape differs from the factor
        gpu.acr_solve_krylov(h, _op3(gpu, other), torch.zeros(other.n, dtype=torch.float64, device="cuda"))
    nan = _scaled_poisson(6, 4, 3)
    nan.north[7] = np.nan
    with pytest.raises(gpu.ACRError):
        gpu.acr_factor_3d(_op3(gpu, nan), 6, 1e-8, "fp64")

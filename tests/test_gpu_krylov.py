"""GPU checks of the Krylov solve (restarted FGMRES right-preconditioned by the
ACR factor) and of the few-RHS solve widths.

- Poisson 64x64, FP64 factor at eps 1e-4: preconditioner applications and
  solution against the oracle FGMRES with the oracle ACR at the same eps, and
  against sparse LU.
- Variable kappa 256x256, mixed factor at eps 1e-6, 2 right-hand sides:
  FGMRES reaches 1e-10 with no more preconditioner applications than
  refinement (plus one).
- Upwind convection-diffusion 128x128 with a loose factor (eps 1e-2): FGMRES
  still reaches 1e-10 (refinement's contraction is reported).
- 2 and 4 right-hand sides through the matvec solve against one at a time.
- The paper's Helmholtz problem (indefinite for k^2 > 2 pi^2, Gaussian source)
  on 128 x 128 and 256 x 256 grids: FGMRES around the FP64 and the mixed factor
  against sparse LU.
- The paper's recirculating convection-diffusion (b = (cos 8 pi x, sin 8 pi y))
  over an alpha sweep (1, 30, 100) on a 256 x 256 grid: FGMRES around the mixed factor
  against sparse LU, with the factor's ranks reported.
"""
import numpy as np
import pytest

import workloads as W
from oracle import acr as OA
from oracle import direct, krylov

pytestmark = pytest.mark.gpu


def _op(acr, st):
    return acr.Operator.from_arrays(st.nx, st.ny, *st.arrays())


def _relerr(x, y):
    return float(np.linalg.norm(x - y) / np.linalg.norm(y))


def test_krylov_fp64_against_oracle_fgmres(gpu):
    import torch
    st = W.poisson(64)
    eps = 1e-4
    op = _op(gpu, st)
    h = gpu.acr_factor(op, 16, eps, "fp64")
    b = W.rhs(st.n, 1, seed=21)[:, 0].copy()
    x, its, rel = gpu.acr_solve_krylov(h, op, torch.from_numpy(b).cuda(), tol=1e-10, maxit=50, restart=20)
    x = x.cpu().numpy()
    A = direct.assemble(st)
    fac = OA.factor(st, 16, eps)
    xo, itso, hist = krylov.fgmres(lambda v: A @ v, b, lambda v: OA.solve(fac, st, v), tol=1e-10, maxit=50,
                                   restart=20)
    xd = direct.solve(st, b)
    print(f"poisson 64, eps 1e-4: GPU {its} applications (relres {rel:.2e}), oracle {itso} ({hist[-1]:.2e}), "
          f"vs LU {_relerr(x, xd):.2e}")
    assert rel <= 1e-10 and hist[-1] <= 1e-10
    assert abs(its - itso) <= 1
    assert _relerr(x, xd) <= 1e-8
    assert direct.residual(st, x, b) <= 1e-10


def test_krylov_mixed_varkappa256(gpu):
    import torch
    st = W.varkappa(256, seed=W.seed_for(3, 256))
    op = _op(gpu, st)
    h = gpu.acr_factor(op, 32, 1e-6, "mixed")
    b = W.rhs(st.n, 2, seed=22)
    B = torch.from_numpy(b).cuda()
    xk, itk, relk = gpu.acr_solve_krylov(h, op, B, tol=1e-10, maxit=40, restart=20)
    xr, itr, relr = gpu.acr_solve_refined(h, op, B, tol=1e-10, maxit=40)
    rk = direct.residual(st, xk.cpu().numpy(), b)
    print(f"varkappa 256 mixed: FGMRES {itk} applications ({relk:.2e}, true {rk:.2e}), refinement {itr} ({relr:.2e})")
    assert relk <= 1e-10 and rk <= 1e-10
    assert itk <= itr + 1


def test_krylov_loose_preconditioner(gpu):
    import torch
    st = W.convdiff(128)
    op = _op(gpu, st)
    h = gpu.acr_factor(op, 32, 1e-2, "mixed")
    b = W.rhs(st.n, 1, seed=23)[:, 0].copy()
    B = torch.from_numpy(b).cuda()
    xk, itk, relk = gpu.acr_solve_krylov(h, op, B, tol=1e-10, maxit=120, restart=30)
    _, itr, relr = gpu.acr_solve_refined(h, op, B, tol=1e-10, maxit=30, raise_on_fail=False)
    rk = direct.residual(st, xk.cpu().numpy(), b)
    print(f"convdiff 128, eps 1e-2: FGMRES {itk} applications (true relres {rk:.2e}); "
          f"refinement after {itr} corrections: {relr:.2e}")
    assert relk <= 1e-10 and rk <= 1e-10


@pytest.mark.parametrize("nrhs", [2, 4])
def test_solve_widths_match_one_at_a_time(gpu, nrhs):
    import torch
    st = W.varkappa(96, seed=W.seed_for(3, 96))
    h = gpu.acr_factor(_op(gpu, st), 24, 1e-9, "fp64")
    b = W.rhs(st.n, nrhs, seed=24 + nrhs)
    xb = gpu.acr_solve(h, torch.from_numpy(b).cuda()).cpu().numpy()
    for q in range(nrhs):
        xq = gpu.acr_solve(h, torch.from_numpy(np.ascontiguousarray(b[:, q])).cuda()).cpu().numpy()
        assert _relerr(xb[:, q], xq) <= 1e-12


@pytest.mark.parametrize("side,k,prec", [(128, 10.0, "fp64"), (128, 40.0, "mixed"), (256, 60.0, "mixed")])
def test_krylov_helmholtz(gpu, side, k, prec):
    import torch
    st = W.helmholtz(side, k)
    op = _op(gpu, st)
    h = gpu.acr_factor(op, 32, 1e-7, prec)
    b = W.helmholtz_rhs(side)[:, 0].copy()
    x, its, rel = gpu.acr_solve_krylov(h, op, torch.from_numpy(b).cuda(), tol=1e-10, maxit=100, restart=30)
    x = x.cpu().numpy()
    xd = direct.solve(st, b)
    err = _relerr(x, xd)
    print(f"helmholtz {side}, k {k}, {prec}: {its} applications, relres {rel:.2e}, vs LU {err:.2e}")
    assert rel <= 1e-10 and direct.residual(st, x, b) <= 1e-10
    assert err <= 1e-6


@pytest.mark.parametrize("alpha", [1.0, 30.0, 100.0])
def test_krylov_recirculating(gpu, alpha):
    """(Beyond alpha ~ 1e3 the upwind operator is too ill-conditioned for a 1e-10
    residual in FP64: at 96 x 96 and alpha = 1e3 sparse LU's own residual is
    8e-6, at alpha = 1e4 it is O(1).)"""
    import torch
    st = W.recirculating(256, alpha)
    op = _op(gpu, st)
    h = gpu.acr_factor(op, 32, 1e-6, "mixed")
    b = W.rhs(st.n, 1, seed=31)[:, 0].copy()
    x, its, rel = gpu.acr_solve_krylov(h, op, torch.from_numpy(b).cuda(), tol=1e-10, maxit=60, restart=30)
    x = x.cpu().numpy()
    xd = direct.solve(st, b)
    info = gpu.acr_get_info(h)
    print(f"recirculating 256, alpha {alpha:g}: {its} applications, relres {rel:.2e}, vs LU {_relerr(x, xd):.2e}, "
          f"max rank {info['max_rank']}")
    assert rel <= 1e-10 and direct.residual(st, x, b) <= 1e-10

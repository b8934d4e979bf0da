"""Pins for the CPU oracle: it is checked against things fixed independently
of its own code (closed forms, brute force, library routines, the paper's
worked example), so that a dropped term, wrong sign/index or a transposed
operand in it fails here before it is trusted as the parity reference."""
import math
import os

import numpy as np
import scipy.sparse as sp
import pytest

import workloads as W
from oracle import acr, bcr, direct, hodlr, krylov, refine

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------- generators
def test_stencils_symmetric_and_signs():
    for st in (W.poisson(9, 7), W.varkappa(12)):
        A = direct.assemble(st)
        assert abs(A - A.T).max() == 0.0
        assert np.all(st.west <= 0) and np.all(st.north <= 0)
    st = W.convdiff(16)
    A = direct.assemble(st).toarray()
    off = A - np.diag(np.diag(A))
    assert np.all(off <= 0.0)                                  # M-matrix signs
    assert np.all(np.diag(A) >= -off.sum(axis=1) - 1e-12)       # diagonal dominance


def test_varkappa_contrast_exact():
    st = W.varkappa(32)
    kw = -st.west.reshape(32, 32)[:, 1:]
    kn = -st.north.reshape(32, 32)[:-1, :]
    vals = np.concatenate([kw.ravel(), kn.ravel()])
    # contrast is defined over all face samples; interior faces cannot exceed it
    assert vals.max() / vals.min() <= 1e4 * (1 + 1e-12)
    assert vals.max() / vals.min() > 1e2


def test_blocks_structure():
    """D_i tridiagonal, E_i and F_i diagonal (Section 3, remark after Eq. system)."""
    st = W.varkappa(10)
    D, E, F = direct.blocks(st)
    for Di, Ei, Fi in zip(D, E, F):
        assert np.count_nonzero(np.triu(Di, 2)) == 0 and np.count_nonzero(np.tril(Di, -2)) == 0
        assert np.count_nonzero(Ei - np.diag(np.diag(Ei))) == 0
        assert np.count_nonzero(Fi - np.diag(np.diag(Fi))) == 0
    assert np.count_nonzero(E[0]) == 0 and np.count_nonzero(F[-1]) == 0


# ------------------------------------------------------------- O1 closed forms
@pytest.mark.parametrize("n,p,q", [(15, 1, 1), (31, 3, 5), (20, 7, 2)])
def test_direct_discrete_eigenfunction(n, p, q):
    """h^2-scaled 5-point Laplacian: A phi = lambda phi, lambda = 4 sin^2(p pi h/2) + 4 sin^2(q pi h/2)."""
    st = W.poisson(n)
    x, y = W.node_coords(n, n)
    h = 1.0 / (n + 1)
    phi = np.sin(p * math.pi * x) * np.sin(q * math.pi * y)
    lam = 4 * math.sin(p * math.pi * h / 2) ** 2 + 4 * math.sin(q * math.pi * h / 2) ** 2
    u = direct.solve(st, phi)
    assert np.linalg.norm(u - phi / lam) / np.linalg.norm(phi / lam) < 1e-12
    ub = bcr.bcr_solve(st, phi)
    assert np.linalg.norm(ub - phi / lam) / np.linalg.norm(phi / lam) < 1e-12


@pytest.mark.parametrize("n,p,q,k", [(15, 1, 1, 0.0), (31, 2, 3, 10.0), (20, 4, 1, 25.0)])
def test_helmholtz_discrete_eigenfunction(n, p, q, k):
    """h^2-scaled -Laplace - k^2: A phi = (lambda_pq - (k h)^2) phi for the
    discrete sine modes (k = 0 is the Poisson operator)."""
    st = W.helmholtz(n, k)
    x, y = W.node_coords(n, n)
    h = 1.0 / (n + 1)
    phi = np.sin(p * math.pi * x) * np.sin(q * math.pi * y)
    lam = 4 * math.sin(p * math.pi * h / 2) ** 2 + 4 * math.sin(q * math.pi * h / 2) ** 2 - (k * h) ** 2
    A = direct.assemble(st)
    assert np.linalg.norm(A @ phi - lam * phi) <= 1e-12 * np.linalg.norm(phi)
    if k == 0.0:
        assert np.array_equal(st.diag, W.poisson(n).diag)


def test_helmholtz_indefinite_and_source():
    st = W.helmholtz(31, 20.0)
    ev = np.linalg.eigvalsh(direct.assemble(st).toarray())
    assert ev.min() < 0.0 < ev.max()          # k^2 = 400 > 2 pi^2: indefinite
    b = W.helmholtz_rhs(31)
    x, y = W.node_coords(31, 31)
    c = np.argmin((x - 0.5) ** 2 + (y - 0.5) ** 2)
    assert abs(b[c, 0] + 100.0 / 32 ** 2) < 1e-12   # f(1/2, 1/2) = 100, scaled by -h^2


@pytest.mark.parametrize("n", [7, 24])
def test_direct_manufactured_variable_kappa(n):
    """u = x(1-x)y(1-y), kappa = 1+x+y at face midpoints: the flux-form 5-point
    scheme is exact for this pair, so the discrete solution equals u at nodes."""
    kx, ky = W.kappa_faces_from_function(lambda X, Y: 1.0 + X + Y, n, n)
    st = W.flux_form(kx, ky, n, n)
    x, y = W.node_coords(n, n)
    kap = 1 + x + y
    f = -((1 - 2 * x) * y * (1 - y) - 2 * kap * y * (1 - y)
          + x * (1 - x) * (1 - 2 * y) - 2 * kap * x * (1 - x))
    h = 1.0 / (n + 1)
    u_exact = x * (1 - x) * y * (1 - y)
    u = direct.solve(st, h * h * f)
    assert np.linalg.norm(u - u_exact) / np.linalg.norm(u_exact) < 1e-12
    ub = bcr.bcr_solve(st, h * h * f)
    assert np.linalg.norm(ub - u_exact) / np.linalg.norm(u_exact) < 1e-12


# ------------------------------------------------------------- O2 brute force
@pytest.mark.parametrize("nx,ny", [(1, 1), (2, 2), (3, 3), (4, 4), (5, 5), (7, 7), (8, 8),
                                   (16, 16), (33, 33), (6, 11), (9, 2), (5, 12)])
def test_bcr_equals_lu(nx, ny):
    st = W.convdiff(nx, ny) if nx != ny else W.varkappa(nx) if nx > 2 else W.poisson(nx)
    b = W.rhs(st.n, 3, seed=W.seed_for(0, nx * 100 + ny))
    A = direct.assemble(st).toarray()
    x_lu = np.linalg.solve(A, b)
    x_bcr = bcr.bcr_solve(st, b)
    cond = np.linalg.cond(A)
    assert np.linalg.norm(x_bcr - x_lu) / np.linalg.norm(x_lu) < 1e-15 * cond * 10 + 1e-14


def test_level_sizes():
    assert bcr.level_sizes(8) == [8, 4, 2, 1]
    assert bcr.level_sizes(1024) == [2 ** k for k in range(10, -1, -1)]
    assert bcr.level_sizes(96) == [96, 48, 24, 12, 6, 3, 1]
    assert bcr.level_sizes(5) == [5, 2, 1]


def _read_patterns():
    pats, cur = {}, None
    with open(os.path.join(GOLDEN, "n8_block_patterns.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tok = line.split()
            if tok[0] == "level":
                cur = int(tok[1])
                pats[cur] = {"order": [int(t) for t in tok[3:]], "rows": []}
            else:
                pats[cur]["rows"].append(tok)
    return pats


def _assemble_blocks(D, E, F):
    m, s = len(D), D[0].shape[0]
    A = np.zeros((m * s, m * s))
    for i in range(m):
        A[i * s:(i + 1) * s, i * s:(i + 1) * s] = D[i]
        if i > 0:
            A[i * s:(i + 1) * s, (i - 1) * s:i * s] = E[i]
        if i + 1 < m:
            A[i * s:(i + 1) * s, (i + 1) * s:(i + 2) * s] = F[i]
    return A


def test_worked_example_n8_patterns_and_schur():
    """The paper's 8-block example: permuted block patterns at each level, and
    each reduced system equals the Schur complement H22 - H21 H11^-1 H12 of the
    permuted system (Eq. "sche", Eq. "fund"), computed here by brute force."""
    pats = _read_patterns()
    rng = np.random.default_rng(5)
    s, m = 3, 8
    D = [np.eye(s) * 8 + rng.standard_normal((s, s)) for _ in range(m)]
    E = [np.zeros((s, s))] + [rng.standard_normal((s, s)) for _ in range(m - 1)]
    F = [rng.standard_normal((s, s)) for _ in range(m - 1)] + [np.zeros((s, s))]
    level = 0
    while True:
        m = len(D)
        order = list(range(0, m, 2)) + list(range(1, m, 2))
        assert pats[level]["order"] == order
        A = _assemble_blocks(D, E, F)
        perm = np.concatenate([np.arange(k * s, (k + 1) * s) for k in order])
        H = A[np.ix_(perm, perm)]
        for r, bi in enumerate(order):
            for c, bj in enumerate(order):
                blk = H[r * s:(r + 1) * s, c * s:(c + 1) * s]
                tok = pats[level]["rows"][r][c]
                if tok == ".":
                    assert np.count_nonzero(blk) == 0
                else:
                    assert np.count_nonzero(blk) > 0
                    assert tok == {0: "D", -1: "E", 1: "F"}[bj - bi]
        if m == 1:
            break
        ne = (m + 1) // 2
        H11, H12 = H[:ne * s, :ne * s], H[:ne * s, ne * s:]
        H21, H22 = H[ne * s:, :ne * s], H[ne * s:, ne * s:]
        S = H22 - H21 @ np.linalg.solve(H11, H12)
        X, D, E, F = bcr.reduce_level(D, E, F)
        assert np.allclose(_assemble_blocks(D, E, F), S, rtol=0, atol=1e-12)
        level += 1
    assert level == 3


# ------------------------------------------------------------------ HODLR T_eps
def test_truncation_rule_prescribed_spectrum():
    rng = np.random.default_rng(0)
    p, q = 40, 30
    Uo, _ = np.linalg.qr(rng.standard_normal((p, q)))
    Vo, _ = np.linalg.qr(rng.standard_normal((q, q)))
    sig = 10.0 ** -np.arange(q, dtype=float)          # 1, 1e-1, ..., 1e-29
    B = (Uo * sig) @ Vo.T
    for eps, t in ((1e-3 * 0.9999, 4), (1e-6 * 0.9999, 7), (1e-3 * 1.0001, 3), (0.5, 1)):
        U, V = hodlr.truncate(B, eps)
        assert U.shape[1] == t
        err = np.linalg.norm(B - U @ V.T, 2)
        assert err <= eps * sig[0]
        assert abs(err - sig[t]) <= 1e-12
    # relative to s1 of the block itself: s = (2, 1, 0.5)
    B2 = (Uo[:, :3] * np.array([2.0, 1.0, 0.5])) @ Vo[:, :3].T
    assert hodlr.truncate(B2, 0.2501)[0].shape[1] == 2
    assert hodlr.truncate(B2, 0.2499)[0].shape[1] == 3
    U, V = hodlr.truncate(np.zeros((5, 4)), 1e-8)
    assert U.shape == (5, 0) and V.shape == (4, 0)


def test_hodlr_roundtrip_matvec_and_tree():
    rng = np.random.default_rng(1)
    M = rng.standard_normal((96, 96))
    H = hodlr.compress(M, 24, 0.0)
    assert np.allclose(hodlr.densify(H), M, atol=1e-12)
    x = rng.standard_normal((96, 3))
    assert np.allclose(hodlr.matvec(H, x), M @ x, atol=1e-11)
    assert hodlr.cluster_sizes(96, 32) == [24, 24, 24, 24]
    assert hodlr.cluster_sizes(1024, 64) == [64] * 16
    assert hodlr.depth(H) == 2
    # smooth kernel: error of every block bounded by eps * its own s1
    xs = np.linspace(0, 1, 128)
    K = 1.0 / (1.0 + 40 * np.abs(xs[:, None] - xs[None, :]))
    Hk = hodlr.compress(K, 16, 1e-6)
    assert np.linalg.norm(hodlr.densify(Hk) - K, 2) <= 1e-6 * np.linalg.norm(K, 2) * 4


def test_level0_ranks_exactly_one():
    """Tridiagonal D_i: every off-diagonal HODLR block is exactly rank 1 (Section 3)."""
    st = W.varkappa(64)
    D, E, F = direct.blocks(st)
    for Di in D[:5]:
        H = hodlr.compress(Di, 16, 1e-14)
        for d, rs in hodlr.ranks(H).items():
            assert all(r == 1 for r in rs)
        assert np.abs(hodlr.densify(H) - Di).max() <= 1e-15 * np.abs(Di).max()
    for Ei in E[1:4]:
        H = hodlr.compress(Ei, 16, 1e-14)
        assert all(r == 0 for rs in hodlr.ranks(H).values() for r in rs)


# -------------------------------------------------------------------- O3 ACR
def test_acr_eps0_reproduces_bcr():
    st = W.varkappa(33)
    b = W.rhs(st.n, 2, seed=3)
    fac = acr.factor(st, 8, 0.0)
    x = acr.solve(fac, st, b)
    xb = bcr.bcr_solve(st, b)
    assert np.linalg.norm(x - xb) / np.linalg.norm(xb) < 1e-12


@pytest.mark.parametrize("stop", [2, 3, 5, 40])
def test_acr_early_stop(stop):
    """Early stop of the recursion (Section 3: the reduction may end once the
    system is small enough): with eps = 0 every stop point reproduces LU, and
    stopping at or beyond the block count is a dense solve of the whole system;
    at eps > 0 the error stays within the truncation band of the full recursion."""
    st = W.strip(W.varkappa(24), 19)          # 19 blocks of 24: odd counts on the way down
    b = W.rhs(st.n, 2, seed=5)
    xl = direct.solve(st, b)
    x0 = acr.solve(acr.factor(st, 6, 0.0, stop_blocks=stop), st, b)
    assert np.linalg.norm(x0 - xl) / np.linalg.norm(xl) < 1e-12
    fac = acr.factor(st, 6, 1e-6, stop_blocks=stop)
    nblk = st.ny
    levels = 0
    while nblk > max(stop, 1):
        nblk //= 2
        levels += 1
    assert len(fac.levels) == levels and (fac.Xdense is not None) == (nblk > 1)
    if fac.Xdense is not None:
        assert fac.Xdense.shape == (nblk * st.nx, nblk * st.nx)
    x = acr.solve(fac, st, b)
    full = acr.solve(acr.factor(st, 6, 1e-6), st, b)
    e, ef = (np.linalg.norm(v - xl) / np.linalg.norm(xl) for v in (x, full))
    assert e <= max(10 * ef, 1e-12)


def test_acr_error_decreases_with_eps():
    st = W.varkappa(64, seed=W.seed_for(1, 2))
    b = W.rhs(st.n, 1)
    x0 = direct.solve(st, b)
    errs = []
    for eps in (1e-2, 1e-4, 1e-6, 1e-8, 1e-10):
        x = acr.solve(acr.factor(st, 16, eps), st, b)
        errs.append(np.linalg.norm(x - x0) / np.linalg.norm(x0))
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1))
    assert errs[-1] < 1e-8


def test_acr_symmetry_preserved():
    """Symmetric operator: T_eps(B^T) = T_eps(B)^T, so the reduced blocks stay
    symmetric (D') and E'_{j+1} = F'_j^T, to rounding."""
    st = W.poisson(32)
    D, E, F = direct.blocks(st)
    fac = acr.factor_blocks(D, E, F, 8, 1e-8)
    for lev in range(1, len(fac.levels)):
        X, El, Fl = fac.levels[lev]
        for k, Xk in X.items():
            Xd = hodlr.densify(Xk)
            assert np.allclose(Xd, Xd.T, atol=1e-10 * np.abs(Xd).max())
        for j in range(len(El) - 1):
            Ed = hodlr.densify(El[j + 1])
            Fd = hodlr.densify(Fl[j])
            assert np.allclose(Ed, Fd.T, atol=1e-10 * np.abs(Fd).max())


def test_acr_ranks_bounded_and_memory_below_dense():
    st = W.poisson(64)
    fac = acr.factor(st, 16, 1e-8)
    assert max(acr.level_ranks(fac)) <= 16
    dense_entries = sum(64 * 64 * (len(X) + len(E) + len(F)) for X, E, F in fac.levels)
    assert acr.stored_entries(fac) < dense_entries


def test_refinement_with_acr_preconditioner():
    st = W.convdiff(48)
    b = W.rhs(st.n, 2, seed=11)
    fac = acr.factor(st, 12, 1e-4)
    x, hist = refine.refine(st, b, lambda r: acr.solve(fac, st, r), tol=1e-10, maxit=30)
    assert hist[-1] <= 1e-10
    assert direct.residual(st, x, b) <= 1e-10
    assert len(hist) - 1 <= 8


def _krylov_min_residual(A, b, k):
    """Definition of the k-th GMRES residual from x_0 = 0 without a
    preconditioner: min over x in span{b, A b, ..., A^(k-1) b} of ||b - A x||
    (least squares on an orthonormalised explicit Krylov basis)."""
    cols = [b]
    for _ in range(k - 1):
        cols.append(A @ cols[-1])
    Q, _ = np.linalg.qr(np.stack(cols, axis=1))
    AQ = A @ Q
    y = np.linalg.lstsq(AQ, b, rcond=None)[0]
    return float(np.linalg.norm(b - AQ @ y))


def test_fgmres_minimal_residual_property():
    """Unpreconditioned FGMRES after k steps (no restart) reaches the minimal
    residual over the k-th Krylov space: brute force on the nonsymmetric 36 x 36
    upwind convection-diffusion operator."""
    st = W.convdiff(6)
    A = direct.assemble(st).toarray()
    b = W.rhs(st.n, 1, seed=5)[:, 0]
    for k in (1, 2, 4, 7):
        _, its, hist = krylov.fgmres(lambda v: A @ v, b, lambda v: v, tol=0.0, maxit=k, restart=20)
        assert its == k
        ref = _krylov_min_residual(A, b, k) / np.linalg.norm(b)
        assert abs(hist[-1] - ref) <= 1e-10 * max(ref, 1e-300) + 1e-14, (k, hist[-1], ref)


def test_fgmres_exact_preconditioner_and_restarts():
    st = W.poisson(8)
    A = direct.assemble(st).toarray()
    b = W.rhs(st.n, 1, seed=6)[:, 0]
    # exact inverse: one application solves the system
    x, its, hist = krylov.fgmres(lambda v: A @ v, b, lambda v: np.linalg.solve(A, v), tol=1e-12, maxit=5)
    assert its == 1 and hist[-1] <= 1e-13
    # no preconditioner, restart 3: the true residual never grows between cycles
    x, its, hist = krylov.fgmres(lambda v: A @ v, b, lambda v: v, tol=1e-10, maxit=400, restart=3)
    assert hist[-1] <= 1e-10
    assert all(h1 <= h0 * (1 + 1e-12) for h0, h1 in zip(hist, hist[1:]))
    assert np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-8 * np.linalg.norm(np.linalg.solve(A, b))


def test_fgmres_with_acr_preconditioner():
    st = W.convdiff(48)
    b = W.rhs(st.n, 1, seed=12)[:, 0]
    A = direct.assemble(st)
    fac = acr.factor(st, 12, 1e-2)
    x, its, hist = krylov.fgmres(lambda v: A @ v, b, lambda v: acr.solve(fac, st, v), tol=1e-10, maxit=60)
    assert hist[-1] <= 1e-10
    xd = direct.solve(st, b)
    assert np.linalg.norm(x - xd) <= 1e-7 * np.linalg.norm(xd)


def test_fgmres_acr_on_indefinite_helmholtz():
    """ACR (no block pivoting) as the FGMRES preconditioner of the indefinite
    Helmholtz operator (k = 20 on a 48 x 48 grid) reaches the LU solution."""
    st = W.helmholtz(48, 20.0)
    b = W.helmholtz_rhs(48)[:, 0]
    A = direct.assemble(st)
    fac = acr.factor(st, 12, 1e-6)
    x, its, hist = krylov.fgmres(lambda v: A @ v, b, lambda v: acr.solve(fac, st, v), tol=1e-10, maxit=40)
    assert hist[-1] <= 1e-10
    xd = direct.solve(st, b)
    assert np.linalg.norm(x - xd) <= 1e-7 * np.linalg.norm(xd)


@pytest.mark.parametrize("alpha", [0.0, 30.0, 3000.0])
def test_recirculating_operator(alpha):
    """b = (cos 8 pi x, sin 8 pi y) with upwinding: an M-matrix for every alpha,
    the Poisson operator at alpha = 0, and exact on linear functions: for
    u = x + 2y the scaled operator gives h^2 alpha (b_x + 2 b_y) at nodes away
    from the boundary (the Laplacian of u vanishes, one-sided differences of a
    linear function are exact)."""
    n = 20
    st = W.recirculating(n, alpha)
    A = direct.assemble(st)
    off = A - sp.diags(A.diagonal())
    assert off.max() <= 0.0
    assert np.all(A.diagonal() + np.asarray(off.sum(axis=1)).ravel() >= -1e-12)
    if alpha == 0.0:
        assert np.allclose(A.toarray(), direct.assemble(W.poisson(n)).toarray(), atol=0, rtol=0)
    x, y = W.node_coords(n, n)
    h = 1.0 / (n + 1)
    u = x + 2 * y
    Au = (A @ u).reshape(n, n)[1:-1, 1:-1]
    bx, by = np.cos(8 * math.pi * x), np.sin(8 * math.pi * y)
    ref = (h * h * alpha * (bx + 2 * by)).reshape(n, n)[1:-1, 1:-1]
    assert np.abs(Au - ref).max() <= 1e-12 * max(1.0, alpha)


# ------------------------------------------------------- 3-D operators (NEXT)
def _grid3(st):
    h = 1.0 / (st.nx + 1)
    x = (np.arange(st.nx) + 1.0) * h
    y = (np.arange(st.ny) + 1.0) / (st.ny + 1)
    z = (np.arange(st.nz) + 1.0) / (st.nz + 1)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X.reshape(-1), Y.reshape(-1), Z.reshape(-1)


@pytest.mark.parametrize("p,q,r", [(1, 1, 1), (2, 3, 1), (5, 1, 4)])
def test_poisson3d_discrete_eigenfunction(p, q, r):
    """The 7-point Laplacian (scaled by h^2) has the eigenvectors
    sin(p pi x) sin(q pi y) sin(r pi z) with eigenvalue
    4 (sin^2(p pi h/2) + sin^2(q pi h/2) + sin^2(r pi h/2)); checked on the
    sparse assembly and on the block form (plane blocks) built separately."""
    n = 7
    st = W.poisson3d(n)
    X, Y, Z = _grid3(st)
    h = 1.0 / (n + 1)
    u = np.sin(p * math.pi * X) * np.sin(q * math.pi * Y) * np.sin(r * math.pi * Z)
    lam = 4.0 * sum(math.sin(k * math.pi * h / 2) ** 2 for k in (p, q, r))
    assert np.abs(direct.assemble3d(st) @ u - lam * u).max() <= 1e-12
    D, E, F = direct.blocks3d(st)
    s = st.s
    Au = np.zeros_like(u)
    for k in range(st.nz):
        Au[k * s:(k + 1) * s] = D[k] @ u[k * s:(k + 1) * s]
        if k > 0:
            Au[k * s:(k + 1) * s] += E[k] @ u[(k - 1) * s:k * s]
        if k + 1 < st.nz:
            Au[k * s:(k + 1) * s] += F[k] @ u[(k + 1) * s:(k + 2) * s]
    assert np.abs(Au - lam * u).max() <= 1e-12
    assert np.all(E[0] == 0) and np.all(F[-1] == 0)


def test_varkappa3d_flux_form():
    """Flux form: symmetric, off-diagonals <= 0, zero row sum at nodes away from
    the boundary (the diagonal is the sum of the six face coefficients), and
    the face contrast is at most the requested 1e3."""
    st = W.varkappa3d(10)
    A = direct.assemble3d(st)
    assert abs(A - A.T).max() == 0.0
    off = A - sp.diags(A.diagonal())
    assert off.max() <= 0.0
    rs = np.asarray(A.sum(axis=1)).ravel().reshape(10, 10, 10)
    assert np.abs(rs[1:-1, 1:-1, 1:-1]).max() <= 1e-12 * st.diag.max()
    faces = -np.concatenate([a[a != 0] for a in (st.west, st.east, st.south, st.north, st.down, st.up)])
    assert faces.max() / faces.min() <= 1e3 * (1 + 1e-12)


@pytest.mark.parametrize("nx,ny,leaf", [(8, 8, 16), (16, 8, 32), (32, 4, 16)])
def test_plane_operator_exact_hodlr_ranks(nx, ny, leaf):
    """A plane's five-point operator with the halving split has off-diagonal
    blocks of exact rank nx where the two clusters hold whole rows (the y
    couplings across the split) and rank 1 inside a row (the x coupling);
    E_k, F_k are diagonal (rank 0 off the leaves)."""
    st = W.varkappa3d(8) if (nx, ny) == (8, 8) else None
    if st is None:
        p = W.poisson3d(nx, ny, 4)
        rng = np.random.default_rng(5)
        for a in (p.west, p.east, p.south, p.north):
            a *= rng.uniform(0.5, 2.0, a.size) * (a != 0)
        st = p
    D, E, F = direct.blocks3d(st)
    s = st.s
    for Dk in D[:2]:
        H = hodlr.compress(Dk, leaf, 1e-14)
        for d, rs in hodlr.ranks(H).items():
            sd = s >> d
            want = nx if sd % nx == 0 else 1
            assert all(r == want for r in rs), (d, rs, want)
        assert np.abs(hodlr.densify(H) - Dk).max() <= 1e-14 * np.abs(Dk).max()
    H = hodlr.compress(E[1], leaf, 1e-14)
    assert all(r == 0 for rs in hodlr.ranks(H).values() for r in rs)


def test_acr3d_eps0_equals_lu_and_error_decreases():
    """ACR over the planes of a 3-D operator: eps = 0 is exact (sparse LU), and
    the error decreases with eps."""
    st = W.varkappa3d(8)
    D, E, F = direct.blocks3d(st)
    s = st.s
    b = W.rhs(st.n, 2, seed=31)
    xd = direct.solve3d(st, b)
    errs = []
    for eps in (0.0, 1e-8, 1e-4, 1e-2):
        fac = acr.factor_blocks(D, E, F, 16, eps)
        x = np.concatenate(acr.solve_blocks(fac, [b[k * s:(k + 1) * s] for k in range(st.nz)]), axis=0)
        errs.append(np.linalg.norm(x - xd) / np.linalg.norm(xd))
    assert errs[0] <= 1e-12
    assert errs[1] <= 1e-6
    assert errs[1] <= errs[2] <= errs[3]


def test_fgmres_with_acr3d_preconditioner():
    """A coarse ACR factor of a 3-D operator as the FGMRES preconditioner
    reaches the sparse-LU solution."""
    st = W.varkappa3d(8)
    D, E, F = direct.blocks3d(st)
    s = st.s
    A = direct.assemble3d(st)
    b = W.rhs(st.n, 1, seed=32)[:, 0]
    fac = acr.factor_blocks(D, E, F, 16, 1e-2)
    apply = lambda v: np.concatenate(acr.solve_blocks(fac, [v[k * s:(k + 1) * s] for k in range(st.nz)]))
    x, its, hist = krylov.fgmres(lambda v: A @ v, b, apply, tol=1e-10, maxit=40)
    assert hist[-1] <= 1e-10
    xd = direct.solve3d(st, b)
    assert np.linalg.norm(x - xd) <= 1e-7 * np.linalg.norm(xd)

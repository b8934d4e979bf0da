"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only *generates problems*: 5-point stencil coefficients of 2-D
elliptic operators on the unit square with homogeneous Dirichlet data, and
random right-hand sides.  It holds none of the solver's arithmetic (no cyclic
reduction, no hierarchical compression, no factorisation), so both the CPU
oracle and the GPU path can consume its outputs without sharing any of the
method.

Operator form (the block-tridiagonal system of the paper's Section 3, Eq.
"system"): unknowns live on the interior nodes of an ``nx`` by ``ny`` grid,
index ``i*nx + j`` with ``i`` the grid row (y, the block index) and ``j`` the
column (x, position inside a block).  A stencil is five arrays of length
``N = nx*ny``::

    (A u)[i,j] = diag*u[i,j] + west*u[i,j-1] + east*u[i,j+1]
                 + south*u[i-1,j] + north*u[i+1,j]

so block row ``i`` has ``D_i = tridiag(west, diag, east)`` (restricted to row
``i``), ``E_i = diag(south)`` and ``F_i = diag(north)``.  Couplings that would
leave the grid are stored as exact zeros.  All operators are scaled by the
cell area (``A = hx*hy * L_h``) so entries are O(1).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 160400617


def seed_for(config_id: int, k: int) -> int:
    """Seed convention: base + 100*config + k (k separates independent fields)."""
    return SEED_BASE + 100 * int(config_id) + int(k)


@dataclasses.dataclass
class Stencil:
    nx: int          # block size (unknowns per grid row)
    ny: int          # number of blocks (grid rows)
    diag: np.ndarray
    west: np.ndarray
    east: np.ndarray
    south: np.ndarray
    north: np.ndarray
    name: str = ""

    @property
    def n(self) -> int:
        return self.nx * self.ny

    def arrays(self):
        return (self.diag, self.west, self.east, self.south, self.north)


def _zero_outside(nx, ny, west, east, south, north):
    west = west.reshape(ny, nx)
    east = east.reshape(ny, nx)
    south = south.reshape(ny, nx)
    north = north.reshape(ny, nx)
    west[:, 0] = 0.0
    east[:, nx - 1] = 0.0
    south[0, :] = 0.0
    north[ny - 1, :] = 0.0


def poisson(nx: int, ny: int | None = None) -> Stencil:
    """Constant-coefficient -Laplace, 5-point, scaled by hx*hy."""
    ny = nx if ny is None else ny
    hx, hy = 1.0 / (nx + 1), 1.0 / (ny + 1)
    ax, ay = hy / hx, hx / hy
    n = nx * ny
    diag = np.full(n, 2.0 * ax + 2.0 * ay)
    west = np.full(n, -ax)
    east = np.full(n, -ax)
    south = np.full(n, -ay)
    north = np.full(n, -ay)
    _zero_outside(nx, ny, west, east, south, north)
    return Stencil(nx, ny, diag, west, east, south, north, name="poisson")


def flux_form(kx_face: np.ndarray, ky_face: np.ndarray, nx: int, ny: int,
              name: str = "varkappa") -> Stencil:
    """-div(kappa grad u) in flux form with kappa given on cell faces.

    ``kx_face[i, f]`` (shape ny x (nx+1)) is kappa on the vertical face between
    node (i, f-1) and (i, f) (f = 0 is the face next to the west boundary);
    ``ky_face[f, j]`` (shape (ny+1) x nx) likewise between rows f-1 and f.
    """
    hx, hy = 1.0 / (nx + 1), 1.0 / (ny + 1)
    ax, ay = hy / hx, hx / hy
    kw = kx_face[:, :nx]
    ke = kx_face[:, 1:]
    ks = ky_face[:ny, :]
    kn = ky_face[1:, :]
    diag = (ax * (kw + ke) + ay * (ks + kn)).reshape(-1).astype(np.float64)
    west = (-ax * kw).reshape(-1).astype(np.float64).copy()
    east = (-ax * ke).reshape(-1).astype(np.float64).copy()
    south = (-ay * ks).reshape(-1).astype(np.float64).copy()
    north = (-ay * kn).reshape(-1).astype(np.float64).copy()
    _zero_outside(nx, ny, west, east, south, north)
    return Stencil(nx, ny, diag, west, east, south, north, name=name)


def kappa_faces_from_function(fun, nx: int, ny: int):
    """Sample kappa(x, y) at the face midpoints of the grid."""
    hx, hy = 1.0 / (nx + 1), 1.0 / (ny + 1)
    xs_face = (np.arange(nx + 1) + 0.5) * hx      # x of vertical faces
    ys_node = (np.arange(ny) + 1.0) * hy
    xs_node = (np.arange(nx) + 1.0) * hx
    ys_face = (np.arange(ny + 1) + 0.5) * hy
    X, Y = np.meshgrid(xs_face, ys_node)
    kx = fun(X, Y)
    X, Y = np.meshgrid(xs_node, ys_face)
    ky = fun(X, Y)
    return kx, ky


def gaussian_random_field(npts_x: int, npts_y: int, spacing: float, length: float,
                          rng: np.random.Generator) -> np.ndarray:
    """Stationary Gaussian field with covariance exp(-r^2 / (2 length^2)).

    Spectral synthesis on a periodic box at least twice the sampled extent (so
    the periodic wrap-around of the covariance is negligible for the short
    correlation lengths used here), then normalised to zero mean and unit
    sample variance over the returned points.  Shape (npts_y, npts_x).
    """
    pad = int(math.ceil(8.0 * length / spacing))
    m = 1
    while m < max(npts_x, npts_y) + pad:
        m *= 2
    box = m * spacing
    k = np.fft.fftfreq(m, d=spacing)                  # cycles per unit length
    kx, ky = np.meshgrid(k, k)
    spec = 2.0 * math.pi * length ** 2 * np.exp(-2.0 * math.pi ** 2 * length ** 2 * (kx ** 2 + ky ** 2))
    amp = np.sqrt(spec) / box
    noise = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    field = np.real(np.fft.ifft2(amp * noise)) * (m * m)
    g = field[:npts_y, :npts_x]
    g = g - g.mean()
    sd = g.std()
    return g / sd if sd > 0 else g


def varkappa(nx: int, ny: int | None = None, seed: int = seed_for(2, 0),
             length: float = 0.05, contrast: float = 1e4) -> Stencil:
    """kappa = exp(g), g a squared-exponential Gaussian random field.

    g is sampled on the half-spacing grid (so every face midpoint is a sample
    point), scaled so that max(kappa)/min(kappa) over the face samples equals
    ``contrast`` exactly.
    """
    ny = nx if ny is None else ny
    hx, hy = 1.0 / (nx + 1), 1.0 / (ny + 1)
    if abs(hx - hy) > 1e-15:
        raise ValueError("varkappa samples the field on a square half-grid; use nx == ny")
    rng = np.random.default_rng(seed)
    npts = 2 * (nx + 1) + 1
    g = gaussian_random_field(npts, npts, hx / 2.0, length, rng)
    # face (i, f) of a vertical face: x index 2f+1, y index 2(i+1)
    iy = 2 * (np.arange(ny) + 1)
    fx = 2 * np.arange(nx + 1) + 1
    gx = g[np.ix_(iy, fx)]
    jx = 2 * (np.arange(nx) + 1)
    fy = 2 * np.arange(ny + 1) + 1
    gy = g[np.ix_(fy, jx)]
    lo = min(gx.min(), gy.min())
    hi = max(gx.max(), gy.max())
    scale = math.log(contrast) / (hi - lo)
    mid = 0.5 * (hi + lo)
    kx = np.exp((gx - mid) * scale)
    ky = np.exp((gy - mid) * scale)
    return flux_form(kx, ky, nx, ny, name="varkappa")


def convdiff(nx: int, ny: int | None = None, seed: int = seed_for(4, 0),
             beta: float = 1000.0, length: float = 0.1) -> Stencil:
    """-Laplace u + b . grad u with first-order upwinding, scaled by hx*hy.

    b = beta * (cos theta, sin theta) at the nodes, theta = pi * g with g a
    unit-variance squared-exponential field of correlation length ``length``.
    """
    ny = nx if ny is None else ny
    hx, hy = 1.0 / (nx + 1), 1.0 / (ny + 1)
    rng = np.random.default_rng(seed)
    g = gaussian_random_field(nx, ny, min(hx, hy), length, rng)
    theta = math.pi * g
    bx = (beta * np.cos(theta)).reshape(-1)
    by = (beta * np.sin(theta)).reshape(-1)
    return _upwind(nx, ny, bx, by, "convdiff")


def _upwind(nx, ny, bx, by, name):
    """-Laplace u + b . grad u, first-order upwinding, scaled by hx*hy (b at the nodes)."""
    hx, hy = 1.0 / (nx + 1), 1.0 / (ny + 1)
    base = poisson(nx, ny)
    # cell-area scaling: x-derivative terms carry hy, y-derivative terms carry hx
    bxp, bxm = np.maximum(bx, 0.0), np.minimum(bx, 0.0)
    byp, bym = np.maximum(by, 0.0), np.minimum(by, 0.0)
    diag = base.diag + hy * np.abs(bx) + hx * np.abs(by)
    west = base.west - hy * bxp
    east = base.east + hy * bxm
    south = base.south - hx * byp
    north = base.north + hx * bym
    _zero_outside(nx, ny, west, east, south, north)
    return Stencil(nx, ny, diag, west, east, south, north, name=name)


def recirculating(nx: int, alpha: float, ny: int | None = None) -> Stencil:
    """The paper's recirculating-flow problem -Laplace u + alpha b . grad u with
    b = (cos 8 pi x, sin 8 pi y), first-order upwinding, scaled by hx*hy."""
    ny = nx if ny is None else ny
    x, y = node_coords(nx, ny)
    return _upwind(nx, ny, alpha * np.cos(8 * math.pi * x), alpha * np.sin(8 * math.pi * y), "recirculating")


def rhs(n: int, nrhs: int = 1, seed: int = seed_for(1, 9)) -> np.ndarray:
    """Right-hand sides ~ N(0, 1), shape (n, nrhs), Fortran (column-major) order."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((nrhs, n)).T)


def node_coords(nx: int, ny: int):
    """Interior node coordinates (x, y) flattened in unknown order i*nx + j."""
    hx, hy = 1.0 / (nx + 1), 1.0 / (ny + 1)
    x = (np.arange(nx) + 1.0) * hx
    y = (np.arange(ny) + 1.0) * hy
    X, Y = np.meshgrid(x, y)
    return X.reshape(-1), Y.reshape(-1)


def helmholtz(nx: int, kwave: float, ny: int | None = None) -> Stencil:
    """Helmholtz operator of the paper's first experiment, written with the sign
    of the Laplace operators here: -Laplace u - k^2 u (= -f for the paper's
    Laplace u + k^2 u = f), 5-point, scaled by hx*hy.  Indefinite once k^2 exceeds
    the smallest Dirichlet eigenvalue 2 pi^2."""
    st = poisson(nx, ny)
    hx, hy = 1.0 / (st.nx + 1), 1.0 / (st.ny + 1)
    st.diag = st.diag - kwave * kwave * hx * hy
    st.name = "helmholtz"
    return st


def helmholtz_rhs(nx: int, ny: int | None = None) -> np.ndarray:
    """The paper's source f = 100 exp(-100 ((x - 1/2)^2 + (y - 1/2)^2)) at the
    nodes, as the right-hand side of -Laplace u - k^2 u = -f scaled by hx*hy;
    shape (n, 1), column-major."""
    ny = nx if ny is None else ny
    x, y = node_coords(nx, ny)
    f = 100.0 * np.exp(-100.0 * ((x - 0.5) ** 2 + (y - 0.5) ** 2))
    hx, hy = 1.0 / (nx + 1), 1.0 / (ny + 1)
    return np.asfortranarray((-hx * hy * f).reshape(-1, 1))


# Named workloads (grid side, operator family, leaf, eps, nrhs).
CONFIGS = {
    1: dict(kind="poisson", n=64, leaf=16, eps=1e-10, nrhs=1),
    2: dict(kind="varkappa", n=1024, leaf=64, eps=1e-6, nrhs=1),
    3: dict(kind="batched", sides=(64, 96, 128, 192, 256), count=256, leaf=32, eps=1e-8, nrhs=8),
    4: dict(kind="convdiff", n=512, leaf=64, eps=1e-7, nrhs=64),
}


def make(kind: str, n: int, config_id: int = 0) -> Stencil:
    if kind == "poisson":
        return poisson(n)
    if kind == "varkappa":
        return varkappa(n, seed=seed_for(config_id or 2, 0))
    if kind == "convdiff":
        return convdiff(n, seed=seed_for(config_id or 4, 1))
    raise ValueError(kind)


def strip(st: Stencil, rows: int, first: int = 0) -> Stencil:
    """The block rows [first, first + rows) of an operator as an operator of its own
    (same block size and coefficients; the couplings to the rows outside are dropped,
    i.e. Dirichlet zeros there).  A bounded sample of a large workload with its real
    block shapes."""
    if not (0 <= first and rows >= 1 and first + rows <= st.ny):
        raise ValueError("strip outside the operator")
    lo, hi = first * st.nx, (first + rows) * st.nx
    arr = [a[lo:hi].copy() for a in st.arrays()]
    arr[3][: st.nx] = 0.0                  # south of the first row
    arr[4][(rows - 1) * st.nx:] = 0.0      # north of the last row
    return Stencil(st.nx, rows, *arr, name=f"{st.name}-strip{rows}")


# ---------------------------------------------------------------------------
# 3-D operators: 7-point stencils on the unit cube (the block-tridiagonal form
# with one block per z plane, Section 4's closing remarks on 3-D problems).
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Stencil3:
    """7-point stencil on the interior nodes of an nx x ny x nz grid, unknown
    index ``(k*ny + i)*nx + j`` (k the plane z, i the row y, j the column x)::

        (A u)[k,i,j] = diag*u + west*u[k,i,j-1] + east*u[k,i,j+1]
                       + south*u[k,i-1,j] + north*u[k,i+1,j]
                       + down*u[k-1,i,j] + up*u[k+1,i,j]

    As a block-tridiagonal system the block is one plane (s = nx*ny unknowns,
    D_k the plane's 5-point operator), E_k = diag(down), F_k = diag(up), and
    there are nz blocks.  Couplings that would leave the grid are exact zeros.
    Operators are scaled by h^2 (h the mesh width), so entries are O(1)."""
    nx: int
    ny: int
    nz: int
    diag: np.ndarray
    west: np.ndarray
    east: np.ndarray
    south: np.ndarray
    north: np.ndarray
    down: np.ndarray
    up: np.ndarray
    name: str = ""

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def s(self) -> int:
        return self.nx * self.ny

    def arrays(self):
        return (self.diag, self.west, self.east, self.south, self.north, self.down, self.up)


def _zero_outside3(nx, ny, nz, west, east, south, north, down, up):
    for a in (west, east, south, north, down, up):
        assert a.shape == (nx * ny * nz,)
    west.reshape(nz, ny, nx)[:, :, 0] = 0.0
    east.reshape(nz, ny, nx)[:, :, nx - 1] = 0.0
    south.reshape(nz, ny, nx)[:, 0, :] = 0.0
    north.reshape(nz, ny, nx)[:, ny - 1, :] = 0.0
    down.reshape(nz, ny, nx)[0] = 0.0
    up.reshape(nz, ny, nx)[nz - 1] = 0.0


def poisson3d(n: int, ny: int | None = None, nz: int | None = None) -> Stencil3:
    """Constant-coefficient -Laplace, 7-point, on a cube grid of equal spacing
    h = 1/(n+1) in every direction (ny, nz default to n), scaled by h^2."""
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    N = n * ny * nz
    diag = np.full(N, 6.0)
    arr = [np.full(N, -1.0) for _ in range(6)]
    _zero_outside3(n, ny, nz, *arr)
    return Stencil3(n, ny, nz, diag, *arr, name="poisson3d")


def random_fourier_field(points: np.ndarray, length: float, rng: np.random.Generator,
                         features: int = 512) -> np.ndarray:
    """Approximately stationary Gaussian field with covariance exp(-r^2/(2 length^2))
    at the given points (shape (..., dim)): sqrt(2/M) sum_m cos(w_m . x + b_m) with
    w_m ~ N(0, I/length^2) and b_m ~ U(0, 2 pi) (random Fourier features),
    normalised to zero mean and unit variance over the points."""
    dim = points.shape[-1]
    w = rng.standard_normal((features, dim)) / length
    b = rng.uniform(0.0, 2.0 * math.pi, features)
    flat = points.reshape(-1, dim)
    g = np.empty(flat.shape[0])
    for lo in range(0, flat.shape[0], 65536):   # bounded memory
        ph = flat[lo:lo + 65536] @ w.T + b
        g[lo:lo + 65536] = np.sqrt(2.0 / features) * np.cos(ph).sum(axis=1)
    g = g - g.mean()
    sd = g.std()
    return (g / sd if sd > 0 else g).reshape(points.shape[:-1])


def varkappa3d(n: int, seed: int = seed_for(6, 0), length: float = 0.1,
               contrast: float = 1e3) -> Stencil3:
    """-div(kappa grad u) on the n^3 cube grid in flux form, kappa = exp(g) at the
    face midpoints with g a random Fourier field, scaled so that
    max(kappa)/min(kappa) over the face samples equals ``contrast``; scaled by h^2."""
    h = 1.0 / (n + 1)
    rng = np.random.default_rng(seed)
    node = (np.arange(n) + 1.0) * h
    face = (np.arange(n + 1) + 0.5) * h
    # faces normal to x: (z node, y node, x face); to y: (z, y face, x); to z: (z face, y, x)
    def pts(zs, ys, xs):
        Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
        return np.stack([X, Y, Z], axis=-1)
    px, py, pz = pts(node, node, face), pts(node, face, node), pts(face, node, node)
    allp = np.concatenate([px.reshape(-1, 3), py.reshape(-1, 3), pz.reshape(-1, 3)])
    g = random_fourier_field(allp, length, rng)
    lo, hi = g.min(), g.max()
    scale = math.log(contrast) / (hi - lo)
    k = np.exp((g - 0.5 * (hi + lo)) * scale)
    nxf = px.shape[0] * px.shape[1] * px.shape[2]
    nyf = py.shape[0] * py.shape[1] * py.shape[2]
    kx = k[:nxf].reshape(n, n, n + 1)
    ky = k[nxf:nxf + nyf].reshape(n, n + 1, n)
    kz = k[nxf + nyf:].reshape(n + 1, n, n)
    kw, ke = kx[:, :, :n], kx[:, :, 1:]
    ks, kn = ky[:, :n, :], ky[:, 1:, :]
    kd, ku = kz[:n], kz[1:]
    diag = (kw + ke + ks + kn + kd + ku).reshape(-1).copy()
    arr = [(-a).reshape(-1).copy() for a in (kw, ke, ks, kn, kd, ku)]
    _zero_outside3(n, n, n, *arr)
    return Stencil3(n, n, n, diag, *arr, name="varkappa3d")

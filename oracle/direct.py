"""Plain definition of the solution: assemble A and solve by LU (oracle O1).

The block-tridiagonal matrix is the paper's Eq. "system" (Section 3):
A = tridiag(E_i, D_i, F_i), D_i tridiagonal, E_i and F_i diagonal, obtained
from a 5-point discretisation (Eq. "probSta").  Test infrastructure only.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def assemble(st) -> sp.csr_matrix:
    """Sparse A from a ``workloads.Stencil`` (unknown index i*nx + j)."""
    nx, ny = st.nx, st.ny
    n = nx * ny
    idx = np.arange(n)
    rows = [idx]
    cols = [idx]
    vals = [st.diag]
    for arr, off in ((st.west, -1), (st.east, 1), (st.south, -nx), (st.north, nx)):
        nz = arr != 0.0
        r = idx[nz]
        rows.append(r)
        cols.append(r + off)
        vals.append(arr[nz])
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    return A


def block(st, i):
    """Dense blocks D_i, E_i, F_i (s x s) of block row i of Eq. "system" (block = grid row)."""
    s = st.nx
    sl = slice(i * s, (i + 1) * s)
    Di = np.diag(st.diag[sl]) + np.diag(st.west[sl][1:], -1) + np.diag(st.east[sl][:-1], 1)
    return Di, np.diag(st.south[sl]), np.diag(st.north[sl])


def blocks(st):
    """Dense blocks D_i (s x s), E_i, F_i (s x s) of Eq. "system" (block = grid row)."""
    D, E, F = [], [], []
    for i in range(st.ny):
        Di, Ei, Fi = block(st, i)
        D.append(Di)
        E.append(Ei)
        F.append(Fi)
    return D, E, F


def solve(st, b: np.ndarray) -> np.ndarray:
    """x = A^{-1} b by LU with partial pivoting (dense for small N, SuperLU otherwise)."""
    A = assemble(st)
    b2 = b.reshape(A.shape[0], -1)
    if A.shape[0] <= 4096:
        x = np.linalg.solve(A.toarray(), b2)
    else:
        lu = spla.splu(A.tocsc())
        x = lu.solve(np.ascontiguousarray(b2))
    return x.reshape(b.shape)


def residual(st, x: np.ndarray, b: np.ndarray) -> float:
    """Relative residual ||b - A x||_2 / ||b||_2 in FP64 (per column max)."""
    A = assemble(st)
    x2 = x.reshape(A.shape[0], -1)
    b2 = b.reshape(A.shape[0], -1)
    r = b2 - A @ x2
    return float(np.max(np.linalg.norm(r, axis=0) / np.linalg.norm(b2, axis=0)))


# --- 3-D operators (one block per z plane; Section 4, closing remarks) ---

def assemble3d(st) -> sp.csr_matrix:
    """Sparse A from a ``workloads.Stencil3`` (unknown index (k*ny + i)*nx + j)."""
    nx, ny = st.nx, st.ny
    n = st.n
    idx = np.arange(n)
    rows, cols, vals = [idx], [idx], [st.diag]
    offs = ((st.west, -1), (st.east, 1), (st.south, -nx), (st.north, nx), (st.down, -nx * ny), (st.up, nx * ny))
    for arr, off in offs:
        nz = arr != 0.0
        r = idx[nz]
        rows.append(r)
        cols.append(r + off)
        vals.append(arr[nz])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))


def blocks3d(st):
    """Dense blocks of the block-tridiagonal form of a 3-D operator: block k is
    the plane z = k, D_k its 5-point operator (s = nx*ny), E_k = diag(down),
    F_k = diag(up)."""
    s = st.nx * st.ny
    D, E, F = [], [], []
    for k in range(st.nz):
        sl = slice(k * s, (k + 1) * s)
        Dk = np.diag(st.diag[sl]) + np.diag(st.west[sl][1:], -1) + np.diag(st.east[sl][:-1], 1)
        Dk += np.diag(st.south[sl][st.nx:], -st.nx) + np.diag(st.north[sl][:-st.nx], st.nx)
        D.append(Dk)
        E.append(np.diag(st.down[sl]))
        F.append(np.diag(st.up[sl]))
    return D, E, F


def solve3d(st, b: np.ndarray) -> np.ndarray:
    """x = A^{-1} b for a 3-D operator by sparse LU."""
    A = assemble3d(st).tocsc()
    b2 = b.reshape(A.shape[0], -1)
    return spla.splu(A).solve(np.ascontiguousarray(b2)).reshape(b.shape)

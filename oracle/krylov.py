"""Restarted flexible GMRES with a right preconditioner (oracle O6).

The paper proposes ACR as a preconditioner whose accuracy is tuned by the
truncation tolerance (Section 4, closing paragraph; Section 5).  Where plain
refinement (``refine``) contracts slowly or not at all, a Krylov method
around the same preconditioner is the natural alternative.  This is the
textbook right-preconditioned FGMRES(m), written out plainly in FP64:

    x_0 = 0.  Each cycle:  r = b - A x,  beta = ||r||,  v_0 = r / beta;
    for j = 0 .. m-1:
        z_j = M^{-1} v_j,   w = A z_j,
        h_ij = v_i . w  and  w -= h_ij v_i  (i <= j; the projection is done twice,
        classical Gram-Schmidt, and the two coefficient sets added),
        h_(j+1) j = ||w||,  v_(j+1) = w / h_(j+1) j;
    y = argmin || beta e_1 - H y ||  (the (j+1) x j Hessenberg matrix H),
    x <- x + Z y.
    Stop when ||b - A x|| / ||b|| <= tol or after maxit applications of M^{-1}.

The least-squares problem is solved with numpy's lstsq (no Givens rotations:
the plainest correct form).  Test infrastructure only.
"""
from __future__ import annotations

import numpy as np


def fgmres(matvec, b: np.ndarray, apply_minv, tol: float = 1e-10, maxit: int = 100, restart: int = 20):
    """Returns (x, number of M^{-1} applications, list of true relative residuals per cycle)."""
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    x = np.zeros_like(b)
    its = 0
    hist = []
    while True:
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        rel = beta / nb if nb > 0 else beta
        hist.append(rel)
        if not rel > tol or its >= maxit:
            break
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart))
        k = 0
        for j in range(restart):
            if its >= maxit:
                break
            Z.append(apply_minv(V[j]))
            its += 1
            w = matvec(Z[j])
            for _ in range(2):
                c = np.array([v @ w for v in V])
                w = w - sum(ci * v for ci, v in zip(c, V))
                H[: j + 1, j] += c
            H[j + 1, j] = np.linalg.norm(w)
            k = j + 1
            e1 = np.zeros(k + 1)
            e1[0] = beta
            y = np.linalg.lstsq(H[: k + 1, :k], e1, rcond=None)[0]
            est = np.linalg.norm(e1 - H[: k + 1, :k] @ y) / (nb if nb > 0 else 1.0)
            if H[j + 1, j] == 0.0 or not est > tol:
                break
            V.append(w / H[j + 1, j])
        e1 = np.zeros(k + 1)
        e1[0] = beta
        y = np.linalg.lstsq(H[: k + 1, :k], e1, rcond=None)[0]
        x = x + sum(yi * z for yi, z in zip(y, Z))
    return x, its, hist


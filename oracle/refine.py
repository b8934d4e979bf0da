"""Iterative refinement with an FP64 residual (oracle O5).

The paper proposes using ACR as a preconditioner whose accuracy is tuned by
the truncation tolerance (Section 4, closing paragraph; Section 5).  The
plainest such use is stationary iterative refinement:

    x_0 = 0;  repeat  r = b - A x (FP64),  x <- x + M^{-1} r
    until ||b - A x||_2 / ||b||_2 <= tol  or  maxit corrections.

``apply_minv`` is any approximate inverse (e.g. an ACR solve).  Test
infrastructure only.
"""
from __future__ import annotations

import numpy as np

from .direct import assemble


def refine(st, b: np.ndarray, apply_minv, tol: float = 1e-10, maxit: int = 50):
    A = assemble(st)
    b2 = b.reshape(A.shape[0], -1)
    nb = np.linalg.norm(b2, axis=0)
    x = np.zeros_like(b2)
    hist = []
    r = b2.copy()
    for it in range(maxit + 1):
        rel = float(np.max(np.linalg.norm(r, axis=0) / nb))
        hist.append(rel)
        if rel <= tol or it == maxit:
            break
        x = x + apply_minv(r)
        r = b2 - A @ x
    return x.reshape(b.shape), hist

"""Exact block cyclic reduction with dense FP64 blocks (oracle O2).

Section 3 of the paper: the reduction phase is block Gaussian elimination
without pivoting on the even/odd permuted system; the even-indexed diagonal
blocks form a block-diagonal H11 whose inverse is the set of independent block
inverses, and the Schur complement H22 - H21 H11^{-1} H12 (Eq. "fund") is again
block tridiagonal, so the step recurses until one block is left; a
back-substitution recovers every unknown.

Written block-wise for block rows 0..m-1 of one level (E_0 = 0, F_{m-1} = 0),
eliminating the even indices k and keeping the odd ones i = 2j+1:

    X_k = D_k^{-1},  P_k = X_k E_k,  Q_k = X_k F_k
    D'_j = D_i - E_i Q_{i-1} - F_i P_{i+1}      (last term only if i+1 < m)
    E'_j = -E_i P_{i-1}                          (zero for j = 0: E_0 = 0)
    F'_j = -F_i Q_{i+1}                          (only if i+1 < m)
    f'_j = f_i - E_i X_{i-1} f_{i-1} - F_i X_{i+1} f_{i+1}

and the back-substitution of the eliminated rows is
u_k = X_k (f_k - E_k u_{k-1} - F_k u_{k+1}).  The next level has floor(m/2)
blocks; the paper's 8-block example takes 3 levels to reach one block.
Test infrastructure only.
"""
from __future__ import annotations

import numpy as np


def level_sizes(m: int):
    """Block counts per level: m, floor(m/2), ... down to 1."""
    sizes = [m]
    while sizes[-1] > 1:
        sizes.append(sizes[-1] // 2)
    return sizes


def reduce_level(D, E, F, inv=np.linalg.inv, mul=lambda a, b: a @ b,
                 combine=lambda terms: sum(terms[1:], terms[0])):
    """One reduction step on dense block lists; returns (X, D', E', F').

    ``inv``, ``mul`` and ``combine`` default to exact dense arithmetic.
    """
    m = len(D)
    s = D[0].shape[0]
    Z = np.zeros((s, s))
    X, P, Q = {}, {}, {}
    for k in range(0, m, 2):
        X[k] = inv(D[k])
        P[k] = mul(X[k], E[k])
        Q[k] = mul(X[k], F[k])
    Dn, En, Fn = [], [], []
    for i in range(1, m, 2):
        terms = [D[i], -mul(E[i], Q[i - 1])]
        if i + 1 < m:
            terms.append(-mul(F[i], P[i + 1]))
        Dn.append(combine(terms))
        En.append(-mul(E[i], P[i - 1]))
        Fn.append(-mul(F[i], Q[i + 1]) if i + 1 < m else Z.copy())
    return X, Dn, En, Fn


def factor(D, E, F):
    """Full reduction; returns the list of per-level (X, E, F) and the last X."""
    levels = []
    while len(D) > 1:
        X, Dn, En, Fn = reduce_level(D, E, F)
        levels.append((X, E, F))
        D, E, F = Dn, En, Fn
    return levels, np.linalg.inv(D[0])


def solve(levels, Xlast, f_blocks):
    """Forward reduction of the right-hand side, final block, back-substitution."""
    fs = [list(f_blocks)]
    for X, E, F in levels:
        f = fs[-1]
        m = len(f)
        g = {k: X[k] @ f[k] for k in range(0, m, 2)}
        fn = []
        for i in range(1, m, 2):
            v = f[i] - E[i] @ g[i - 1]
            if i + 1 < m:
                v = v - F[i] @ g[i + 1]
            fn.append(v)
        fs.append(fn)
    u = [Xlast @ fs[-1][0]]
    for lev in range(len(levels) - 1, -1, -1):
        X, E, F = levels[lev]
        f = fs[lev]
        m = len(f)
        un = [None] * m
        for j, v in enumerate(u):
            un[2 * j + 1] = v
        for k in range(0, m, 2):
            rhs = f[k].copy()
            if k - 1 >= 0:
                rhs = rhs - E[k] @ un[k - 1]
            if k + 1 < m:
                rhs = rhs - F[k] @ un[k + 1]
            un[k] = X[k] @ rhs
        u = un
    return u


def bcr_solve(st, b):
    """x = A^{-1} b by exact dense BCR (b: (N,) or (N, nrhs))."""
    from .direct import blocks
    D, E, F = blocks(st)
    levels, Xl = factor(D, E, F)
    s = st.nx
    b2 = b.reshape(st.n, -1)
    f = [b2[i * s:(i + 1) * s] for i in range(st.ny)]
    u = solve(levels, Xl, f)
    return np.concatenate(u, axis=0).reshape(b.shape)

"""Accelerated Cyclic Reduction on the CPU (oracle O3, FP64).

Section 3 of the paper: block cyclic reduction in which every block that
arises is approximated by a HODLR matrix and the dense arithmetic of each
step (block inverse, block product, block sum) is replaced by H-arithmetic.
The H-arithmetic is realised here in its plainest form, formatted arithmetic
with best truncation: each operation is evaluated exactly on the *stored*
(already truncated) operands and its result is stored as ``compress(., eps)``
(every off-diagonal block cut by T_eps, leaves exact).  One CR level, with
the same index conventions as the exact oracle in ``bcr``:

    X_k  = T(D_k^{-1})                        even k (independent inverses)
    P_k  = T(X_k E_k),   Q_k = T(X_k F_k)
    D'_j = T(D_i - E_i Q_{i-1} - F_i P_{i+1})  odd i = 2j+1, one truncation
    E'_j = T(-E_i P_{i-1}),  F'_j = T(-F_i Q_{i+1})

until one block remains, whose inverse is T(D^{-1}).  The solve (forward
reduction of the right-hand side, final block, back-substitution
u_k = X_k (f_k - E_k u_{k-1} - F_k u_{k+1})) applies the stored HODLR blocks
with HODLR matvecs.  With eps = 0 nothing is truncated and the result is the
exact BCR of ``bcr``.  Test infrastructure only.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import hodlr
from .direct import blocks


@dataclass
class Factor:
    leaf: int
    eps: float
    levels: list = field(default_factory=list)   # per level: (X dict, E list, F list)
    Xlast: object = None
    Xdense: object = None    # early stop: inverse of the remaining block-tridiagonal system


def factor_blocks(D, E, F, leaf: int, eps: float, stop_blocks: int = 1) -> Factor:
    """ACR reduction of dense level-0 blocks (lists of s x s arrays).

    The recursion may stop early (Section 3: the reduction can end once the
    system is small enough): levels run while more than ``stop_blocks`` blocks
    remain, and the remaining block-tridiagonal system (its stored blocks) is
    then inverted as one dense matrix, without truncation."""
    T = lambda M: hodlr.compress(M, leaf, eps)
    dn = hodlr.densify
    fac = Factor(leaf, eps)
    # Level 0: D_i tridiagonal (exact rank-1 off-diagonal blocks), E_i/F_i diagonal.
    Dh = [T(Di) for Di in D]
    Eh = [T(Ei) for Ei in E]
    Fh = [T(Fi) for Fi in F]
    while len(Dh) > max(stop_blocks, 1):
        m = len(Dh)
        X, P, Q = {}, {}, {}
        for k in range(0, m, 2):
            X[k] = T(np.linalg.inv(dn(Dh[k])))
            Xd = dn(X[k])
            P[k] = T(Xd @ dn(Eh[k]))
            Q[k] = T(Xd @ dn(Fh[k]))
        s = dn(Dh[0]).shape[0]
        Dn, En, Fn = [], [], []
        for i in range(1, m, 2):
            acc = dn(Dh[i]) - dn(Eh[i]) @ dn(Q[i - 1])
            if i + 1 < m:
                acc = acc - dn(Fh[i]) @ dn(P[i + 1])
            Dn.append(T(acc))
            En.append(T(-dn(Eh[i]) @ dn(P[i - 1])))
            Fn.append(T(-dn(Fh[i]) @ dn(Q[i + 1])) if i + 1 < m else T(np.zeros((s, s))))
        fac.levels.append((X, Eh, Fh))
        Dh, Eh, Fh = Dn, En, Fn
    if len(Dh) == 1:
        fac.Xlast = T(np.linalg.inv(dn(Dh[0])))
    else:
        m, s = len(Dh), dn(Dh[0]).shape[0]
        A = np.zeros((m * s, m * s))
        for i in range(m):
            A[i * s:(i + 1) * s, i * s:(i + 1) * s] = dn(Dh[i])
            if i > 0:
                A[i * s:(i + 1) * s, (i - 1) * s:i * s] = dn(Eh[i])
            if i + 1 < m:
                A[i * s:(i + 1) * s, (i + 1) * s:(i + 2) * s] = dn(Fh[i])
        fac.Xdense = np.linalg.inv(A)
    return fac


def factor(st, leaf: int, eps: float, stop_blocks: int = 1) -> Factor:
    D, E, F = blocks(st)
    return factor_blocks(D, E, F, leaf, eps, stop_blocks)


def solve_blocks(fac: Factor, f_blocks):
    mv = hodlr.matvec
    fs = [list(f_blocks)]
    for X, E, F in fac.levels:
        f = fs[-1]
        m = len(f)
        g = {k: mv(X[k], f[k]) for k in range(0, m, 2)}
        fn = []
        for i in range(1, m, 2):
            v = f[i] - mv(E[i], g[i - 1])
            if i + 1 < m:
                v = v - mv(F[i], g[i + 1])
            fn.append(v)
        fs.append(fn)
    if fac.Xdense is not None:   # early stop: the remaining system at once
        fl = fs[-1]
        s = fl[0].shape[0]
        ud = fac.Xdense @ np.concatenate(fl, axis=0)
        u = [ud[i * s:(i + 1) * s] for i in range(len(fl))]
    else:
        u = [mv(fac.Xlast, fs[-1][0])]
    for lev in range(len(fac.levels) - 1, -1, -1):
        X, E, F = fac.levels[lev]
        f = fs[lev]
        m = len(f)
        un = [None] * m
        for j, v in enumerate(u):
            un[2 * j + 1] = v
        for k in range(0, m, 2):
            r = f[k].copy()
            if k - 1 >= 0:
                r = r - mv(E[k], un[k - 1])
            if k + 1 < m:
                r = r - mv(F[k], un[k + 1])
            un[k] = mv(X[k], r)
        u = un
    return u


def solve(fac: Factor, st, b: np.ndarray) -> np.ndarray:
    s = st.nx
    b2 = b.reshape(st.n, -1)
    f = [b2[i * s:(i + 1) * s] for i in range(st.ny)]
    u = solve_blocks(fac, f)
    return np.concatenate(u, axis=0).reshape(b.shape)


def level_ranks(fac: Factor):
    """Per level: max off-diagonal rank of the stored X, E, F blocks."""
    out = []
    for X, E, F in fac.levels:
        r = 0
        for H in list(X.values()) + list(E) + list(F):
            for d, rs in hodlr.ranks(H).items():
                r = max(r, max(rs))
        out.append(r)
    return out


def stored_entries(fac: Factor) -> int:
    tot = 0
    for X, E, F in fac.levels:
        for H in list(X.values()) + list(E) + list(F):
            tot += hodlr.stored_entries(H)
    last = fac.Xdense.size if fac.Xdense is not None else hodlr.stored_entries(fac.Xlast)
    return tot + last

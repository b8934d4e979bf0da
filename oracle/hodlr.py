"""HODLR matrices: the paper's H-matrix format with weak admissibility.

Section 3: every dense block is approximated by a Hackbusch H-matrix with weak
admissibility, i.e. a HODLR matrix.  A square block of size s is split into
two index clusters of sizes floor(s/2) and s - floor(s/2) while s > leaf; the
two diagonal sub-blocks recurse, the two off-diagonal sub-blocks are stored
as low-rank products U V^T; blocks of size <= leaf are stored dense.

The truncation rule T_eps (the paper only says that the rank is tuned to a
specified accuracy; this is the reading used throughout): for an off-diagonal
block B with singular values s_1 >= s_2 >= ..., keep exactly the terms with
s_t > eps * s_1 (strictly greater; a zero block gets rank 0), storing
U = U_t diag(s_t) and V = V_t.  The 2-norm truncation error is then s_{t+1}
<= eps * s_1.  Leaves are stored exactly.  Test infrastructure only.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Leaf:
    M: np.ndarray

    @property
    def size(self):
        return self.M.shape[0]


@dataclass
class Node:
    n1: int
    A11: object
    A22: object
    U12: np.ndarray
    V12: np.ndarray
    U21: np.ndarray
    V21: np.ndarray

    @property
    def size(self):
        return self.n1 + self.A22.size


def truncate(B: np.ndarray, eps: float):
    """T_eps of one off-diagonal block via a full SVD; returns (U, V)."""
    p, q = B.shape
    if p == 0 or q == 0:
        return np.zeros((p, 0)), np.zeros((q, 0))
    W, sig, Zt = np.linalg.svd(B, full_matrices=False)
    if sig.size == 0 or sig[0] == 0.0:
        return np.zeros((p, 0)), np.zeros((q, 0))
    t = int(np.count_nonzero(sig > eps * sig[0]))
    return W[:, :t] * sig[:t], Zt[:t, :].T.copy()


def compress(M: np.ndarray, leaf: int, eps: float):
    """HODLR approximation of a dense square matrix (all off-diagonal blocks T_eps)."""
    s = M.shape[0]
    if s <= leaf:
        return Leaf(M.copy())
    n1 = s // 2
    U12, V12 = truncate(M[:n1, n1:], eps)
    U21, V21 = truncate(M[n1:, :n1], eps)
    return Node(n1, compress(M[:n1, :n1], leaf, eps), compress(M[n1:, n1:], leaf, eps),
                U12, V12, U21, V21)


def densify(H) -> np.ndarray:
    if isinstance(H, Leaf):
        return H.M.copy()
    n1, s = H.n1, H.size
    M = np.zeros((s, s))
    M[:n1, :n1] = densify(H.A11)
    M[n1:, n1:] = densify(H.A22)
    M[:n1, n1:] = H.U12 @ H.V12.T
    M[n1:, :n1] = H.U21 @ H.V21.T
    return M


def matvec(H, x: np.ndarray) -> np.ndarray:
    """y = H x without densifying (x: (s,) or (s, nrhs))."""
    if isinstance(H, Leaf):
        return H.M @ x
    n1 = H.n1
    x1, x2 = x[:n1], x[n1:]
    y1 = matvec(H.A11, x1) + H.U12 @ (H.V12.T @ x2)
    y2 = matvec(H.A22, x2) + H.U21 @ (H.V21.T @ x1)
    return np.concatenate([y1, y2], axis=0)


def depth(H) -> int:
    return 0 if isinstance(H, Leaf) else 1 + max(depth(H.A11), depth(H.A22))


def ranks(H, d: int = 1, out=None):
    """Ranks of the off-diagonal blocks, grouped by depth (top split = depth 1).

    Returns a dict depth -> list of ranks in cluster order (upper-right block
    of a split first, then its lower-left block).
    """
    out = {} if out is None else out
    if isinstance(H, Leaf):
        return out
    out.setdefault(d, []).extend([H.U12.shape[1], H.U21.shape[1]])
    ranks(H.A11, d + 1, out)
    ranks(H.A22, d + 1, out)
    return out


def stored_entries(H) -> int:
    """Number of stored floating-point values (leaves + U/V factors)."""
    if isinstance(H, Leaf):
        return H.M.size
    return (stored_entries(H.A11) + stored_entries(H.A22)
            + H.U12.size + H.V12.size + H.U21.size + H.V21.size)


def cluster_sizes(s: int, leaf: int):
    """Leaf cluster sizes in order for the split rule above."""
    if s <= leaf:
        return [s]
    n1 = s // 2
    return cluster_sizes(n1, leaf) + cluster_sizes(s - n1, leaf)

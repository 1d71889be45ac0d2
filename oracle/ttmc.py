"""Tensor-times-block contractions over the stored entries (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Definitions (section "Multilinear tensor-matrix multiplication", mode-i and multilinear products; section "Block-Krylov methods" block
steps; section "Block-Krylov methods for (1,2)-symmetric tensors" for the (1,2)-symmetric case).  With the transposed
notation A.(X, Y)_{1,2} = (X^T, Y^T)_{1,2} . A:

  FREE3   T3 = A.(X, Y)_{1,2} in R^{px x py x n}
          T3(a, b, k) = sum_{i,j} A(i,j,k) X(i,a) Y(j,b)
  FREE1   T1 = A.(Y, Z)_{2,3} in R^{m x py x pz}
          T1(i, b, c) = sum_{j,k} A(i,j,k) Y(j,b) Z(k,c)
  MODE3   t  = A.(Z)_3 restricted to the stored (i <= j) pair pattern
          t(i, j, c) = sum_k A(i,j,k) Z(k,c)

Each is evaluated as a plain sum over the stored entries (i <= j, k, a) and
their mirrors (j, i, k, a) for i != j.

Unfolding convention (the paper leaves the column order of unfold_i and
triunfold_3 open, section "Multilinear rank" and section "Block-Krylov methods for (1,2)-symmetric tensors"): Matlab column-major, first
remaining index fastest.
  FREE3 (X != Y):  row k, column a + px*b            (n x px*py)
  FREE3 sym-half:  row k, column b*(b+1)/2 + a, a<=b (n x p(p+1)/2),
                   the mode-3 unfolding of the upper triangular part
                   (triunfold_3)
  FREE1:           row i, column b + py*c            (m x py*pz)
  MODE3:           row = pair index in (i, j)-sorted order (P x pz)
"""
from __future__ import annotations

import numpy as np

from .sptensor import SymTensor

_CHUNK_ELEMS = 4_000_000


def _full_entries(T: SymTensor):
    """Both orientations of every stored entry: (row, col, k, a)."""
    off = T.i != T.j
    row = np.concatenate([T.i, T.j[off]])
    col = np.concatenate([T.j, T.i[off]])
    k = np.concatenate([T.k, T.k[off]])
    a = np.concatenate([T.a, T.a[off]])
    return row, col, k, a


def _scatter_rows(out: np.ndarray, rows: np.ndarray, contrib: np.ndarray) -> None:
    """out[rows[e], c] += contrib[e, c] for every e (plain accumulation)."""
    nrows = out.shape[0]
    for c in range(contrib.shape[1]):
        out[:, c] += np.bincount(rows, weights=contrib[:, c], minlength=nrows)


def sym_half_index(p: int):
    """(a, b) pairs with a <= b in triunfold_3 column order."""
    return [(a, b) for b in range(p) for a in range(b + 1)]


def free3(T: SymTensor, X: np.ndarray, Y: np.ndarray | None = None,
          sym_half: bool = False) -> np.ndarray:
    """T3 = A.(X, Y)_{1,2} unfolded in mode 3 (rows k).  With ``sym_half`` (only
    for Y = X) returns triunfold_3: the columns a <= b.

    Slice by slice: T3(:, :, k) = X_R^T diag(a) Y_C over the full entries
    (R, C, k, a) of slice k, with a library matrix product as the step."""
    X = np.asarray(X, dtype=np.float64)
    same = Y is None
    Y = X if same else np.asarray(Y, dtype=np.float64)
    if sym_half and not same:
        raise ValueError("sym_half requires Y = X")
    px, py = X.shape[1], Y.shape[1]
    row, col, k, a = _full_entries(T)
    order = np.argsort(k, kind="stable")
    row, col, k, a = row[order], col[order], k[order], a[order]
    bounds = np.searchsorted(k, np.arange(T.n + 1))
    out = np.zeros((T.n, px * py))
    for kk in range(T.n):
        e = slice(bounds[kk], bounds[kk + 1])
        if bounds[kk] == bounds[kk + 1]:
            continue
        M = (a[e, None] * X[row[e]]).T @ Y[col[e]]  # px x py
        out[kk] = M.reshape(-1, order="F")  # column alpha + px*beta
    if not sym_half:
        return out
    cols = [a_ + px * b_ for (a_, b_) in sym_half_index(px)]
    return out[:, cols]


def free1(T: SymTensor, Y: np.ndarray, Z: np.ndarray) -> np.ndarray:
    """T1 = A.(Y, Z)_{2,3} unfolded in mode 1 (rows i), column b + py*c."""
    Y = np.asarray(Y, dtype=np.float64)
    Z = np.asarray(Z, dtype=np.float64)
    py, pz = Y.shape[1], Z.shape[1]
    row, col, k, a = _full_entries(T)
    out = np.zeros((T.m, py * pz))
    step = max(1, _CHUNK_ELEMS // max(1, py * pz))
    for s in range(0, a.shape[0], step):
        e = slice(s, s + step)
        c = a[e, None, None] * Y[col[e], :, None] * Z[k[e], None, :]
        c = c.transpose(0, 2, 1).reshape(-1, py * pz)
        _scatter_rows(out, row[e], c)
    return out


def free1_rows(T: SymTensor, Y: np.ndarray, Z: np.ndarray, rows) -> np.ndarray:
    """The rows `rows` of T1 = A.(Y, Z)_{2,3}, one at a time: row i is the
    sum over the full entries (i, j, k, a) of a Y(j,:) (x) Z(k,:), formed as
    the product Y_J^T diag(a) Z_K (a library matrix product as the step),
    column b + py*c.  For sampled rows of a large tensor."""
    Y = np.asarray(Y, dtype=np.float64)
    Z = np.asarray(Z, dtype=np.float64)
    py, pz = Y.shape[1], Z.shape[1]
    out = np.zeros((len(rows), py * pz))
    for q, r in enumerate(rows):
        as_i = T.i == r
        as_j = (T.j == r) & (T.i != r)   # the mirror (j, i, k) of an off-diagonal entry
        col = np.concatenate([T.j[as_i], T.i[as_j]])
        k = np.concatenate([T.k[as_i], T.k[as_j]])
        a = np.concatenate([T.a[as_i], T.a[as_j]])
        M = (a[:, None] * Y[col]).T @ Z[k]          # py x pz, M(b, c)
        out[q] = M.reshape(-1, order="F")           # column b + py*c
    return out


def pairs(T: SymTensor):
    """Distinct stored (i <= j) pairs in (i, j)-sorted order, and the pair
    index of every stored entry."""
    key = T.i * T.m + T.j
    uk, inv = np.unique(key, return_inverse=True)
    return uk // T.m, uk % T.m, inv


def mode3(T: SymTensor, Z: np.ndarray):
    """t = A.(Z)_3 on the stored pair pattern; returns (pi, pj, t) with t of
    shape P x pz."""
    Z = np.asarray(Z, dtype=np.float64)
    pi, pj, inv = pairs(T)
    out = np.zeros((pi.shape[0], Z.shape[1]))
    _scatter_rows(out, inv, T.a[:, None] * Z[T.k])
    return pi, pj, out


def triu_to_full(T3h: np.ndarray, p: int) -> np.ndarray:
    """Expand a sym-half mode-3 unfolding (n x p(p+1)/2) to the full one
    (n x p*p, column a + p*b) using the 1-2 symmetry of A.(X, X)_{1,2}."""
    n = T3h.shape[0]
    full = np.zeros((n, p * p))
    for c, (a, b) in enumerate(sym_half_index(p)):
        full[:, a + p * b] = T3h[:, c]
        full[:, b + p * a] = T3h[:, c]
    return full

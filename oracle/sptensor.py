"""Stored-entry representation of a (1,2)-symmetric tensor (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

A (1,2)-symmetric A in R^{m x m x n} satisfies A(i,j,k) = A(j,i,k)
(Definition in section "Notation").  The oracle keeps the distinct positions
(i <= j, k) and their values in FP64; the entry at (j, i, k) is implied.
"""
from __future__ import annotations

import dataclasses
import numpy as np


@dataclasses.dataclass
class SymTensor:
    m: int
    n: int
    i: np.ndarray  # int64, i <= j
    j: np.ndarray
    k: np.ndarray
    a: np.ndarray  # float64

    @property
    def nnz(self) -> int:
        return int(self.a.shape[0])


def from_coo(m: int, n: int, i, j, k, val, sum_duplicates: bool = True) -> SymTensor:
    """Canonicalise (i, j) -> (min, max) and merge repeated positions.

    A position given as both (i, j, k) and (j, i, k) names the same entry of a
    symmetric tensor; with ``sum_duplicates`` the values are added, otherwise a
    repeat is an error."""
    i = np.asarray(i, dtype=np.int64)
    j = np.asarray(j, dtype=np.int64)
    k = np.asarray(k, dtype=np.int64)
    a = np.asarray(val, dtype=np.float64)
    if i.size and (i.min() < 0 or j.min() < 0 or k.min() < 0 or i.max() >= m
                   or j.max() >= m or k.max() >= n):
        raise IndexError("index out of range")
    if not np.all(np.isfinite(a)):
        raise ValueError("non-finite value")
    lo = np.minimum(i, j)
    hi = np.maximum(i, j)
    key = (k * m + lo) * m + hi
    uk, inv = np.unique(key, return_inverse=True)
    if uk.shape[0] != key.shape[0] and not sum_duplicates:
        raise ValueError("repeated position")
    s = np.zeros(uk.shape[0])
    np.add.at(s, inv, a)
    jj = uk % m
    t = uk // m
    return SymTensor(m, n, t % m, jj, t // m, s)


def dense(T: SymTensor) -> np.ndarray:
    """The full m x m x n array (small tensors only)."""
    A = np.zeros((T.m, T.m, T.n))
    A[T.i, T.j, T.k] = T.a
    A[T.j, T.i, T.k] = T.a
    return A


def from_dense(A: np.ndarray) -> SymTensor:
    """Stored entries of a dense (1,2)-symmetric array (zeros dropped)."""
    m, m2, n = A.shape
    assert m == m2
    if not np.allclose(A, A.transpose(1, 0, 2), rtol=0, atol=0):
        raise ValueError("not (1,2)-symmetric")
    iu, ju = np.triu_indices(m)
    i = np.repeat(iu, n)
    j = np.repeat(ju, n)
    k = np.tile(np.arange(n), iu.shape[0])
    a = A[i, j, k]
    keep = a != 0
    return SymTensor(m, n, i[keep], j[keep], k[keep], a[keep])


def frob2(T: SymTensor) -> float:
    """||A||^2 over the full tensor: off-diagonal stored entries count twice
    (inner product and norm, section "Inner product and norm, contractions")."""
    w = np.where(T.i == T.j, 1.0, 2.0)
    return float(np.sum(w * T.a * T.a))

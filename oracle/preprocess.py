"""Slice scalings of a (1,2)-symmetric tensor (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section "Experiments": Example 3 normalises every mode-3 slice of a graph
tensor so that its largest eigenvalue equals 1; Example 4 instead scales
every slice to Frobenius norm 1.  A slice A(:,:,k) is the full symmetric
matrix (a stored off-diagonal entry stands for both orientations).  For a
nonnegative (adjacency) slice the largest eigenvalue is its spectral radius
(Perron-Frobenius); for a general slice the reading taken is the spectral
radius, max |lambda|.  A zero slice stays zero.
"""
from __future__ import annotations

import numpy as np

from .sptensor import SymTensor


def slice_matrix(T: SymTensor, k: int):
    """Dense slice k on its touched rows: (rows, matrix)."""
    sel = T.k == k
    i, j, a = T.i[sel], T.j[sel], T.a[sel]
    rows = np.unique(np.concatenate([i, j]))
    li, lj = np.searchsorted(rows, i), np.searchsorted(rows, j)
    M = np.zeros((rows.size, rows.size))
    M[li, lj] = a
    M[lj, li] = a
    return rows, M


def scale_slices(T: SymTensor, how: str) -> SymTensor:
    """how: "frobenius" or "lambda_max"; returns the scaled tensor."""
    a = T.a.copy()
    for k in np.unique(T.k):
        _, M = slice_matrix(T, k)
        if how == "frobenius":
            f = np.linalg.norm(M)
        elif how == "lambda_max":
            f = np.abs(np.linalg.eigvalsh(M)).max()
        else:
            raise ValueError(how)
        if f > 0:
            a[T.k == k] /= f
    return SymTensor(T.m, T.n, T.i, T.j, T.k, a)

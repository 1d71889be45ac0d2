"""Block orthogonalisation with deflation (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Algorithm 3 steps (ii)-(iv) project a new block onto the complement of the
current ON-basis and orthonormalise its mode-1 fibres (a thin QR); Appendix B
keeps the block in matrix form and orthogonalises it directly.  Here that is
done column by column, in column order, with classical Gram-Schmidt against
every previous column (the existing basis and the new columns kept so far),
applied twice (reorthogonalisation).

Deflation (the paper only caps the basis at the mode size, section "BK method";
this rule is a reading): column b is dropped when the norm left after
orthogonalisation is at most ``tau`` times ||b||, or when the basis already
spans the whole space.  The barred block U(:, 1:p) means the first p kept
columns.  ``tau`` must sit just above the noise level of the product
(1e-14 for FP64-accurate products): near convergence the new gradient
direction is only about ||grad|| / ||F|| of the product's norm, and it lies
below the block's other residual directions, so any coarser rule (or one
relative to the block instead of the column) throws the gradient away.
"""
from __future__ import annotations

import numpy as np

TAU_F64 = 1e-14


def orthonormalize(B: np.ndarray) -> np.ndarray:
    """Orthonormal basis of the column span of a full-rank B (thin QR)."""
    Q, R = np.linalg.qr(np.asarray(B, dtype=np.float64))
    return Q


def orth_append(Q: np.ndarray, B: np.ndarray, dim: int, tau: float = TAU_F64):
    """Orthonormalise the columns of B against the basis Q (m x k, may have 0
    columns) and against each other, in order, dropping dependent columns.

    Returns (Qnew, kept): Qnew has the kept columns (m x q'), ``kept`` their
    indices in B."""
    m = B.shape[0]
    basis = Q if Q is not None else np.zeros((m, 0))
    new = []
    kept = []
    for c in range(B.shape[1]):
        if basis.shape[1] >= dim:
            break
        b = np.array(B[:, c], dtype=np.float64)
        before = np.sqrt(b @ b)
        if before == 0.0:
            continue
        v = b
        for _ in range(2):
            v = v - basis @ (basis.T @ v)
        after = np.sqrt(v @ v)
        if after <= tau * before:
            continue
        q = v / after
        new.append(q)
        kept.append(c)
        basis = np.concatenate([basis, q[:, None]], axis=1)
    Qnew = np.stack(new, axis=1) if new else np.zeros((m, 0))
    return Qnew, kept

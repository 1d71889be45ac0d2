"""Symmetric HOOI for a sparse (1,2)-symmetric tensor (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

section "Higher Order Orthogonal Iteration": HOOI alternates maximisations.  For a (1,2)-symmetric tensor
each iteration updates U as the r leading left singular vectors of
C1 = A.(U, W)_{2,3} (mode-1 unfolding, using the previous U), then W as the
r3 leading left singular vectors of C3 = A.(U, U)_{1,2} with the new U.  The
start is random with orthonormal columns; the G-gradient (global
coordinates, section "Gradient on the product manifold") is evaluated every ten iterations:

  Gamma1 = <A.(U, W)_{2,3}, F>_{-1} = T1 F_(1)^T,   grad_U = (I - U U^T) Gamma1
  Gamma3 = T3 F_(3)^T,                              grad_W = (I - W W^T) Gamma3
  ||grad||^2 = 2 ||grad_U||^2 + ||grad_W||^2   (modes 1 and 2 coincide)
"""
from __future__ import annotations

import time

import numpy as np

from . import core, ttmc
from .orth import orthonormalize
from .sptensor import SymTensor, frob2


def left_singular(M: np.ndarray, r: int) -> np.ndarray:
    U, s, Vt = np.linalg.svd(M, full_matrices=False)
    return U[:, :r]


def global_gradient(T: SymTensor, U: np.ndarray, W: np.ndarray):
    r, r3 = U.shape[1], W.shape[1]
    T1 = ttmc.free1(T, U, W)
    F1 = U.T @ T1
    F = F1.reshape(r, r, r3, order="F")
    T3f = ttmc.triu_to_full(ttmc.free3(T, U, sym_half=True), r)
    F3 = core.unfold3(F)
    G1 = T1 @ F1.T
    G1 = G1 - U @ (U.T @ G1)
    G3 = T3f @ F3.T
    G3 = G3 - W @ (W.T @ G3)
    nf = np.sqrt(np.sum(F * F))
    g = np.sqrt(2.0 * np.sum(G1 * G1) + np.sum(G3 * G3))
    return g / nf if nf > 0 else np.inf, F


def hooi_solve(T: SymTensor, r: int, r3: int, U_init: np.ndarray, W_init: np.ndarray,
               tol: float = 1e-13, max_iter: int = 2000, grad_every: int = 10):
    t0 = time.perf_counter()
    U = orthonormalize(U_init)
    W = orthonormalize(W_init)
    hist = []
    it = 0
    rel, F = global_gradient(T, U, W)
    while True:
        T1 = ttmc.free1(T, U, W)
        U = left_singular(T1, r)
        T3f = ttmc.triu_to_full(ttmc.free3(T, U, sym_half=True), r)
        W = left_singular(T3f, r3)
        it += 1
        if it % grad_every == 0 or it >= max_iter:
            rel, F = global_gradient(T, U, W)
            hist.append((it, rel))
            if rel <= tol or it >= max_iter:
                break
    return {"U": U, "W": W, "F": F, "rel_hist": hist, "iters": it,
            "converged": rel <= tol, "normA": np.sqrt(frob2(T)),
            "seconds": time.perf_counter() - t0}

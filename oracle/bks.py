"""Tensor Krylov-Schur (BKS) for a sparse (1,2)-symmetric tensor (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Algorithm 5 (tensor Krylov-Schur) with U = V (section "A Tensor Krylov-Schur like method", symmetric case):

  start  (U0, W0) orthonormal (the paper does not state the BKS start; here it
         is the same seeded random start HOOI uses, section "Higher Order Orthogonal Iteration")
  expand stages 1..s of a BK method to X = [U0 U1 ...], Z = [W0 W1 ...]
  loop
    (i)   best rank-(r, r, r3) approximation of C = A.(X, X, Z) (eq. tkd,
          eq. maxrC) by HOSVD + 5 HOOI + Newton-Grassmann (section "Experiments")
    (ii)  U0 = X P, W0 = Z S (eq. tks1)
    (iii) one BK step from (U0, W0): T1 = A.(U0, W0)_{2,3} and
          T3 = A.(U0, U0)_{1,2}, orthogonalised against U0, W0 -> U1, W1
    (iv)  G-gradient at (U0, W0) from that step (Proposition 3.2, Lemma 3.1):
          ||grad||^2 = 2 ||<H0, H1^1>_{-1}||^2 + ||<H0, H1^3>_{-3}||^2,
          modes 1 and 2 equal because U = V; stop at ||grad|| / ||F|| <= tol
          (section "Experiments")
    (v)   expand stages 2..s from ([U0 U1], [W0 W1])

With H0 = F = U0^T T1 (as r x r x r3) and H1^1 = U1^T (I - U0 U0^T) T1 = R1,
<H0, H1^1>_{-1} is R1 F_(1)^T; in mode 3, R3 = W1^T (I - W0 W0^T) T3 on the
full (not sym-half) unfolding and <H0, H1^3>_{-3} = R3 F_(3)^T.

S-values (section "Conditioning of the best approximation problem"): s_i^(k) = sqrt(lambda_i(<F, F>_{-k})) and
s_{r_k+1}^(k) = sqrt(lambda_max(<F_perp^k, F_perp^k>_{-k})), which by
Lemma 3.1 equals the largest singular value of R1 (resp. R3).
"""
from __future__ import annotations

import time

import numpy as np

from . import bk, core, ttmc
from .orth import orth_append, orthonormalize
from .sptensor import SymTensor, frob2


def core_tensor(T: SymTensor, X: np.ndarray, Z: np.ndarray) -> np.ndarray:
    """C = A.(X, X, Z) (eq. tkd) as Z^T . A.(X, X)_{1,2}, shape (k1, k1, k3)."""
    k1 = X.shape[1]
    T3h = ttmc.free3(T, X, sym_half=True)
    T3f = ttmc.triu_to_full(T3h, k1)          # n x k1*k1, column a + k1*b
    C3 = Z.T @ T3f                              # k3 x k1*k1
    return C3.reshape(Z.shape[1], k1, k1, order="F").transpose(1, 2, 0)


def bk_step(T: SymTensor, U0: np.ndarray, W0: np.ndarray, tau: float = 1e-14):
    """Step (iii) and (iv): one BK step from (U0, W0), F, the gradient and the
    S-values."""
    r, r3 = U0.shape[1], W0.shape[1]
    T1 = ttmc.free1(T, U0, W0)                        # m x r*r3
    T3h = ttmc.free3(T, U0, sym_half=True)            # n x r(r+1)/2
    T3f = ttmc.triu_to_full(T3h, r)                   # n x r*r
    U1, _ = orth_append(U0, T1, T.m, tau)
    W1, _ = orth_append(W0, T3h, T.n, tau)
    F1 = U0.T @ T1                                    # F_(1): r x r*r3
    F = F1.reshape(r, r, r3, order="F")
    F3 = core.unfold3(F)                              # r3 x r*r
    R1 = U1.T @ (T1 - U0 @ F1)
    R3 = W1.T @ (T3f - W0 @ (W0.T @ T3f))
    g1 = R1 @ F1.T
    g3 = R3 @ F3.T
    nf = np.sqrt(np.sum(F * F))
    grad = np.sqrt(2.0 * np.sum(g1 * g1) + np.sum(g3 * g3))
    s1 = np.sqrt(np.maximum(np.linalg.eigvalsh(F1 @ F1.T)[::-1], 0.0))
    s3 = np.sqrt(np.maximum(np.linalg.eigvalsh(F3 @ F3.T)[::-1], 0.0))
    s1n = np.linalg.norm(R1, 2) if R1.size else 0.0
    s3n = np.linalg.norm(R3, 2) if R3.size else 0.0
    return {
        "U1": U1, "W1": W1, "F": F, "T1": T1, "T3f": T3f,
        "grad": grad, "normF": nf, "rel": grad / nf if nf > 0 else np.inf,
        "svals1": np.concatenate([s1, [s1n]]), "svals3": np.concatenate([s3, [s3n]]),
        "R1": R1, "R3": R3,
    }


def bks_solve(T: SymTensor, r: int, r3: int, U_init: np.ndarray, W_init: np.ndarray,
              p: int = 4, s: int = 2, variant: str = "bk", tol: float = 1e-13,
              max_outer: int = 200, tau: float = 1e-14,
              inner_tol: float | None = None,
              hooi_iters: int = 5, ng_max: int = 50):
    """Algorithm 5.  Returns a dict with U, W, F, the per-iteration relative
    gradients and ||F||, k1/k3 and the S-values at the returned point."""
    if inner_tol is None:
        inner_tol = tol
    t0 = time.perf_counter()
    U0 = orthonormalize(U_init)
    W0 = orthonormalize(W_init)
    pbar = None if variant == "max" else p
    basis = bk.Basis(U0, W0)
    for stage in range(1, s + 1):
        bk.run_stage(T, basis, variant, stage, pbar, tau)
    hist, normF, k1s, k3s, inner = [], [], [], [], []
    step = None
    it = 0
    while True:
        X, Z = basis.X, basis.Z
        k1s.append(X.shape[1])
        k3s.append(Z.shape[1])
        C = core_tensor(T, X, Z)
        P, S, info = core.inner_solve(C, r, r3, inner_tol, hooi_iters, ng_max)
        # eq. Fnon-decr needs the inner solve to end no lower than the current
        # point E0 (the leading coordinates of X, Z); a HOSVD start can reach
        # a lower local maximum, so then solve again from E0 (a reading)
        E1 = np.eye(C.shape[0], r)
        E3 = np.eye(C.shape[2], r3)
        if core.objective(C, P, S) < core.objective(C, E1, E3) * (1.0 - 1e-14):
            P, S, _, _, _ = core.newton_grassmann(C, E1, E3, inner_tol, ng_max)
        inner.append(info)
        U0 = orthonormalize(X @ P)
        W0 = orthonormalize(Z @ S)
        step = bk_step(T, U0, W0, tau)
        hist.append(step["rel"])
        normF.append(step["normF"])
        it += 1
        if step["rel"] <= tol or it >= max_outer:
            break
        basis = bk.Basis(U0, W0)
        basis.ub.append(step["U1"])
        basis.wb.append(step["W1"])
        basis.used_u.add((0, 0))
        basis.used_w.add((0, 0))
        for stage in range(2, s + 1):
            bk.run_stage(T, basis, variant, stage, pbar, tau)
    return {
        "U": U0, "W": W0, "F": step["F"], "rel_hist": hist, "normF_hist": normF,
        "converged": step["rel"] <= tol, "outer_iters": it, "k1": k1s, "k3": k3s,
        "svals1": step["svals1"], "svals3": step["svals3"], "normA": np.sqrt(frob2(T)),
        "inner": inner, "seconds": time.perf_counter() - t0,
    }


def subspace_distance(U_ref: np.ndarray, U: np.ndarray) -> float:
    """sin of the largest principal angle between span(U_ref) and span(U),
    ||(I - U_ref U_ref^T) U||_2, for orthonormal U_ref and U."""
    D = U - U_ref @ (U_ref.T @ U)
    return float(np.linalg.norm(D, 2))

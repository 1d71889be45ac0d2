"""Tensor Krylov-Schur for a general (non-symmetric) sparse 3-tensor
(oracle, FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Algorithm 5 as stated for a non-symmetric A in R^{l x m x n} (section "A
Tensor Krylov-Schur like method"): three bases X, Y, Z, built by the mode-1,
mode-2 and mode-3 block-Krylov steps of Algorithm 3 (section "Block-Krylov
methods"); the core C = A.(X, Y, Z) (eq. tkd); its best rank-(r1, r2, r3)
approximation (eq. maxrC); the restart U0 = X U^, V0 = Y V^, W0 = Z W^ (eq.
tks1); one block-Krylov step in each mode from (U0, V0, W0), and the
G-gradient of Proposition 3.2:

  ||grad||^2 = ||<H0, H1^1>_{-1}||^2 + ||<H0, H1^2>_{-2}||^2 + ||<H0, H1^3>_{-3}||^2

with H0 = A.(U0, V0, W0) and H1^1 = A.(U1, V0, W0), etc.

Readings (the paper gives the BK schedules for the (1,2)-symmetric case
only, and cites the inner solver):
- schedule: the min-BK rule in every mode -- stage t computes
  U_t = A.(Vbar_{t-1}, Wbar_{t-1})_{2,3}, V_t = A.(Ubar_{t-1}, Wbar_{t-1})_{1,3},
  W_t = A.(Ubar_{t-1}, Vbar_{t-1})_{1,2}; a bar is the first p columns, except
  that U0, V0, W0 are used whole (the paper's assumption that the blocks with
  subscript 1 come from U0, V0, W0);
- inner solve: truncated HOSVD, then HOOI iterations until the projected
  problem's relative gradient reaches the tolerance (the paper's alternative
  to Newton-Grassmann; both have the same fixed points).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .orth import orth_append, orthonormalize


@dataclasses.dataclass
class GenTensor:
    l: int
    m: int
    n: int
    i: np.ndarray
    j: np.ndarray
    k: np.ndarray
    a: np.ndarray

    @property
    def nnz(self):
        return int(self.a.shape[0])


def from_coo(l, m, n, i, j, k, val) -> GenTensor:
    """Distinct positions (repeated ones summed), FP64 values."""
    i, j, k = (np.asarray(x, dtype=np.int64) for x in (i, j, k))
    a = np.asarray(val, dtype=np.float64)
    if i.size and (i.min() < 0 or j.min() < 0 or k.min() < 0 or i.max() >= l or j.max() >= m
                   or k.max() >= n):
        raise IndexError("index out of range")
    key = (i * m + j) * n + k
    uk, inv = np.unique(key, return_inverse=True)
    s = np.zeros(uk.shape[0])
    np.add.at(s, inv, a)
    return GenTensor(l, m, n, uk // (m * n), (uk // n) % m, uk % n, s)


def dense(T: GenTensor):
    A = np.zeros((T.l, T.m, T.n))
    A[T.i, T.j, T.k] = T.a
    return A


def frob2(T: GenTensor) -> float:
    return float(np.sum(T.a * T.a))


def _scatter(rows, nrows, contrib):
    out = np.zeros((nrows, contrib.shape[1]))
    for c in range(contrib.shape[1]):
        out[:, c] = np.bincount(rows, weights=contrib[:, c], minlength=nrows)
    return out


def mode_product(T: GenTensor, mode: int, B1, B2):
    """The product with one free mode, unfolded in it (first remaining index
    fastest, as the mode unfoldings of section "Multilinear rank"):
      mode 1: A.(B1, B2)_{2,3}, row i, column b + p1 c   (B1 on mode 2, B2 on mode 3)
      mode 2: A.(B1, B2)_{1,3}, row j, column a + p1 c   (B1 on mode 1, B2 on mode 3)
      mode 3: A.(B1, B2)_{1,2}, row k, column a + p1 b   (B1 on mode 1, B2 on mode 2)"""
    B1 = np.asarray(B1, dtype=np.float64)
    B2 = np.asarray(B2, dtype=np.float64)
    idx = {1: (T.i, T.j, T.k, T.l), 2: (T.j, T.i, T.k, T.m), 3: (T.k, T.i, T.j, T.n)}
    row, c1, c2, nrows = idx[mode]
    contrib = T.a[:, None, None] * B1[c1][:, :, None] * B2[c2][:, None, :]
    return _scatter(row, nrows, contrib.transpose(0, 2, 1).reshape(T.nnz, -1))


def unfold(C, mode):
    """Mode-k unfolding of a dense 3-tensor, first remaining index fastest."""
    if mode == 1:
        return C.reshape(C.shape[0], -1, order="F")
    if mode == 2:
        return C.transpose(1, 0, 2).reshape(C.shape[1], -1, order="F")
    return C.transpose(2, 0, 1).reshape(C.shape[2], -1, order="F")


def mprod(C, P, Q, S):
    return np.einsum("abc,ai,bj,ck->ijk", C, P, Q, S, optimize=True)


def core_tensor(T: GenTensor, X, Y, Z):
    """C = A.(X, Y, Z) (eq. tkd) as Z^T A.(X, Y)_{1,2}."""
    T3 = mode_product(T, 3, X, Y)                   # n x k1 k2, column a + k1 b
    C3 = Z.T @ T3                                   # k3 x k1 k2
    return C3.reshape(Z.shape[1], X.shape[1], Y.shape[1], order="F").transpose(1, 2, 0)


def top_left(M, r):
    w, V = np.linalg.eigh(M @ M.T)
    return V[:, ::-1][:, :r]


def local_gradient(C, P, Q, S):
    """Relative G-gradient of ||C.(P, Q, S)||^2 at (P, Q, S): the three terms
    <F, F_perp^k>_{-k} with F_perp from the orthogonal complements."""
    F = mprod(C, P, Q, S)
    nf = np.sqrt(np.sum(F * F))
    g = 0.0
    for mode, (B, rest) in enumerate(((P, (Q, S)), (Q, (P, S)), (S, (P, Q))), start=1):
        M = unfold(mprod(C, *([np.eye(C.shape[0]) if mode == 1 else P,
                               np.eye(C.shape[1]) if mode == 2 else Q,
                               np.eye(C.shape[2]) if mode == 3 else S])), mode)
        Fk = unfold(F, mode)
        G = (M - B @ (B.T @ M)) @ Fk.T
        g += np.sum(G * G)
    return np.sqrt(g) / nf if nf > 0 else np.inf


def inner_solve(C, r1, r2, r3, tol, max_iter=5000):
    """Best rank-(r1, r2, r3) approximation of the dense core: truncated
    HOSVD, then HOOI until the relative gradient is <= tol."""
    P = top_left(unfold(C, 1), r1)
    Q = top_left(unfold(C, 2), r2)
    S = top_left(unfold(C, 3), r3)
    it = 0
    rel = local_gradient(C, P, Q, S)
    while rel > tol and it < max_iter:
        P = top_left(unfold(mprod(C, np.eye(C.shape[0]), Q, S), 1), r1)
        Q = top_left(unfold(mprod(C, P, np.eye(C.shape[1]), S), 2), r2)
        S = top_left(unfold(mprod(C, P, Q, np.eye(C.shape[2])), 3), r3)
        it += 1
        if it % 5 == 0 or it == max_iter:
            rel = local_gradient(C, P, Q, S)
    return P, Q, S, {"iters": it, "rel_grad": rel}


def _bar(B, p, first):
    return B if (first or p is None) else B[:, :p]


def expand(T: GenTensor, Ub, Vb, Wb, stages, p, tau, start_stage=1):
    """Stages start_stage..stages of the min-BK rule in every mode, appending
    to the block lists (orthogonalised against the whole basis, Algorithm 3
    steps (ii)-(iv))."""
    for t in range(start_stage, stages + 1):
        q = t - 1
        Vq, Wq, Uq = _bar(Vb[q], p, q == 0), _bar(Wb[q], p, q == 0), _bar(Ub[q], p, q == 0)
        new = []
        for mode, (B1, B2), blocks, rows in ((1, (Vq, Wq), Ub, T.l), (2, (Uq, Wq), Vb, T.m),
                                             (3, (Uq, Vq), Wb, T.n)):
            basis = np.concatenate(blocks, axis=1)
            if B1.shape[1] == 0 or B2.shape[1] == 0 or basis.shape[1] >= rows:
                new.append((blocks, np.zeros((rows, 0))))
                continue
            B = mode_product(T, mode, B1, B2)
            Q, _ = orth_append(basis, B, rows, tau)
            new.append((blocks, Q))
        for blocks, Q in new:
            blocks.append(Q)


def bk_step(T: GenTensor, U0, V0, W0, tau):
    """Step (iii)-(iv): one block-Krylov step in each mode from (U0, V0, W0)
    and the G-gradient of Proposition 3.2."""
    T1 = mode_product(T, 1, V0, W0)
    T2 = mode_product(T, 2, U0, W0)
    T3 = mode_product(T, 3, U0, V0)
    r1, r2, r3 = U0.shape[1], V0.shape[1], W0.shape[1]
    F = (U0.T @ T1).reshape(r1, r2, r3, order="F")     # H0 = A.(U0, V0, W0)
    out = {"F": F}
    g2 = 0.0
    for mode, (B0, Tk) in enumerate(((U0, T1), (V0, T2), (W0, T3)), start=1):
        rows = Tk.shape[0]
        B1, _ = orth_append(B0, Tk, rows, tau)
        H1 = B1.T @ (Tk - B0 @ (B0.T @ Tk))               # H1^k, unfolded in mode k
        G = H1 @ unfold(F, mode).T                        # <H0, H1^k>_{-k}
        g2 += np.sum(G * G)
        out[f"B1_{mode}"] = B1
        out[f"s{mode}"] = np.linalg.norm(H1, 2) if H1.size else 0.0
    nf = np.sqrt(np.sum(F * F))
    out["normF"] = nf
    out["rel"] = np.sqrt(g2) / nf if nf > 0 else np.inf
    return out


def bks_solve(T: GenTensor, r, U_init, V_init, W_init, p=4, s=2, tol=1e-13, max_outer=200,
              tau=1e-14, inner_tol=None):
    """Algorithm 5 for a general tensor; r = (r1, r2, r3)."""
    r1, r2, r3 = r
    inner_tol = tol if inner_tol is None else inner_tol
    U0, V0, W0 = (orthonormalize(x) for x in (U_init, V_init, W_init))
    Ub, Vb, Wb = [U0], [V0], [W0]
    expand(T, Ub, Vb, Wb, s, p, tau)
    hist, fh = [], []
    step = None
    it = 0
    while True:
        X, Y, Z = (np.concatenate(b, axis=1) for b in (Ub, Vb, Wb))
        C = core_tensor(T, X, Y, Z)
        P, Q, S, _ = inner_solve(C, r1, r2, r3, inner_tol)
        # keep the outer objective non-decreasing: solve again from the
        # current point's coordinates if the HOSVD start ended lower
        E = [np.eye(C.shape[d], rr) for d, rr in zip(range(3), (r1, r2, r3))]
        if np.sum(mprod(C, P, Q, S) ** 2) < np.sum(mprod(C, *E) ** 2) * (1 - 1e-14):
            P, Q, S = E
            rel = local_gradient(C, P, Q, S)
            k = 0
            while rel > inner_tol and k < 5000:
                P = top_left(unfold(mprod(C, np.eye(C.shape[0]), Q, S), 1), r1)
                Q = top_left(unfold(mprod(C, P, np.eye(C.shape[1]), S), 2), r2)
                S = top_left(unfold(mprod(C, P, Q, np.eye(C.shape[2])), 3), r3)
                k += 1
                if k % 5 == 0:
                    rel = local_gradient(C, P, Q, S)
        U0, V0, W0 = orthonormalize(X @ P), orthonormalize(Y @ Q), orthonormalize(Z @ S)
        step = bk_step(T, U0, V0, W0, tau)
        hist.append(step["rel"])
        fh.append(step["normF"])
        it += 1
        if step["rel"] <= tol or it >= max_outer:
            break
        Ub, Vb, Wb = [U0, step["B1_1"]], [V0, step["B1_2"]], [W0, step["B1_3"]]
        expand(T, Ub, Vb, Wb, s, p, tau, start_stage=2)
    return {"U": U0, "V": V0, "W": W0, "F": step["F"], "rel_hist": hist, "normF_hist": fh,
            "converged": step["rel"] <= tol, "outer_iters": it, "k": (X.shape[1], Y.shape[1], Z.shape[1]),
            "normA": np.sqrt(frob2(T))}

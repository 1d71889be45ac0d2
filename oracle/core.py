"""Best rank-(r, r, r3) approximation of a small dense (1,2)-symmetric core
(oracle, FP64): Algorithm 5 step (i).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The projected problem (eq. maxrC) maximises g(P, S) = ||C.(P, P, S)||^2 over
P^T P = I_r, S^T S = I_r3 (U = V for a (1,2)-symmetric tensor, section "A Tensor Krylov-Schur like method").
The paper's recipe (section "Experiments"): truncated HOSVD of C, then 5 HOOI
iterations, then Newton-Grassmann to the same relative-gradient tolerance.

The Newton-Grassmann method is only cited by the paper, so its equations are
derived here (a reading of the paper): at the current (P, S) rotate C into
the bases [P P_perp], [S S_perp] (Appendix A's local coordinates, where the
point is E0 = ([I;0], [I;0]) and the tangent space is spanned by [0; I]),
write the objective along the curve P(D) = [I; D] (I + D^T D)^{-1/2},
S(T) = [I; T] (I + T^T T)^{-1/2} and keep terms to second order:

  phi(D, T) = ||F||^2 + 4<Gamma1, D> + 2<Gamma3, T> + d^T A d + O(|d|^3)

with F = B000, Gamma1 = <B100, F>_{-1}, Gamma3 = <B001, F>_{-3} (the local
gradient blocks of section "Gradient on the product manifold") and

  d^T A d = ||G1||^2 + 2 <F, G2> - 2 tr(D S1 D^T) - tr(T S3 T^T)
  G1 = B100 . (D)_1 + B010 . (D)_2 + B001 . (T)_3
  G2 = B110 . (D, D)_{1,2} + B101 . (D, T)_{1,3} + B011 . (D, T)_{2,3}
  S1 = <F, F>_{-1},  S3 = <F, F>_{-3}

(block index 0 = first r (or r3) coordinates, 1 = the rest).  The Newton
step solves (-2A) d = (4 Gamma1, 2 Gamma3) and retracts by a thin QR.  When
-2A is not positive definite (not near a maximum) one HOOI iteration is taken
instead.
"""
from __future__ import annotations

import numpy as np


def unfold1(C):
    """Mode-1 unfolding, column b + k2*c (first remaining index fastest)."""
    k1, k2, k3 = C.shape
    return C.reshape(k1, k2 * k3, order="F")


def unfold3(C):
    """Mode-3 unfolding, column a + k1*b."""
    k1, k2, k3 = C.shape
    return C.transpose(2, 0, 1).reshape(k3, k1 * k2, order="F")


def mprod(C, P, Q, S):
    """C.(P, Q, S) = (P^T, Q^T, S^T) . C (multilinear product, section "Multilinear tensor-matrix multiplication")."""
    return np.einsum("abc,ai,bj,ck->ijk", C, P, Q, S, optimize=True)


def top_eigvecs(G, r):
    """Eigenvectors of the symmetric G for its r largest eigenvalues."""
    w, V = np.linalg.eigh(G)
    return V[:, ::-1][:, :r]


def hosvd(C, r, r3):
    """Truncated HOSVD start: leading left singular vectors of the mode-1 and
    mode-3 unfoldings (via their Gram matrices)."""
    C1 = unfold1(C)
    C3 = unfold3(C)
    return top_eigvecs(C1 @ C1.T, r), top_eigvecs(C3 @ C3.T, r3)


def hooi_step(C, P, S):
    """One symmetric HOOI iteration (section "Higher Order Orthogonal Iteration"): P from C.(P, S)_{2,3} with
    the previous P, then S from C.(P, P)_{1,2} with the new P."""
    r = P.shape[1]
    r3 = S.shape[1]
    M1 = np.einsum("abc,bj,ck->ajk", C, P, S, optimize=True).reshape(C.shape[0], r * r3, order="F")
    P = top_eigvecs(M1 @ M1.T, r)
    M3 = np.einsum("abc,ai,bj->cij", C, P, P, optimize=True).reshape(C.shape[2], r * r, order="F")
    S = top_eigvecs(M3 @ M3.T, r3)
    return P, S


def complement(P):
    """P_perp with [P P_perp] orthogonal."""
    k, r = P.shape
    # columns r.. of a complete QR of [P I] span the complement of span(P)
    Qf, _ = np.linalg.qr(np.concatenate([P, np.eye(k)], axis=1), mode="complete")
    return Qf[:, r:k]


def blocks(C, P, S):
    """Rotate C into [P P_perp], [S S_perp] and return the blocks used by the
    gradient and the Newton model."""
    r, r3 = P.shape[1], S.shape[1]
    Qp = np.concatenate([P, complement(P)], axis=1)
    Qs = np.concatenate([S, complement(S)], axis=1)
    B = mprod(C, Qp, Qp, Qs)
    return {
        "F": B[:r, :r, :r3],
        "B100": B[r:, :r, :r3],
        "B001": B[:r, :r, r3:],
        "B110": B[r:, r:, :r3],
        "B101": B[r:, :r, r3:],
        "Qp": Qp,
        "Qs": Qs,
    }


def local_gradient(bl):
    """Gamma1 = <B100, F>_{-1}, Gamma3 = <B001, F>_{-3} (section "Gradient on the product manifold", local
    coordinates), and the relative gradient sqrt(2|G1|^2 + |G3|^2) / |F| (the
    mode-1 and mode-2 blocks are equal when U = V)."""
    F = bl["F"]
    G1 = np.einsum("xbc,abc->xa", bl["B100"], F)
    G3 = np.einsum("abz,abc->zc", bl["B001"], F)
    nf = np.sqrt(np.sum(F * F))
    rel = np.sqrt(2.0 * np.sum(G1 * G1) + np.sum(G3 * G3)) / nf if nf > 0 else np.inf
    return G1, G3, rel


def newton_model(bl):
    """Linear term b and symmetric matrix A of the second-order model
    phi(d) = phi0 + b^T d + d^T A d with d = [vec(D); vec(T)] (row-major
    vec: D[x, a] -> x*r + a, T[z, c] -> z*r3 + c)."""
    F, B100, B001, B110, B101 = bl["F"], bl["B100"], bl["B001"], bl["B110"], bl["B101"]
    r, _, r3 = F.shape
    A1 = B100.shape[0]
    C1 = B001.shape[2]
    nd, nt = A1 * r, C1 * r3
    N = nd + nt
    G1, G3, _ = local_gradient(bl)
    b = np.concatenate([4.0 * G1.reshape(-1), 2.0 * G3.reshape(-1)])

    # Jacobian of G1 (r*r*r3 x N), built column by column from unit directions
    J = np.zeros((r * r * r3, N))
    for x in range(A1):
        for a in range(r):
            g = np.zeros((r, r, r3))
            g[a, :, :] += B100[x]            # B100.(D)_1 with D = e_x e_a^T
            g[:, a, :] += B100[x]            # B010.(D)_2, B010[a,y,c] = B100[y,a,c]
            J[:, x * r + a] = g.reshape(-1)
    for z in range(C1):
        for c in range(r3):
            g = np.zeros((r, r, r3))
            g[:, :, c] += B001[:, :, z]
            J[:, nd + z * r3 + c] = g.reshape(-1)
    A = J.T @ J

    # 2<F, G2>
    K = 2.0 * np.einsum("abc,xyc->xayb", F, B110).reshape(nd, nd)
    L = 4.0 * np.einsum("abc,xbz->xazc", F, B101).reshape(nd, nt)
    A[:nd, :nd] += K
    A[:nd, nd:] += 0.5 * L
    A[nd:, :nd] += 0.5 * L.T

    # -2 tr(D S1 D^T) - tr(T S3 T^T)
    S1 = np.einsum("abc,dbc->ad", F, F)
    S3 = np.einsum("abc,abd->cd", F, F)
    A[:nd, :nd] -= 2.0 * np.kron(np.eye(A1), S1)
    A[nd:, nd:] -= np.kron(np.eye(C1), S3)
    return b, 0.5 * (A + A.T)


def objective(C, P, S):
    F = mprod(C, P, P, S)
    return float(np.sum(F * F))


def retract(Q, D):
    """Point reached from Q = [P P_perp] along D: orth(P + P_perp D)."""
    r = D.shape[1]
    Y = Q[:, :r] + Q[:, r:] @ D
    q, _ = np.linalg.qr(Y)
    return q


def newton_grassmann(C, P, S, tol, maxit):
    """Newton-Grassmann iterations from (P, S) until the relative local
    gradient is <= tol.  Returns (P, S, iterations, rel, newton_steps).

    Safeguard (a reading; the paper only cites the method): the step solves
    (-2A + mu I) d = b with mu = 0 when -2A is positive definite and the
    step does not decrease g (the plain Newton step near a maximum);
    otherwise mu is raised (to beyond the most negative eigenvalue of -2A,
    then by factors of 4) until both hold.  After 40 failed shifts one HOOI
    step is taken.

    "Does not decrease" is decided up to the rounding error of evaluating g:
    g = sum of squares of C.(P, P, S) is a chain of three contractions of
    lengths k1, k1, k3 followed by a sum of r*r*r3 squares, so each
    evaluation carries a relative forward error of at most gamma_N =
    N u / (1 - N u), N = 2 k1 + k3 + r^2 r3, u = 2^-53 (the standard bound for
    sums of products).  A step is rejected only when g falls by more than
    2 gamma_N: near a maximum a Newton step changes g by about rel^2 g,
    far below what FP64 resolves, and a sharper test rejects good steps."""
    r, r3 = P.shape[1], S.shape[1]
    it = 0
    newton = 0
    rel = np.inf
    mu = 0.0
    u = 2.0 ** -53
    N = 2 * C.shape[0] + C.shape[2] + r * r * r3
    gam = N * u / (1.0 - N * u)
    while True:
        bl = blocks(C, P, S)
        _, _, rel = local_gradient(bl)
        if rel <= tol or it >= maxit:
            break
        b, A = newton_model(bl)
        H = -2.0 * A
        mu0 = 1e-8 * max(np.abs(np.diag(H)).max(), 1e-300)
        g0 = objective(C, P, S)
        nd = (C.shape[0] - r) * r
        accepted = False
        for _ in range(40):
            Hs = H + mu * np.eye(H.shape[0])
            try:
                Lc = np.linalg.cholesky(Hs)
            except np.linalg.LinAlgError:
                lam_min = np.linalg.eigvalsh(Hs)[0]
                mu = max(4.0 * mu, mu0, mu + 2.0 * abs(lam_min))
                continue
            d = np.linalg.solve(Lc.T, np.linalg.solve(Lc, b))
            Pn = retract(bl["Qp"], d[:nd].reshape(C.shape[0] - r, r))
            Sn = retract(bl["Qs"], d[nd:].reshape(C.shape[2] - r3, r3))
            if objective(C, Pn, Sn) >= g0 * (1.0 - 2.0 * gam):
                P, S = Pn, Sn
                accepted = True
                mu = mu / 4.0 if mu > mu0 else 0.0
                break
            mu = max(4.0 * mu, mu0)
        it += 1
        if accepted:
            newton += 1
        else:
            P, S = hooi_step(C, P, S)
    return P, S, it, rel, newton


def inner_solve(C, r, r3, tol, hooi_iters=5, ng_max=50):
    """Algorithm 5 step (i): truncated HOSVD, ``hooi_iters`` HOOI iterations,
    then Newton-Grassmann.  Returns (P, S, info)."""
    P, S = hosvd(C, r, r3)
    for _ in range(hooi_iters):
        P, S = hooi_step(C, P, S)
    P, S, it, rel, newton = newton_grassmann(C, P, S, tol, ng_max)
    return P, S, {"ng_iters": it, "newton_steps": newton, "rel_grad": rel}

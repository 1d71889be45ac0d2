"""Pins for the non-symmetric BKS oracle (oracle/nonsym.py): the three
products against dense brute force, the block-Krylov gradient of Proposition
3.2 against the G-gradient computed with full orthogonal complements, the
n = 1 case (a matrix: the leading singular subspaces and sum of squared
singular values), exact recovery of a planted rank-(3, 2, 2) tensor, and a
(1,2)-symmetric tensor given in full reaching the symmetric oracle's
subspace from a start with V0 = U0."""
import numpy as np
import pytest

from oracle import bks as sbks, nonsym, sptensor


def random_tensor(l, m, n, nnz, seed):
    rng = np.random.default_rng(seed)
    return nonsym.from_coo(l, m, n, rng.integers(0, l, nnz), rng.integers(0, m, nnz),
                           rng.integers(0, n, nnz), rng.standard_normal(nnz))


def orth(rows, cols, seed):
    return np.linalg.qr(np.random.default_rng(seed).standard_normal((rows, cols)))[0]


def test_products_against_dense():
    T = random_tensor(9, 7, 5, 120, 1)
    A = nonsym.dense(T)
    rng = np.random.default_rng(2)
    U, V, W = rng.standard_normal((9, 3)), rng.standard_normal((7, 2)), rng.standard_normal((5, 4))
    want1 = np.einsum("ijk,jb,kc->ibc", A, V, W).reshape(9, -1, order="F")
    want2 = np.einsum("ijk,ia,kc->jac", A, U, W).reshape(7, -1, order="F")
    want3 = np.einsum("ijk,ia,jb->kab", A, U, V).reshape(5, -1, order="F")
    np.testing.assert_allclose(nonsym.mode_product(T, 1, V, W), want1, atol=1e-12)
    np.testing.assert_allclose(nonsym.mode_product(T, 2, U, W), want2, atol=1e-12)
    np.testing.assert_allclose(nonsym.mode_product(T, 3, U, V), want3, atol=1e-12)
    X, Y, Z = orth(9, 4, 3), orth(7, 3, 4), orth(5, 2, 5)
    np.testing.assert_allclose(nonsym.core_tensor(T, X, Y, Z),
                               np.einsum("ijk,ia,jb,kc->abc", A, X, Y, Z), atol=1e-12)


def test_krylov_gradient_equals_global_gradient():
    """Proposition 3.2: one block-Krylov step per mode gives the G-gradient
    without the orthogonal complements."""
    T = random_tensor(12, 10, 8, 400, 7)
    A = nonsym.dense(T)
    U0, V0, W0 = orth(12, 2, 1), orth(10, 3, 2), orth(8, 2, 3)
    st = nonsym.bk_step(T, U0, V0, W0, 1e-14)
    want = nonsym.local_gradient(A, U0, V0, W0)
    assert abs(st["rel"] - want) <= 1e-12 * want
    np.testing.assert_allclose(st["F"], np.einsum("ijk,ia,jb,kc->abc", A, U0, V0, W0), atol=1e-12)


def test_matrix_case():
    """n = 1, r3 = 1: the best rank-(r, r, 1) approximation of a matrix M is
    its leading r singular pairs, ||F||^2 = sum of their squares."""
    rng = np.random.default_rng(4)
    M = rng.standard_normal((30, 20)) * (rng.random((30, 20)) < 0.4)
    M += 6.0 * np.outer(rng.standard_normal(30), rng.standard_normal(20)) / 10
    ii, jj = np.nonzero(M)
    T = nonsym.from_coo(30, 20, 1, ii, jj, np.zeros_like(ii), M[ii, jj])
    res = nonsym.bks_solve(T, (3, 3, 1), orth(30, 3, 1), orth(20, 3, 2), np.ones((1, 1)), tol=1e-12)
    Us, s, Vt = np.linalg.svd(M)
    assert res["converged"]
    assert sbks.subspace_distance(Us[:, :3], res["U"]) <= 1e-10
    assert sbks.subspace_distance(Vt[:3].T, res["V"]) <= 1e-10
    assert abs(np.sum(res["F"] ** 2) - np.sum(s[:3] ** 2)) <= 1e-10 * np.sum(s[:3] ** 2)


def test_planted_recovery():
    rng = np.random.default_rng(5)
    l, m, n = 200, 150, 60
    # disjoint sparse supports make the factors orthonormal
    def factor(rows, cols, per):
        F = np.zeros((rows, cols))
        idx = rng.permutation(rows)[: cols * per].reshape(cols, per)
        for c in range(cols):
            v = rng.standard_normal(per)
            F[idx[c], c] = v / np.linalg.norm(v)
        return F
    Uf, Vf, Wf = factor(l, 3, 6), factor(m, 2, 6), factor(n, 2, 5)
    G = np.zeros((3, 2, 2))
    G[0, 0, 0], G[1, 1, 1], G[2, 0, 1], G[1, 0, 0] = 10.0, 6.0, 4.0, 1.5
    A = np.einsum("abc,ia,jb,kc->ijk", G, Uf, Vf, Wf)
    ii, jj, kk = np.nonzero(A)
    T = nonsym.from_coo(l, m, n, ii, jj, kk, A[ii, jj, kk])
    res = nonsym.bks_solve(T, (3, 2, 2), orth(l, 3, 1), orth(m, 2, 2), orth(n, 2, 3), tol=1e-12)
    assert res["converged"]
    for key, F in (("U", Uf), ("V", Vf), ("W", Wf)):
        assert sbks.subspace_distance(F, res[key]) <= 1e-10, key
    assert abs(np.sqrt(np.sum(res["F"] ** 2)) - np.sqrt(np.sum(A ** 2))) <= 1e-10 * np.sqrt(np.sum(A ** 2))


def test_symmetric_tensor_matches_the_symmetric_oracle():
    """A (1,2)-symmetric tensor given in full: from a start with V0 = U0 the
    general iteration reaches the symmetric oracle's subspace (a planted,
    well-separated rank-(2, 2, 2) part)."""
    from paper_2012_07595_amd import workloads
    c = workloads.dense_signal_noise(30, 30, 2, 2, 1e-2, seed=3)
    S = sptensor.from_coo(c.m, c.n, c.i, c.j, c.k, c.val.astype(np.float64))
    A = sptensor.dense(S)
    ii, jj, kk = np.nonzero(A)
    T = nonsym.from_coo(30, 30, 30, ii, jj, kk, A[ii, jj, kk])
    U0, W0 = workloads.random_start(30, 30, 2, 2, 5)
    ref = sbks.bks_solve(S, 2, 2, U0, W0)
    got = nonsym.bks_solve(T, (2, 2, 2), U0, U0, W0, tol=1e-12)
    assert got["converged"]
    assert sbks.subspace_distance(ref["U"], got["U"]) <= 1e-9
    assert sbks.subspace_distance(ref["U"], got["V"]) <= 1e-9
    assert sbks.subspace_distance(ref["W"], got["W"]) <= 1e-9

"""Pins for the oracle's contractions (section "Multilinear tensor-matrix multiplication"): dense brute force on tiny
tensors, (1,2)-symmetry of every product, the cross-kernel identity, norm
invariance under orthogonal transforms (section "Inner product and norm, contractions") and the p = 1 vector
case (tensor-times-vector products of the minimal Krylov recursion)."""
import numpy as np
import pytest

from oracle import sptensor, ttmc
from paper_2012_07595_amd import workloads


def tiny(seed, m=9, n=5, nnz=60):
    c = workloads.sparse_sym(m, n, nnz, zipf=0.0, values="normal", seed=seed, dtype=np.float64)
    return sptensor.from_coo(c.m, c.n, c.i, c.j, c.k, c.val)


def dense_free3(A, X, Y):
    # T3(a, b, k) = sum_ij A(i,j,k) X(i,a) Y(j,b), unfolded column a + px*b
    T = np.zeros((A.shape[2], X.shape[1], Y.shape[1]))
    m = A.shape[0]
    for i in range(m):
        for j in range(m):
            T += A[i, j, :][:, None, None] * np.outer(X[i], Y[j])[None]
    return T.transpose(0, 2, 1).reshape(A.shape[2], -1)


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("px,py", [(1, 1), (2, 3), (4, 2)])
def test_free3_brute_force(seed, px, py):
    T = tiny(seed)
    A = sptensor.dense(T)
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((T.m, px))
    Y = rng.standard_normal((T.m, py))
    np.testing.assert_allclose(ttmc.free3(T, X, Y), dense_free3(A, X, Y), rtol=0, atol=1e-12)


@pytest.mark.parametrize("p", [1, 2, 3, 5])
def test_free3_sym_half_is_triunfold3(p):
    T = tiny(7)
    A = sptensor.dense(T)
    X = np.random.default_rng(p).standard_normal((T.m, p))
    full = np.einsum("ijk,ia,jb->kab", A, X, X)
    # the product is (1,2)-symmetric
    np.testing.assert_allclose(full, full.transpose(0, 2, 1), atol=1e-12)
    half = ttmc.free3(T, X, sym_half=True)
    assert half.shape == (T.n, p * (p + 1) // 2)
    col = 0
    for b in range(p):
        for a in range(b + 1):
            np.testing.assert_allclose(half[:, col], full[:, a, b], atol=1e-12)
            col += 1
    np.testing.assert_allclose(ttmc.triu_to_full(half, p),
                               full.transpose(0, 2, 1).reshape(T.n, -1), atol=1e-12)


@pytest.mark.parametrize("py,pz", [(1, 1), (2, 3), (3, 2)])
def test_free1_brute_force_and_symmetry(py, pz):
    T = tiny(11)
    A = sptensor.dense(T)
    rng = np.random.default_rng(3)
    Y = rng.standard_normal((T.m, py))
    Z = rng.standard_normal((T.n, pz))
    ref23 = np.einsum("ijk,jb,kc->icb", A, Y, Z).reshape(T.m, -1)   # column b + py*c
    ref13 = np.einsum("ijk,ib,kc->jcb", A, Y, Z).reshape(T.m, -1)   # A.(Y, Z)_{1,3}
    got = ttmc.free1(T, Y, Z)
    np.testing.assert_allclose(got, ref23, atol=1e-12)
    np.testing.assert_allclose(got, ref13, atol=1e-12)


@pytest.mark.parametrize("py,pz", [(1, 1), (2, 3), (4, 2)])
def test_free1_rows_brute_force(py, pz):
    """The per-row FREE1 (sampled rows of large tensors) against the dense
    definition, on a tensor with diagonal (i = j) entries, an empty row and a
    repeated row in the sample."""
    T = tiny(13, m=12, n=4, nnz=50)
    A = sptensor.dense(T)
    assert np.any(T.i == T.j)
    rng = np.random.default_rng(4)
    Y = rng.standard_normal((T.m, py))
    Z = rng.standard_normal((T.n, pz))
    ref = np.einsum("ijk,jb,kc->icb", A, Y, Z).reshape(T.m, -1)
    deg = np.bincount(np.concatenate([T.i, T.j]), minlength=T.m)
    rows = [0, int(np.argmax(deg)), int(np.argmax(deg)), T.m - 1]
    if np.any(deg == 0):
        rows.append(int(np.flatnonzero(deg == 0)[0]))
    np.testing.assert_allclose(ttmc.free1_rows(T, Y, Z, rows), ref[rows], rtol=0, atol=1e-12)


def test_mode3_brute_force():
    T = tiny(5)
    A = sptensor.dense(T)
    Z = np.random.default_rng(9).standard_normal((T.n, 3))
    pi, pj, t = ttmc.mode3(T, Z)
    assert np.all(pi <= pj)
    key = pi * T.m + pj
    assert np.all(np.diff(key) > 0)
    ref = np.einsum("ijk,kc->ijc", A, Z)
    np.testing.assert_allclose(t, ref[pi, pj], atol=1e-12)
    # every stored pair appears, nothing else
    assert set(zip(pi.tolist(), pj.tolist())) == set(zip(T.i.tolist(), T.j.tolist()))


def test_cross_kernel_identity():
    """X^T A.(X, Z)_{2,3} and Z^T A.(X, X)_{1,2} are both C = A.(X, X, Z)."""
    T = tiny(13)
    rng = np.random.default_rng(1)
    X = rng.standard_normal((T.m, 3))
    Z = rng.standard_normal((T.n, 2))
    C1 = X.T @ ttmc.free1(T, X, Z)                      # (a) x (b + 3c)
    C3 = Z.T @ ttmc.triu_to_full(ttmc.free3(T, X, sym_half=True), 3)  # (c) x (a + 3b)
    Ca = C1.reshape(3, 3, 2, order="F")
    Cb = C3.reshape(2, 3, 3, order="F").transpose(1, 2, 0)
    np.testing.assert_allclose(Ca, Cb, atol=1e-12)
    np.testing.assert_allclose(Ca, Ca.transpose(1, 0, 2), atol=1e-12)


def test_norm_invariance_square_orthogonal():
    """||A.(Q, Q, Q3)|| = ||A|| for square orthogonal Q, Q3 (section "Inner product and norm, contractions")."""
    T = tiny(17)
    rng = np.random.default_rng(2)
    Q = np.linalg.qr(rng.standard_normal((T.m, T.m)))[0]
    Q3 = np.linalg.qr(rng.standard_normal((T.n, T.n)))[0]
    C = Q3.T @ ttmc.triu_to_full(ttmc.free3(T, Q, sym_half=True), T.m)
    assert abs(np.sum(C * C) - sptensor.frob2(T)) < 1e-10 * sptensor.frob2(T)
    A = sptensor.dense(T)
    assert abs(np.sum(A * A) - sptensor.frob2(T)) < 1e-12 * sptensor.frob2(T)


def test_vector_case():
    """p = 1: A.(u, v)_{1,2} and A.(v, w)_{2,3} are the tensor-times-vector
    products of the minimal Krylov recursion."""
    T = tiny(19)
    A = sptensor.dense(T)
    rng = np.random.default_rng(4)
    u, v = rng.standard_normal(T.m), rng.standard_normal(T.m)
    w = rng.standard_normal(T.n)
    np.testing.assert_allclose(ttmc.free3(T, u[:, None], v[:, None])[:, 0],
                               np.einsum("ijk,i,j->k", A, u, v), atol=1e-12)
    np.testing.assert_allclose(ttmc.free1(T, v[:, None], w[:, None])[:, 0],
                               np.einsum("ijk,j,k->i", A, v, w), atol=1e-12)


def test_canonicalisation_and_duplicates():
    # (0,1,0) and (1,0,0) name one entry; with summing they add
    T = sptensor.from_coo(3, 2, [0, 1, 2], [1, 0, 2], [0, 0, 1], [1.0, 2.0, 4.0])
    assert T.nnz == 2
    A = sptensor.dense(T)
    assert A[0, 1, 0] == 3.0 and A[1, 0, 0] == 3.0 and A[2, 2, 1] == 4.0
    assert sptensor.frob2(T) == 2 * 9.0 + 16.0
    with pytest.raises(ValueError):
        sptensor.from_coo(3, 2, [0, 1], [1, 0], [0, 0], [1.0, 2.0], sum_duplicates=False)
    with pytest.raises(IndexError):
        sptensor.from_coo(3, 2, [3], [0], [0], [1.0])
    with pytest.raises(ValueError):
        sptensor.from_coo(3, 2, [0], [0], [0], [np.nan])

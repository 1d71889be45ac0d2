"""Pins for two parts of the oracle that the solver parity tests lean on.

- oracle.bks.subspace_distance, the comparison behind every subspace parity
  claim, against principal angles fixed by construction and against SciPy's
  subspace_angles (an independent computation: Bjorck-Golub, with the sine
  form for small angles).
- The inner Newton-Grassmann solve (Algorithm 5 step (i), section
  "Experiments": the inner iteration uses the same tolerance as the outer
  one) must reach the requested relative gradient on its own, with no stop
  rule other than the tolerance and the iteration cap; and its step
  acceptance must not reject a plain Newton step because of rounding noise
  in the objective (the case that used to stall it with an ever larger
  shift).
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import bks, core


def rotated_pair(m, sines, seed):
    """Orthonormal U_ref, U (m x r) whose principal angles have the given
    sines: U_ref = Q[:, :r], U = Q (cos t_i e_i + sin t_i e_{r+i}) for a
    random orthogonal Q."""
    rng = np.random.default_rng(seed)
    r = len(sines)
    Q, _ = np.linalg.qr(rng.standard_normal((m, m)))
    s = np.asarray(sines, dtype=np.float64)
    c = np.sqrt((1.0 - s) * (1.0 + s))
    B = np.zeros((m, r))
    B[np.arange(r), np.arange(r)] = c
    B[r + np.arange(r), np.arange(r)] = s
    return Q[:, :r], Q @ B


@pytest.mark.parametrize("smax", [1e-12, 1e-8, 0.3])
def test_subspace_distance_known_angles(smax):
    sines = [smax, 0.5 * smax, 0.1 * smax, 0.0]
    Uref, U = rotated_pair(60, sines, seed=int(-np.log10(smax) * 7) + 1)
    d = bks.subspace_distance(Uref, U)
    # Q is orthogonal to ~1e-15, which bounds the absolute error
    assert abs(d - smax) <= 1e-14 + 1e-10 * smax, (d, smax)
    # invariant under a change of basis inside either subspace
    R, _ = np.linalg.qr(np.random.default_rng(2).standard_normal((4, 4)))
    assert abs(bks.subspace_distance(Uref @ R, U @ R.T) - d) <= 1e-14 + 1e-10 * smax
    # symmetric in its arguments for equal dimensions
    assert abs(bks.subspace_distance(U, Uref) - d) <= 1e-14 + 1e-10 * smax


def test_subspace_distance_against_scipy():
    rng = np.random.default_rng(7)
    for m, r in [(40, 3), (200, 8), (25, 25)]:
        A, _ = np.linalg.qr(rng.standard_normal((m, r)))
        B, _ = np.linalg.qr(A + 1e-3 * rng.standard_normal((m, r)))
        for X, Y in [(A, B), (A, np.linalg.qr(rng.standard_normal((m, r)))[0])]:
            want = np.sin(scipy.linalg.subspace_angles(X, Y).max())
            got = bks.subspace_distance(X, Y)
            assert abs(got - want) <= 1e-12 * max(want, 1e-3), (m, r, got, want)
    # identical spans: zero up to rounding; orthogonal spans: one
    A, _ = np.linalg.qr(rng.standard_normal((30, 4)))
    assert bks.subspace_distance(A, A) <= 1e-15
    Q, _ = np.linalg.qr(rng.standard_normal((30, 30)))
    assert abs(bks.subspace_distance(Q[:, :4], Q[:, 4:8]) - 1.0) <= 1e-14


def sym_core(k1, k3, r, r3, noise, seed):
    """Dense (1,2)-symmetric core: planted rank-(r, r, r3) part with a
    decaying superdiagonal plus symmetric N(0, noise^2) entries, rotated by
    random orthogonal matrices."""
    rng = np.random.default_rng(seed)
    C = np.zeros((k1, k1, k3))
    for t in range(min(r, r3)):
        C[t, t, t] = 10.0 * 0.8 ** t
    for t in range(min(r, r3), r):
        C[t, t, r3 - 1] = 10.0 * 0.8 ** t
    N = rng.standard_normal((k1, k1, k3)) * noise
    C = C + 0.5 * (N + N.transpose(1, 0, 2))
    Q1, _ = np.linalg.qr(rng.standard_normal((k1, k1)))
    Q3, _ = np.linalg.qr(rng.standard_normal((k3, k3)))
    return core.mprod(C, Q1, Q1, Q3)


@pytest.mark.parametrize("k1,k3,r,r3,noise,seed", [
    (12, 8, 2, 2, 0.3, 1),
    (20, 13, 2, 2, 1.0, 2),
    (36, 21, 3, 3, 0.5, 3),
    (70, 40, 5, 5, 0.2, 4),
])
def test_inner_solve_reaches_the_tolerance(k1, k3, r, r3, noise, seed):
    C = sym_core(k1, k3, r, r3, noise, seed)
    P, S, info = core.inner_solve(C, r, r3, 1e-13, hooi_iters=5, ng_max=50)
    assert info["rel_grad"] <= 1e-13 and info["ng_iters"] < 50, info
    # the returned point is a stationary point of the projected problem
    bl = core.blocks(C, P, S)
    assert core.local_gradient(bl)[2] <= 1e-13


@pytest.mark.parametrize("variant,s", [("min", 3), ("bk", 2), ("max", 2)])
def test_every_inner_solve_of_a_bks_run_reaches_the_tolerance(variant, s):
    """Whole oracle BKS runs on an Example-1-like tensor (rank-(2,2,2) signal
    plus 1% noise): every inner solve ends at the tolerance, none at the cap.
    Here a plain Newton step from a relative gradient of ~1e-8 changes g by
    ~1e-15 relative, within the rounding of its evaluation; an acceptance
    test sharper than that bound rejects it, the shift then grows, and the
    iteration crawls for tens of steps or stalls at ~1e-10 until the cap."""
    from oracle import sptensor
    from paper_2012_07595_amd import workloads
    c = workloads.dense_signal_noise(30, 30, 2, 2, 1e-2, seed=4)
    T = sptensor.from_coo(c.m, c.n, c.i, c.j, c.k, c.val.astype(np.float64))
    U0, W0 = workloads.random_start(30, 30, 2, 2, 6)
    res = bks.bks_solve(T, 2, 2, U0, W0, variant=variant, s=s, p=4)
    assert res["converged"]
    for info in res["inner"]:
        # quadratic convergence: a handful of steps (the paper reports 4-5
        # typical inner iterations), never the cap
        assert info["rel_grad"] <= 1e-13 and info["ng_iters"] <= 10, info


def test_slice_scaling_closed_forms():
    """Slice scalings (Examples 3 and 4) against closed forms: the complete
    graph K_q times c has largest eigenvalue c (q - 1); a diagonal slice has
    spectral radius max |d|; a rank-one slice u u^T has ||u||^2; the 2 x 2
    slice [[a, b], [b, c]] has Frobenius norm sqrt(a^2 + 2 b^2 + c^2)."""
    from oracle import preprocess, sptensor
    m, q, c = 30, 7, 2.5
    A = np.zeros((m, m, 4))
    idx = np.arange(3, 3 + q)
    A[np.ix_(idx, idx, [0])] = c
    A[idx, idx, 0] = 0.0                       # K_q: no self loops
    d = np.array([1.0, -4.0, 2.0])
    A[[5, 9, 12], [5, 9, 12], 1] = d           # diagonal slice
    u = np.zeros(m)
    u[[2, 8, 20]] = [1.0, -2.0, 0.5]
    A[:, :, 2] = np.outer(u, u)                # rank one
    A[[0, 0, 1, 1], [0, 1, 0, 1], 3] = [1.5, -0.7, -0.7, 3.0]
    T = sptensor.from_dense(A)
    L = preprocess.scale_slices(T, "lambda_max")
    F = preprocess.scale_slices(T, "frobenius")
    want_l = [c * (q - 1), 4.0, u @ u, None]
    for k, w in enumerate(want_l):
        if w is None:
            continue
        np.testing.assert_allclose(L.a[L.k == k], T.a[T.k == k] / w, rtol=1e-13)
    np.testing.assert_allclose(F.a[F.k == 3], T.a[T.k == 3] / np.sqrt(1.5 ** 2 + 2 * 0.7 ** 2 + 9.0),
                               rtol=1e-14)
    # every nonempty slice of the Frobenius-scaled tensor has norm 1, so
    # ||A||^2 is the number of nonempty slices
    assert abs(sptensor.frob2(F) - 4.0) <= 1e-13

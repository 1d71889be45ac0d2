"""CPU baseline B (C++/OpenMP FP64 products + the oracle's BKS algorithm)
against the FP64 oracle: every product kind to rounding, and a whole BKS
solve to the same subspaces.  CPU only."""
import numpy as np
import pytest

from baseline import cpu
from oracle import bks, sptensor, ttmc
from paper_2012_07595_amd import workloads


@pytest.fixture(scope="module")
def T():
    c = workloads.sparse_sym(800, 60, 30_000, zipf=1.2, values="normal", seed=5, dtype=np.float64)
    return sptensor.from_coo(c.m, c.n, c.i, c.j, c.k, c.val)


def close(a, b):
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-12 * np.abs(b).max())


def test_products_match_the_oracle(T):
    rng = np.random.default_rng(1)
    X, Y = rng.standard_normal((T.m, 5)), rng.standard_normal((T.m, 3))
    Z = rng.standard_normal((T.n, 4))
    close(cpu.free3(T, X, sym_half=True), ttmc.free3(T, X, sym_half=True))
    close(cpu.free3(T, X, Y), ttmc.free3(T, X, Y))
    close(cpu.free3(T, X), ttmc.free3(T, X))
    close(cpu.free1(T, Y, Z), ttmc.free1(T, Y, Z))
    a, b, t = cpu.mode3(T, Z)
    ra, rb, rt = ttmc.mode3(T, Z)
    np.testing.assert_array_equal(a, ra)
    np.testing.assert_array_equal(b, rb)
    close(t, rt)
    # the oracle's own functions are restored after the context
    with cpu.products():
        assert ttmc.free3 is cpu.free3
    assert ttmc.free3 is not cpu.free3


def test_bks_solve_matches_the_oracle():
    c = workloads.dense_signal_noise(40, 40, 2, 2, 1e-2, seed=3)
    T = sptensor.from_coo(c.m, c.n, c.i, c.j, c.k, c.val.astype(np.float64))
    U0, W0 = workloads.random_start(40, 40, 2, 2, 5)
    ref = bks.bks_solve(T, 2, 2, U0, W0)
    got = cpu.bks_solve(T, 2, 2, U0, W0)
    assert got["converged"] and ref["converged"]
    assert bks.subspace_distance(ref["U"], got["U"]) <= 1e-10
    assert bks.subspace_distance(ref["W"], got["W"]) <= 1e-10
    assert cpu.threads() >= 1

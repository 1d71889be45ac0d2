"""General (non-symmetric) tensors: bks_gttmc against the oracle's mode
products (FP32 to the 1e-5 bar of the symmetric products, FP64 and FP32
values with FP64 accumulation to 1e-12), and bks_gsolve against the
oracle's non-symmetric BKS (oracle/nonsym.py) from the same start: planted
rank-(3, 2, 2) recovery, and a noisy tensor at rank (2, 3, 2) in FP64 and
mixed precision (subspace angle <= 1e-8, ||F|| to 1e-10)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import bks as obks, nonsym
from paper_2012_07595_amd import bks

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def ctx():
    c = bks.Ctx(0)
    yield c
    c.close()


def random_coo(l, m, n, nnz, seed, zipf=False):
    rng = np.random.default_rng(seed)
    if zipf:
        def draw(d):
            w = np.arange(1, d + 1, dtype=np.float64) ** -1.2
            return np.minimum(np.searchsorted(np.cumsum(w) / w.sum(), rng.random(nnz)), d - 1)
        i, j, k = draw(l), draw(m), rng.integers(0, n, nnz)
    else:
        i, j, k = rng.integers(0, l, nnz), rng.integers(0, m, nnz), rng.integers(0, n, nnz)
    key = np.unique((i * m + j) * n + k)
    return (key // (m * n), (key // n) % m, key % n, rng.standard_normal(key.shape[0]))


@pytest.mark.parametrize("prec", [bks.F32, bks.F64, bks.F32IN_F64ACC])
@pytest.mark.parametrize("p1,p2", [(1, 1), (3, 4), (5, 5), (8, 6), (20, 20)])
def test_gttmc_matches_the_oracle(ctx, prec, p1, p2):
    l, m, n = 700, 500, 90
    i, j, k, v = random_coo(l, m, n, 40_000, 11, zipf=True)
    if prec != bks.F64:
        v = v.astype(np.float32).astype(np.float64)
    t = ctx.upload_general(l, m, n, i, j, k, v if prec == bks.F64 else v.astype(np.float32))
    o = nonsym.from_coo(l, m, n, i, j, k, v)
    rng = np.random.default_rng(12)
    dims = (l, m, n)
    dt = torch.float32 if prec == bks.F32 else torch.float64
    for mode in range(3):
        a, b = [x for x in range(3) if x != mode]
        B1 = rng.standard_normal((dims[a], p1))
        B2 = rng.standard_normal((dims[b], p2))
        if prec == bks.F32:
            B1 = B1.astype(np.float32).astype(np.float64)
            B2 = B2.astype(np.float32).astype(np.float64)
        out = torch.full((dims[mode], p1 * p2), float("nan"), dtype=dt, device=DEV)
        ctx.gttmc(t, mode, torch.tensor(B1, dtype=dt, device=DEV),
                  torch.tensor(B2, dtype=dt, device=DEV), out, prec=prec)
        torch.cuda.synchronize()
        got = out.cpu().numpy().astype(np.float64)
        want = nonsym.mode_product(o, mode + 1, B1, B2)
        tol = 1e-5 if prec == bks.F32 else 1e-12
        assert np.all(np.isfinite(got))
        err = np.linalg.norm(got - want) / np.linalg.norm(want)
        assert err <= tol, (mode, err)
    t.free()


def orth(rows, cols, seed):
    return np.linalg.qr(np.random.default_rng(seed).standard_normal((rows, cols)))[0]


def planted(l, m, n, seed):
    rng = np.random.default_rng(seed)

    def factor(rows, cols, per):
        F = np.zeros((rows, cols))
        idx = rng.permutation(rows)[: cols * per].reshape(cols, per)
        for c in range(cols):
            x = rng.standard_normal(per)
            F[idx[c], c] = x / np.linalg.norm(x)
        return F
    Uf, Vf, Wf = factor(l, 3, 6), factor(m, 2, 6), factor(n, 2, 5)
    G = np.zeros((3, 2, 2))
    G[0, 0, 0], G[1, 1, 1], G[2, 0, 1], G[1, 0, 0] = 10.0, 6.0, 4.0, 1.5
    A = np.einsum("abc,ia,jb,kc->ijk", G, Uf, Vf, Wf)
    ii, jj, kk = np.nonzero(A)
    return (ii, jj, kk, A[ii, jj, kk]), (Uf, Vf, Wf), np.sqrt(np.sum(A * A))


def test_gsolve_planted_recovery(ctx):
    l, m, n = 300, 200, 80
    (i, j, k, v), (Uf, Vf, Wf), normA = planted(l, m, n, 5)
    t = ctx.upload_general(l, m, n, i, j, k, v)
    U0, V0, W0 = orth(l, 3, 1), orth(m, 2, 2), orth(n, 2, 3)
    for prec in (bks.PREC_FP64, bks.PREC_MIXED):
        U, V, W, F, info, rc = ctx.gsolve(t, (3, 2, 2), U0, V0, W0, precision=prec, tol=1e-11)
        assert info.converged, (prec, info.rel_grad)
        for got, want in ((U, Uf), (V, Vf), (W, Wf)):
            assert obks.subspace_distance(want, got) <= 1e-9
        assert abs(np.sqrt(np.sum(F ** 2)) - normA) <= 1e-10 * normA
    t.free()


@pytest.mark.parametrize("precision", [bks.PREC_FP64, bks.PREC_MIXED])
def test_gsolve_matches_the_oracle(ctx, precision):
    l, m, n = 400, 300, 60
    (pi, pj, pk, pv), _, _ = planted(l, m, n, 7)
    i, j, k, v = random_coo(l, m, n, 20_000, 8)
    # a planted part well above the noise keeps the subspaces well conditioned
    ii = np.concatenate([i, pi]); jj = np.concatenate([j, pj]); kk = np.concatenate([k, pk])
    vv = np.concatenate([0.05 * v, 5.0 * pv]).astype(np.float32).astype(np.float64)
    o = nonsym.from_coo(l, m, n, ii, jj, kk, vv)
    t = ctx.upload_general(l, m, n, o.i, o.j, o.k, o.a)
    U0, V0, W0 = orth(l, 2, 4), orth(m, 3, 5), orth(n, 2, 6)
    ref = nonsym.bks_solve(o, (2, 3, 2), U0, V0, W0, tol=1e-11)
    U, V, W, F, info, rc = ctx.gsolve(t, (2, 3, 2), U0, V0, W0, precision=precision, tol=1e-11)
    print(f"gsolve: converged {info.converged} iters {info.outer_iters} (oracle "
          f"{ref['outer_iters']}) rel {info.rel_grad:.1e}")
    assert info.converged and ref["converged"]
    for key, got in (("U", U), ("V", V), ("W", W)):
        assert obks.subspace_distance(ref[key], got) <= 1e-8, key
    nf, nr = np.sqrt(np.sum(F ** 2)), np.sqrt(np.sum(ref["F"] ** 2))
    assert abs(nf - nr) <= 1e-10 * nr
    t.free()


def test_general_argument_errors(ctx):
    t = ctx.upload_general(10, 8, 6, [0, 9], [1, 7], [2, 5], np.array([1.0, 2.0]))
    with pytest.raises(bks.BksError) as e:
        ctx.upload_general(10, 8, 6, [0, 10], [1, 7], [2, 5], np.array([1.0, 2.0]))
    assert e.value.code == bks.EINDEX
    with pytest.raises(bks.BksError) as e:
        ctx.upload_general(10, 8, 6, [0, 0], [1, 1], [2, 2], np.array([1.0, 2.0]))
    assert e.value.code == bks.EDUP
    for r in [(0, 1, 1), (3, 1, 1), (2, 2, 5)]:
        with pytest.raises(bks.BksError) as e:
            ctx.gsolve(t, r)
        assert e.value.code == bks.EINVAL
    # the symmetric entry points refuse a general tensor
    with pytest.raises(bks.BksError) as e:
        ctx.solve(t, 2, 2)
    assert e.value.code == bks.EINVAL

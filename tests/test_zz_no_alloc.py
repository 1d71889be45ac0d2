"""bks_ttmc_noalloc: the product entry point that allocates no device memory
(its workspaces live in the library's fixed per-device scratch).  Checked
against bks_ttmc on the same inputs -- bitwise, since both run the same
kernels on the same schedule -- and against the FP64 oracle to the product
parity bar, on two calls in a row of which the second is smaller, for
every narrow product kind and precision.  Sizes beyond the scratch and the
wide symmetric product are refused with an error, and nothing is written."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import sptensor, ttmc as ref
from paper_2012_07595_amd import bks, workloads

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def dev(a, prec):
    return torch.tensor(a, dtype=torch.float32 if prec == bks.F32 else torch.float64, device=DEV)


def products(ctx, t, o, prec, seed, noalloc):
    """Every narrow product kind on tensor t: (name, device result, oracle)."""
    rng = np.random.default_rng(seed)
    cast = (lambda a: a.astype(np.float32).astype(np.float64)) if prec == bks.F32 else (lambda a: a)
    X = cast(rng.standard_normal((o.m, 5)))
    Y = cast(rng.standard_normal((o.m, 4)))
    Z = cast(rng.standard_normal((o.n, 3)))
    X20 = cast(rng.standard_normal((o.m, 20)))
    out = []
    dt = torch.float32 if prec == bks.F32 else torch.float64

    def run(name, op, B1, B2, rows, q, sym, want):
        res = torch.full((rows, q), float("nan"), dtype=dt, device=DEV)
        ctx.ttmc(t, op, None if B1 is None else dev(B1, prec), None if B2 is None else dev(B2, prec),
                 res, sym_half=sym, prec=prec, noalloc=noalloc)
        torch.cuda.synchronize()
        out.append((name, res.cpu().numpy().astype(np.float64), want))

    run("free3_sym5", bks.FREE3, X, None, o.n, 15, True, ref.free3(o, X, sym_half=True))
    run("free3_sym20", bks.FREE3, X20, None, o.n, 210, True, ref.free3(o, X20, sym_half=True))
    run("free3_xy", bks.FREE3, X, Y, o.n, 20, False, ref.free3(o, X, Y))
    run("free1", bks.FREE1, Y, Z, o.m, 12, False, ref.free1(o, Y, Z))
    run("mode3", bks.MODE3, None, Z, t.npairs, 3, False, ref.mode3(o, Z)[2])
    return out


@pytest.mark.parametrize("prec", [bks.F32, bks.F64, bks.F32IN_F64ACC])
def test_noalloc_matches_ttmc_on_two_calls(prec):
    ctx = bks.Ctx(0)
    try:
        big = workloads.sparse_sym(6000, 300, 150_000, zipf=1.3, values="abs", seed=81,
                                   dtype=np.float64)
        small = workloads.sparse_sym(700, 40, 9_000, zipf=1.1, values="normal", seed=82,
                                     dtype=np.float64)
        for q, coo in enumerate((big, small)):   # the second call is smaller
            if prec != bks.F64:
                coo = coo.astype(np.float32)
            t = ctx.upload_coo(coo)
            o = sptensor.from_coo(coo.m, coo.n, coo.i, coo.j, coo.k, coo.val.astype(np.float64))
            na = products(ctx, t, o, prec, 90 + q, noalloc=True)
            wa = products(ctx, t, o, prec, 90 + q, noalloc=False)
            tol = 1e-5 if prec == bks.F32 else 1e-12
            for (name, got, want), (_, got_ref, _) in zip(na, wa):
                assert np.all(np.isfinite(got)), name
                assert np.array_equal(got, got_ref), f"{name}: differs from bks_ttmc"
                err = np.linalg.norm(got - want) / max(np.linalg.norm(want), 1e-300)
                assert err <= tol, (name, err)
            t.free()
    finally:
        ctx.close()


def test_noalloc_refuses_what_does_not_fit():
    ctx = bks.Ctx(0)
    try:
        # 2.5e6 rows of a 20-wide factor: the packed copy alone is 320 MB,
        # beyond the 256 MiB scratch
        m = 2_500_000
        coo = workloads.sparse_sym(m, 4, 1000, seed=83).astype(np.float32)
        t = ctx.upload_coo(coo)
        Y = torch.ones((m, 20), dtype=torch.float32, device=DEV)
        Z = torch.ones((4, 1), dtype=torch.float32, device=DEV)
        out = torch.full((m, 20), 7.0, dtype=torch.float32, device=DEV)
        with pytest.raises(bks.BksError) as e:
            ctx.ttmc(t, bks.FREE1, Y, Z, out, noalloc=True)
        assert e.value.code == bks.EINVAL and "scratch" in str(e.value)
        torch.cuda.synchronize()
        assert bool((out == 7.0).all()), "a refused call wrote its output"
        # the wide symmetric (core) product is not offered
        X = torch.ones((m, 30), dtype=torch.float32, device=DEV)
        o3 = torch.zeros((4, 465), dtype=torch.float32, device=DEV)
        with pytest.raises(bks.BksError) as e:
            ctx.ttmc(t, bks.FREE3, X, None, o3, sym_half=True, noalloc=True)
        assert e.value.code == bks.EINVAL
        # and the entry point still works afterwards
        small = workloads.sparse_sym(300, 20, 3000, seed=84).astype(np.float32)
        ts = ctx.upload_coo(small)
        Xs = torch.randn((300, 3), dtype=torch.float32, device=DEV)
        a = torch.empty((20, 6), dtype=torch.float32, device=DEV)
        b = torch.empty((20, 6), dtype=torch.float32, device=DEV)
        ctx.ttmc(ts, bks.FREE3, Xs, None, a, sym_half=True, noalloc=True)
        ctx.ttmc(ts, bks.FREE3, Xs, None, b, sym_half=True)
        torch.cuda.synchronize()
        assert torch.equal(a, b)
    finally:
        ctx.close()

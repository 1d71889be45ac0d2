"""Slice scaling at upload (BKS_SCALE_FROBENIUS, BKS_SCALE_LAMBDA_MAX; section
"Experiments", Examples 3 and 4) against the oracle's scale_slices: the
products of the scaled tensor (FP64 values, FP64 accumulation) to 1e-12, its
norm, and a rank-(2,2,2) BKS solve of the lambda_max-scaled tensor (the
scaled-Reuters experiment's setting) against the oracle's solve."""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import bks as obks, preprocess, sptensor, ttmc as ref
from paper_2012_07595_amd import bks, workloads

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def ctx():
    c = bks.Ctx(0)
    yield c
    c.close()


def reuters_like(seed=71):
    # positive integer weights on Zipf(1.0) indices: graph slices with a
    # Perron eigenvalue, small enough for the oracle's dense slice eigensolves
    c = workloads.sparse_sym(1200, 24, 40_000, zipf=1.0, values="ones", seed=seed,
                             dtype=np.float64)
    w = 1.0 + np.floor(np.random.default_rng(seed).pareto(2.0, c.val.shape[0]))
    return dataclasses.replace(c, val=w)


def products_match(ctx, t, o):
    rng = np.random.default_rng(3)
    X = rng.standard_normal((o.m, 4))
    Z = rng.standard_normal((o.n, 3))
    dt = torch.float64
    out = torch.empty((o.n, 10), dtype=dt, device=DEV)
    ctx.ttmc(t, bks.FREE3, torch.tensor(X, device=DEV), None, out, sym_half=True, prec=bks.F64)
    o1 = torch.empty((o.m, 12), dtype=dt, device=DEV)
    ctx.ttmc(t, bks.FREE1, torch.tensor(X, device=DEV), torch.tensor(Z, device=DEV), o1,
             prec=bks.F64)
    torch.cuda.synchronize()
    for got, want in ((out, ref.free3(o, X, sym_half=True)), (o1, ref.free1(o, X, Z))):
        got = got.cpu().numpy()
        assert np.linalg.norm(got - want) <= 1e-12 * np.linalg.norm(want)


@pytest.mark.parametrize("how,flag", [("frobenius", bks.SCALE_FROBENIUS),
                                      ("lambda_max", bks.SCALE_LAMBDA_MAX)])
def test_scaled_upload_matches_the_oracle(ctx, how, flag):
    c = reuters_like()
    t = ctx.upload_coo(c, flags=flag)
    o = preprocess.scale_slices(sptensor.from_coo(c.m, c.n, c.i, c.j, c.k, c.val), how)
    assert abs(t.frob - np.sqrt(sptensor.frob2(o))) <= 1e-12 * t.frob
    products_match(ctx, t, o)
    t.free()


def test_darpa_shaped_frobenius_scaling(ctx):
    """The DARPA-shaped stand-in's binary tensor scaled at upload equals the
    stand-in as generated (its generator scales the same way): every
    nonempty slice at norm 1."""
    raw = workloads.sparse_sym(8891, 371, 1_000_000, zipf=1.2, values="ones", seed=1012,
                               dtype=np.float64)
    t = ctx.upload_coo(raw, flags=bks.SCALE_FROBENIUS)
    nonempty = np.unique(raw.k).size
    assert abs(t.frob ** 2 - nonempty) <= 1e-9 * nonempty
    pre = ctx.upload_coo(workloads.p_darpa())
    assert abs(pre.frob - t.frob) <= 1e-6 * t.frob
    t.free()
    pre.free()


def test_bks_on_lambda_max_scaled_tensor(ctx):
    c = reuters_like(72)
    o = preprocess.scale_slices(sptensor.from_coo(c.m, c.n, c.i, c.j, c.k, c.val), "lambda_max")
    U0, W0 = workloads.random_start(c.m, c.n, 2, 2, 9)
    ref_res = obks.bks_solve(o, 2, 2, U0, W0, tol=1e-11, max_outer=300)
    t = ctx.upload_coo(c, flags=bks.SCALE_LAMBDA_MAX)
    U, W, F, info, rc = ctx.solve(t, 2, 2, U0=U0, W0=W0, precision=bks.PREC_FP64, tol=1e-11,
                                  max_outer=300)
    print(f"scaled solve: converged {info.converged} iters {info.outer_iters} "
          f"(oracle {ref_res['outer_iters']}) rel {info.rel_grad:.1e}")
    assert info.converged and ref_res["converged"]
    assert obks.subspace_distance(ref_res["U"], U) <= 1e-8
    assert obks.subspace_distance(ref_res["W"], W) <= 1e-8
    t.free()

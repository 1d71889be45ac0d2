"""Full-size BKS solves in the bench's configurations, checked by properties
that hold at any size, and at C2 also against the oracle's own solve (the
oracle cannot solve the C3 shape in test time).

C2-shaped planted tensor (20000 x 20000 x 2000, 2e6 stored; rank (5,5,5),
BKS(2,4)) and C3-shaped planted tensor (200000 x 200000 x 10000, 5e7 stored;
rank (10,10,10)), both from the bench's seeded start:
- the mixed-precision solve converges to a relative G-gradient <= 1e-11 and
  its U, W lie within a 1e-8 subspace angle of the plain FP64 GPU solve's
  (the precision target);
- the S-values (section "Conditioning of the best approximation problem") are the singular values of F_(1) and F_(3), so
  sum_i s_i^2 = ||F||^2 in both modes, and ||F|| <= ||A||;
- the planted core is recovered: ||F||^2 is at least the plant's energy,
  s_{r+1} is far below s_r, and the S-values of the planted components that
  stand above the noise are within 1% of the planted superdiagonal.  (At C3
  the heaviest Zipf rows carry ~1e7 |N(0,1)| entries each, noise directions
  of norm ~3.4e3: the planted 3500 is not separated from them and the 10th
  S-value is a mixture, ~3.7e3.)
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2012_07595_amd import bks, workloads

pytestmark = pytest.mark.gpu


def angle(Ua, Ub):
    Qa = np.linalg.qr(Ua)[0]
    Qb = np.linalg.qr(Ub)[0]
    return float(np.linalg.norm(Qb - Qa @ (Qa.T @ Qb), 2))


@pytest.fixture(scope="module")
def ctx():
    c = bks.Ctx(0)
    yield c
    c.close()


def solve_pair(ctx, coo, r):
    t = ctx.upload_coo(coo)
    U0, W0 = workloads.random_start(coo.m, coo.n, r, r, 2024)
    kw = dict(U0=U0, W0=W0, p=4, s=2, max_outer=200, tol=1e-11)
    U64, W64, F64, i64, rc64 = ctx.solve(t, r, r, precision=bks.PREC_FP64, **kw)
    U, W, F, info, rc = ctx.solve(t, r, r, precision=bks.PREC_MIXED, **kw)
    return t, (U64, W64, F64, i64, rc64), (U, W, F, info, rc)


def check_solve(t, ref, mix, r, core, n_clean):
    U64, W64, F64, i64, rc64 = ref
    U, W, F, info, rc = mix
    assert rc == 0 and info.converged and info.rel_grad <= 1e-11, (rc, info.rel_grad)
    assert rc64 == 0 and i64.converged, (rc64, i64.rel_grad)
    assert angle(U64, U) <= 1e-8 and angle(W64, W) <= 1e-8, (angle(U64, U), angle(W64, W))
    nF = float(np.linalg.norm(F))
    assert abs(nF - info.normF) <= 1e-12 * nF
    assert nF <= t.frob * (1 + 1e-12) and abs(info.normA - t.frob) <= 1e-12 * t.frob
    s1 = np.array(info.svals1[: r + 1])
    s3 = np.array(info.svals3[: r + 1])
    assert abs(np.sum(s1[:r] ** 2) - nF ** 2) <= 1e-10 * nF ** 2
    assert abs(np.sum(s3[:r] ** 2) - nF ** 2) <= 1e-10 * nF ** 2
    core = np.asarray(core)
    assert nF ** 2 >= (1 - 1e-3) * np.sum(core ** 2), (nF, np.sqrt(np.sum(core ** 2)))
    assert s1[r] <= 1e-2 * s1[r - 1] and s3[r] <= 1e-2 * s3[r - 1], (s1[r], s3[r])
    c = slice(0, n_clean)
    assert np.all(np.abs(s1[c] - core[c]) <= 1e-2 * core[c]), s1
    assert np.all(np.abs(s3[c] - core[c]) <= 1e-2 * core[c]), s3


def test_c2_planted_full(ctx):
    t, ref, mix = solve_pair(ctx, workloads.c2_planted(), 5)
    check_solve(t, ref, mix, 5, [3000.0, 2500.0, 2000.0, 1500.0, 1000.0], 5)


def test_c3_planted_full(ctx):
    print("[fullsize] generating the planted C3-shaped tensor (5e7 stored)", flush=True)
    t, ref, mix = solve_pair(ctx, workloads.c3_planted(), 10)
    check_solve(t, ref, mix, 10, [8000.0 - 500.0 * x for x in range(10)], 9)


def test_c2_planted_vs_oracle(ctx):
    """The bench's C2 solve itself against the oracle: the oracle's FP64 BKS
    solve of the whole C2-shaped planted tensor from the bench's start
    (BKS(2,4), tolerance 1e-11; about a minute of CPU time) and the
    mixed-precision GPU solve converge to U, W within a 1e-8 subspace angle
    and to the same ||F|| within 1e-10."""
    from oracle import bks as obks, sptensor
    coo = workloads.c2_planted()
    U0, W0 = workloads.random_start(coo.m, coo.n, 5, 5, 2024)
    t = ctx.upload_coo(coo)
    U, W, F, info, rc = ctx.solve(t, 5, 5, U0=U0, W0=W0, p=4, s=2, max_outer=200, tol=1e-11,
                                  precision=bks.PREC_MIXED)
    assert rc == 0 and info.converged, (rc, info.rel_grad)
    print("[fullsize] oracle FP64 BKS solve of the C2-shaped tensor", flush=True)
    T = sptensor.from_coo(coo.m, coo.n, coo.i, coo.j, coo.k, coo.val.astype(np.float64))
    ref = obks.bks_solve(T, 5, 5, U0, W0, p=4, s=2, tol=1e-11, max_outer=200)
    assert ref["converged"]
    a = max(obks.subspace_distance(ref["U"], U), obks.subspace_distance(ref["W"], W))
    nF, nref = float(np.linalg.norm(F)), float(np.linalg.norm(ref["F"]))
    print(f"[fullsize] C2 mixed vs oracle: outer {info.outer_iters} / {ref.get('outer_iters')}, "
          f"angle {a:.1e}, normF {nF:.12e} ref {nref:.12e}", flush=True)
    assert a <= 1e-8, a
    assert abs(nF - nref) <= 1e-10 * nref

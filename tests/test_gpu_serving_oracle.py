"""Served mixed-precision solves against the FP64 CPU oracle.

The C4-shaped serving trace (512 requests, the bench's trace: I, K, nnz
uniform on [1e3, 1e5], [100, 5000], [1e4, 5e6], Zipf(1.3), planted rank r
in {2, 3, 5, 8, 10}, seeded) is too large to check whole against the CPU
oracle; its 32 requests with at most 3e5 stored entries are submitted
together to a server (8 sessions, mixed precision, the bench's starts and
tolerance) and every result is compared with the oracle's FP64 BKS solve of
the same tensor and start: both converge, and U and W agree within a 1e-8
subspace angle (the precision target)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import bks as obks, sptensor
from paper_2012_07595_amd import bks, workloads

pytestmark = pytest.mark.gpu


def test_c4_small_requests_vs_oracle():
    reqs = [q for q in workloads.c4_requests(count=512, rate_per_s=1.0,
                                             nnz_range=(10_000, 5_000_000))
            if q.nnz <= 300_000]
    assert len(reqs) == 32
    coos = [workloads.request_tensor(q) for q in reqs]
    starts = [workloads.random_start(q.m, q.n, q.r, q.r, q.seed + 1) for q in reqs]
    ctx = bks.Ctx(0)
    srv = bks.Server(ctx, max_active=8, host_workers=8)
    ids = [srv.submit(None, q.r, q.r, precision=bks.PREC_MIXED, U0=U0, W0=W0, coo=coo,
                      tol=1e-11)
           for q, coo, (U0, W0) in zip(reqs, coos, starts)]
    got = []
    for rid in ids:
        U, W, F, res = srv.wait(rid)
        assert res.done and res.status == 0 and res.info.converged, res.status
        got.append((U, W))
    srv.close()
    ctx.close()
    worst = 0.0
    for q, coo, (U0, W0), (U, W) in zip(reqs, coos, starts, got):
        T = sptensor.from_coo(coo.m, coo.n, coo.i, coo.j, coo.k, coo.val.astype(np.float64))
        ref = obks.bks_solve(T, q.r, q.r, U0, W0, p=4, s=2, tol=1e-11)
        assert ref["converged"], q.rid
        a = max(obks.subspace_distance(ref["U"], U), obks.subspace_distance(ref["W"], W))
        print(f"[serving-oracle] request {q.rid} m={q.m} n={q.n} nnz={q.nnz} r={q.r} "
              f"angle {a:.1e}", flush=True)
        worst = max(worst, a)
        assert a <= 1e-8, (q.rid, a)
    print(f"[serving-oracle] largest angle {worst:.1e}", flush=True)


@pytest.mark.parametrize("precision", [bks.PREC_MIXED, bks.PREC_FP64])
def test_served_solves_on_dirty_memory(precision):
    """Four of those requests served (mixed precision, and plain FP64) by a
    new ctx after 4 GiB of device memory was filled with NaN and returned to
    the HIP runtime: the sessions' buffers are likely to land on NaN, and
    every result must still match the oracle."""
    reqs = sorted((q for q in workloads.c4_requests(count=512, rate_per_s=1.0,
                                                    nnz_range=(10_000, 5_000_000))
                   if q.nnz <= 300_000), key=lambda q: q.nnz)[:4]
    coos = [workloads.request_tensor(q) for q in reqs]
    starts = [workloads.random_start(q.m, q.n, q.r, q.r, q.seed + 1) for q in reqs]
    x = torch.full((1 << 29,), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    del x
    torch.cuda.empty_cache()
    ctx = bks.Ctx(0)
    srv = bks.Server(ctx, max_active=4, host_workers=4)
    try:
        ids = [srv.submit(None, q.r, q.r, precision=precision, U0=U0, W0=W0, coo=coo,
                          tol=1e-11)
               for q, coo, (U0, W0) in zip(reqs, coos, starts)]
        got = []
        for rid in ids:
            U, W, F, res = srv.wait(rid)
            assert res.done and res.status == 0 and res.info.converged, res.status
            got.append((U, W))
    finally:
        srv.close()
        ctx.close()
    for q, coo, (U0, W0), (U, W) in zip(reqs, coos, starts, got):
        assert np.all(np.isfinite(U)) and np.all(np.isfinite(W))
        T = sptensor.from_coo(coo.m, coo.n, coo.i, coo.j, coo.k, coo.val.astype(np.float64))
        ref = obks.bks_solve(T, q.r, q.r, U0, W0, p=4, s=2, tol=1e-11)
        a = max(obks.subspace_distance(ref["U"], U), obks.subspace_distance(ref["W"], W))
        print(f"[serving-dirty] precision {precision} request {q.rid} nnz={q.nnz} r={q.r} "
              f"angle {a:.1e}", flush=True)
        assert a <= 1e-8, (q.rid, a)

"""Serving: requests of different tensor sizes and ranks, submitted while
others run, are admitted by memory footprint and free slots; each result is
the same alone and in the mix (the kernels use fixed-order reductions, so
equality is exact); refusal of requests larger than the budget; latencies
are ordered submit <= start <= end."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import bks as obks
from paper_2012_07595_amd import bks, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = bks.Ctx(0)
    yield c
    c.close()


def requests():
    out = []
    specs = [(3000, 200, 60_000, 2), (5000, 300, 120_000, 3), (2000, 150, 40_000, 5),
             (8000, 400, 200_000, 2), (4000, 250, 80_000, 3), (2500, 120, 50_000, 2)]
    for q, (m, n, nnz, r) in enumerate(specs):
        base = workloads.sparse_sym(m, n, nnz, zipf=1.3, values="abs", seed=4000 + q)
        plant = workloads.planted(m, n, tuple(300.0 - 40 * x for x in range(r)), 12, 6, 5000 + q)
        coo = workloads.merge(base.astype(np.float64), plant).astype(np.float32)
        U0, W0 = workloads.random_start(m, n, r, r, 6000 + q)
        out.append((coo, r, U0, W0))
    return out


def test_alone_equals_mix(ctx):
    reqs = requests()
    solo = []
    tensors = []
    for coo, r, U0, W0 in reqs:
        t = ctx.upload_coo(coo)
        tensors.append(t)
        U, W, F, info, rc = ctx.solve(t, r, r, U0=U0, W0=W0, precision=bks.PREC_MIXED)
        assert info.converged
        solo.append((U, W, F))
    srv = bks.Server(ctx, max_active=3, host_workers=3)
    ids = []
    for q, (coo, r, U0, W0) in enumerate(reqs):
        if q % 2 == 0:
            ids.append(srv.submit(tensors[q], r, r, U0=U0, W0=W0))
        else:
            ids.append(srv.submit(None, r, r, U0=U0, W0=W0, coo=coo))
    overlap = False
    results = []
    for q, rid in enumerate(ids):
        U, W, F, res = srv.wait(rid)
        assert res.done and res.status == 0
        assert res.t_submit <= res.t_start <= res.t_end
        results.append(res)
        Us, Ws, Fs = solo[q]
        assert obks.subspace_distance(Us, U) <= 1e-12
        assert obks.subspace_distance(Ws, W) <= 1e-12
        assert np.array_equal(U, Us) and np.array_equal(W, Ws) and np.array_equal(F, Fs)
    starts = sorted((r.t_start, r.t_end) for r in results)
    for a, b in zip(starts, starts[1:]):
        if b[0] < a[1]:
            overlap = True
    assert overlap, "no two sessions ran at the same time"
    srv.close()


def test_budget_refusal_and_serialisation(ctx):
    coo, r, U0, W0 = requests()[0]
    t = ctx.upload_coo(coo)
    srv = bks.Server(ctx, max_active=2, mem_budget=1 << 20)
    with pytest.raises(bks.BksError) as e:
        srv.submit(t, r, r, U0=U0, W0=W0)
    assert e.value.code == bks.ENOMEM
    srv.close()
    # a budget that holds one session at a time serialises the two requests
    big = bks.Server(ctx, max_active=2, mem_budget=1 << 40)
    rid = big.submit(t, r, r, U0=U0, W0=W0)
    big.wait(rid)
    big.close()
    # the smallest power-of-two budget that admits the request holds less
    # than two of its footprints: two such requests run one after the other
    one = None
    for sh in range(21, 40):
        s = bks.Server(ctx, max_active=2, mem_budget=1 << sh)
        try:
            a = s.submit(t, r, r, U0=U0, W0=W0)
        except bks.BksError as e:
            assert e.code == bks.ENOMEM
            s.close()
            continue
        b = s.submit(t, r, r, U0=U0, W0=W0)
        ra = s.wait(a)[3]
        rb = s.wait(b)[3]
        one = (ra, rb)
        s.close()
        break
    assert one is not None
    ra, rb = one
    assert ra.status == 0 and rb.status == 0
    assert rb.t_start >= ra.t_end - 1e-6

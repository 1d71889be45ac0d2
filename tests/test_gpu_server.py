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


def slow_request(seed, m=5000, n=300, nnz=120_000, r=3):
    """An unplanted Zipf tensor: the gradient falls slowly, so a solve with a
    tolerance it cannot reach runs for many outer iterations."""
    coo = workloads.sparse_sym(m, n, nnz, zipf=1.3, values="abs", seed=seed).astype(np.float32)
    U0, W0 = workloads.random_start(m, n, r, r, seed + 1)
    return coo, r, U0, W0


def wait_started(srv, rid, timeout=60.0):
    import time
    t0 = time.time()
    while srv.poll(rid).t_start == 0.0:
        assert time.time() - t0 < timeout, "request never started"
        time.sleep(0.005)


def test_cancel_queued_and_running(ctx):
    import time
    # rank 10 on a 2e6-entry tensor: each outer iteration takes tens of ms,
    # and a tolerance of 1e-300 is never met
    coo, r, U0, W0 = slow_request(7100, m=20000, n=2000, nnz=2_000_000, r=10)
    t = ctx.upload_coo(coo)
    srv = bks.Server(ctx, max_active=1, host_workers=1)
    a = srv.submit(t, r, r, U0=U0, W0=W0, tol=1e-300, max_outer=2000)
    b = srv.submit(t, r, r, U0=U0, W0=W0)
    # b waits behind a (one slot): cancelled at once, never run
    assert srv.cancel(b) == bks.OK
    Ub, Wb, Fb, rb = srv.wait(b)
    assert rb.done and rb.status == bks.ECANCELED and rb.info.outer_iters == 0
    assert not Ub.any()
    # a is running: it stops at its next outer iteration with its iterate
    wait_started(srv, a)
    time.sleep(0.5)
    assert srv.cancel(a) == bks.OK
    Ua, Wa, Fa, ra = srv.wait(a)
    print(f"cancelled after {ra.info.outer_iters} outer iterations, "
          f"{ra.t_end - ra.t_start:.2f} s")
    assert ra.status == bks.ECANCELED
    assert 0 <= ra.info.outer_iters < 2000
    np.testing.assert_allclose(Ua.T @ Ua, np.eye(r), atol=1e-12)
    np.testing.assert_allclose(Wa.T @ Wa, np.eye(r), atol=1e-12)
    assert abs(np.sqrt(np.sum(Fa ** 2)) - ra.info.normF) <= 1e-10 * ra.info.normF
    # finished and unknown requests
    assert srv.cancel(a) == bks.EINVAL
    assert srv.cancel(123456789) == bks.ENOTFOUND
    # the slot is free again and serves the next request normally
    coo2, r2, U02, W02 = requests()[2]
    t2 = ctx.upload_coo(coo2)
    c = srv.submit(t2, r2, r2, U0=U02, W0=W02)
    assert srv.wait(c)[3].status == 0
    srv.close()


def test_head_of_line_request_is_passed_over(ctx):
    """With a budget that cannot hold the running request and the large one
    behind it together, a small request queued after the large one is
    admitted first; the large one starts once the running one ends."""
    import time
    slow = slow_request(7200)
    big = slow_request(7300, m=20000, n=1500, nnz=400_000, r=5)
    small = requests()[2]
    probe = bks.Server(ctx, max_active=1)
    fp = []
    for coo, r, U0, W0 in (slow, big, small):
        rid = probe.submit(None, r, r, U0=U0, W0=W0, coo=coo, max_outer=1)
        fp.append(probe.wait(rid)[3].footprint)
    probe.close()
    fa, fb, fc = fp
    # the first and the small request fit together, the first and the large
    # one do not
    assert fc < fb
    srv = bks.Server(ctx, max_active=2, mem_budget=fa + fb - 1)
    coo, r, U0, W0 = slow
    a = srv.submit(None, r, r, U0=U0, W0=W0, coo=coo, tol=1e-300, max_outer=150)
    wait_started(srv, a)
    coo, r, U0, W0 = big
    b = srv.submit(None, r, r, U0=U0, W0=W0, coo=coo, max_outer=2)
    coo, r, U0, W0 = small
    c = srv.submit(None, r, r, U0=U0, W0=W0, coo=coo)
    rc_ = srv.wait(c)[3]
    ra = srv.wait(a)[3]
    rb = srv.wait(b)[3]
    assert rc_.status == 0 and ra.status in (0, bks.ENOTCONV) and rb.status in (0, bks.ENOTCONV)
    assert rc_.t_start < ra.t_end, "the small request waited behind the large one"
    assert rb.t_start >= ra.t_end - 1e-6, "the large request ran beside the first"
    srv.close()


def test_device_bytes_within_footprint(ctx):
    """The device bytes a served session holds (library buffers, tensor
    formats of server-side uploads included) never exceed the footprint it
    was admitted with, also for a rank-10 solve whose core product keeps
    one 190 x 190 partial per slice chunk over 5000 slices (> 512 MB)."""
    reqs = requests()[:4]
    wide = workloads.sparse_sym(3000, 5000, 300_000, zipf=1.3, values="abs",
                                seed=7400).astype(np.float32)
    srv = bks.Server(ctx, max_active=2, host_workers=2)
    ids = []
    tensors = []  # uploaded tensors must outlive their requests
    for q, (coo, r, U0, W0) in enumerate(reqs):
        if q % 2:
            ids.append(srv.submit(None, r, r, U0=U0, W0=W0, coo=coo))
        else:
            tensors.append(ctx.upload_coo(coo))
            ids.append(srv.submit(tensors[-1], r, r, U0=U0, W0=W0))
    U0, W0 = workloads.random_start(wide.m, wide.n, 10, 10, 7401)
    ids.append(srv.submit(None, 10, 10, U0=U0, W0=W0, coo=wide, max_outer=1))
    for rid in ids:
        res = srv.wait(rid)[3]
        assert res.status in (0, bks.ENOTCONV), (res.status, res.error)
        print(f"footprint {res.footprint / 2**20:.1f} MiB peak {res.dev_peak / 2**20:.1f} MiB")
        assert 0 < res.dev_peak <= res.footprint
    srv.close()

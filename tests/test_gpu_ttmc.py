"""GPU parity of bks_ttmc against the FP64 oracle (section "Multilinear tensor-matrix multiplication" products).

Tolerances (normwise, per call): FP32 ||T_gpu - T_ref||_F <= 1e-5 ||T_ref||_F
plus row-wise 1e-5 on rows with ||row_ref|| >= 1e-3 max_row, where a row that
is cancellation-dominated may instead sit within the FP32 accumulation bound
of parity_bounds; FP64 and FP32-values/FP64-accumulation 1e-12 (normwise and
row-wise).  The reference is the oracle in FP64 on
the very inputs the kernel sees (FP32 factors and values promoted exactly)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import sptensor, ttmc as ref
from paper_2012_07595_amd import bks, workloads

import parity_bounds as pb

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def ctx():
    c = bks.Ctx(0)
    yield c
    c.close()


def oracle_tensor(coo):
    return sptensor.from_coo(coo.m, coo.n, coo.i, coo.j, coo.k, coo.val.astype(np.float64))


def run(ctx, t, op, B1, B2, rows, q, prec, sym=False):
    dt = torch.float32 if prec == bks.F32 else torch.float64
    b1 = torch.tensor(B1, dtype=dt, device=DEV) if B1 is not None else None
    b2 = torch.tensor(B2, dtype=dt, device=DEV) if B2 is not None else None
    out = torch.full((rows, q), float("nan"), dtype=dt, device=DEV)
    ctx.ttmc(t, op, b1, b2, out, sym_half=sym, prec=prec)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


def absprod(o, op, B1, B2=None, sym=False):
    """(the product with |A|, |B1|, |B2|, terms per output element) for the
    cancellation allowance of parity_bounds."""
    a = pb.abs_tensor(o)
    if op == "free3":
        w = ref.free3(a, np.abs(B1), None if B2 is None else np.abs(B2), sym_half=sym)
    elif op == "free1":
        w = ref.free1(a, np.abs(B1), np.abs(B2))
    else:
        w = ref.mode3(a, np.abs(B2))[2]
    return w, pb.max_terms(o, op)


def check(got, want, prec, absw=None, L=1):
    """absw: the same product with |A|, |B1|, |B2|; L: terms per output
    element (parity_bounds; the unit roundoff is that of the accumulation)."""
    if isinstance(absw, tuple):
        absw, L = absw
    assert np.all(np.isfinite(got)), "unwritten output rows"
    tol = 1e-5 if prec == bks.F32 else 1e-12
    nw = np.linalg.norm(want)
    if nw == 0:
        assert np.abs(got).max() == 0
        return
    assert np.linalg.norm(got - want) <= tol * nw, np.linalg.norm(got - want) / nw
    if absw is None:
        absw = np.zeros_like(want)
    ratio = pb.rows_ok(got, want, absw, L, tol, pb.U32 if prec == bks.F32 else pb.U64)
    assert ratio <= 1.0, ratio


def factors(rows, p, seed, prec):
    X = workloads.random_block(rows, p, seed)
    if prec == bks.F32:
        X = X.astype(np.float32).astype(np.float64)
    return X


CASES = [
    # m, n, nnz, zipf, values
    (3000, 200, 60_000, 0.0, "normal"),
    (4000, 7, 50_000, 1.5, "abs"),        # few long slices: split segments
    (2500, 300, 40_000, 1.3, "normal"),
]
PRECS = [bks.F32, bks.F64, bks.F32IN_F64ACC]


@pytest.fixture(scope="module")
def tensors(ctx):
    out = []
    for (m, n, nnz, z, v) in CASES:
        dt = np.float64
        coo = workloads.sparse_sym(m, n, nnz, zipf=z, values=v, seed=m + n, dtype=dt)
        c32 = coo.astype(np.float32)
        out.append((ctx.upload_coo(coo), ctx.upload_coo(c32), oracle_tensor(coo),
                    oracle_tensor(c32)))
    return out


def pick(tensors, idx, prec):
    t64, t32, o64, o32 = tensors[idx]
    # F64 reads the FP64 values; F32 paths read the FP32 copy
    return (t64, o64) if prec == bks.F64 else (t32, o32)


@pytest.mark.parametrize("idx", range(len(CASES)))
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("px,py", [(1, 1), (2, 3), (4, 4), (5, 5), (5, 4), (7, 3), (10, 10), (20, 20)])
def test_free3_rect(ctx, tensors, idx, prec, px, py):
    t, o = pick(tensors, idx, prec)
    X = factors(o.m, px, 11, prec)
    Y = factors(o.m, py, 12, prec)
    got = run(ctx, t, bks.FREE3, X, Y, o.n, px * py, prec)
    check(got, ref.free3(o, X, Y), prec, absprod(o, "free3", X, Y))


@pytest.mark.parametrize("idx", range(len(CASES)))
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 8, 10, 20, 23, 24, 25, 40, 70, 130, 193, 260])
def test_free3_sym(ctx, tensors, idx, prec, p):
    t, o = pick(tensors, idx, prec)
    X = factors(o.m, p, 13, prec)
    got = run(ctx, t, bks.FREE3, X, None, o.n, p * (p + 1) // 2, prec, sym=True)
    check(got, ref.free3(o, X, sym_half=True), prec, absprod(o, "free3", X, sym=True))


@pytest.fixture(scope="module")
def many_slices(ctx):
    """1200 slices (enough for the one-workgroup-per-slice form of the core
    product), every seventh of them empty."""
    c = workloads.sparse_sym(3000, 1200, 36_000, zipf=0.8, values="normal", seed=77,
                             dtype=np.float64)
    keep = c.k % 7 != 3
    c = workloads.SymCOO(c.m, c.n, c.i[keep], c.j[keep], c.k[keep], c.val[keep])
    c32 = c.astype(np.float32)
    return ctx.upload_coo(c), ctx.upload_coo(c32), oracle_tensor(c), oracle_tensor(c32)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("p", [25, 40, 70, 96, 97])
def test_free3_sym_many_slices(ctx, many_slices, prec, p):
    """Widths up to 96 write each slice's row from one workgroup (FP32),
    97 takes the chunked form; empty slices give zero rows."""
    t64, t32, o64, o32 = many_slices
    t, o = (t64, o64) if prec == bks.F64 else (t32, o32)
    X = factors(o.m, p, 15, prec)
    got = run(ctx, t, bks.FREE3, X, None, o.n, p * (p + 1) // 2, prec, sym=True)
    assert np.all(got[3::7] == 0.0)
    check(got, ref.free3(o, X, sym_half=True), prec, absprod(o, "free3", X, sym=True))


@pytest.mark.parametrize("prec", PRECS)
def test_free3_sym_580(ctx, tensors, prec):
    """The core product's width at rank 20 (k1 = 580: 37 output tiles per
    side, cut into blocks of workgroups on the matrix cores in FP32) on the
    tensor with seven long slices."""
    t, o = pick(tensors, 1, prec)
    X = factors(o.m, 580, 14, prec)
    got = run(ctx, t, bks.FREE3, X, None, o.n, 580 * 581 // 2, prec, sym=True)
    check(got, ref.free3(o, X, sym_half=True), prec, absprod(o, "free3", X, sym=True))


@pytest.mark.parametrize("idx", range(len(CASES)))
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("py,pz", [(1, 1), (2, 2), (3, 4), (5, 5), (4, 5), (8, 8), (10, 10), (20, 20)])
def test_free1(ctx, tensors, idx, prec, py, pz):
    t, o = pick(tensors, idx, prec)
    Y = factors(o.m, py, 14, prec)
    Z = factors(o.n, pz, 15, prec)
    got = run(ctx, t, bks.FREE1, Y, Z, o.m, py * pz, prec)
    check(got, ref.free1(o, Y, Z), prec, absprod(o, "free1", Y, Z))


@pytest.mark.parametrize("idx", range(len(CASES)))
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("pz", [1, 3, 5, 10, 20])
def test_mode3(ctx, tensors, idx, prec, pz):
    t, o = pick(tensors, idx, prec)
    Z = factors(o.n, pz, 16, prec)
    pi, pj = t.pairs()
    ri, rj, want = ref.mode3(o, Z)
    np.testing.assert_array_equal(pi, ri)
    np.testing.assert_array_equal(pj, rj)
    got = run(ctx, t, bks.MODE3, None, Z, t.npairs, pz, prec)
    check(got, want, prec, absprod(o, "mode3", None, Z))


def test_products_on_dirty_memory():
    """Every product kind in a new ctx after 4 GiB of device memory was
    filled with NaN and handed back, so that the ctx's formats, schedules
    and workspaces are likely to land on NaN: a read of a workspace entry
    that the launch did not write shows up as a wrong or non-finite row (a
    freshly mapped allocation reads as zeros and would hide it)."""
    m, n, nnz, z, v = CASES[2]
    coo = workloads.sparse_sym(m, n, nnz, zipf=z, values=v, seed=m + n, dtype=np.float64)
    x = torch.full((1 << 29,), float("nan"), dtype=torch.float64, device=DEV)
    torch.cuda.synchronize()
    del x
    torch.cuda.empty_cache()
    c = bks.Ctx(0)
    try:
        for prec in PRECS:
            cc = coo if prec == bks.F64 else coo.astype(np.float32)
            t, o = c.upload_coo(cc), oracle_tensor(cc)
            for p in (5, 70, 130):
                X = factors(o.m, p, 13, prec)
                got = run(c, t, bks.FREE3, X, None, o.n, p * (p + 1) // 2, prec, sym=True)
                check(got, ref.free3(o, X, sym_half=True), prec, absprod(o, "free3", X, sym=True))
            X, Y = factors(o.m, 5, 11, prec), factors(o.m, 4, 12, prec)
            check(run(c, t, bks.FREE3, X, Y, o.n, 20, prec), ref.free3(o, X, Y), prec,
                  absprod(o, "free3", X, Y))
            Y, Z = factors(o.m, 4, 14, prec), factors(o.n, 5, 15, prec)
            check(run(c, t, bks.FREE1, Y, Z, o.m, 20, prec), ref.free1(o, Y, Z), prec,
                  absprod(o, "free1", Y, Z))
            Z = factors(o.n, 5, 16, prec)
            check(run(c, t, bks.MODE3, None, Z, t.npairs, 5, prec), ref.mode3(o, Z)[2], prec,
                  absprod(o, "mode3", None, Z))
            t.free()
    finally:
        c.close()


def test_deterministic(ctx, tensors):
    t, o = pick(tensors, 1, bks.F32)
    X = factors(o.m, 5, 1, bks.F32)
    a = run(ctx, t, bks.FREE3, X, None, o.n, 15, bks.F32, sym=True)
    b = run(ctx, t, bks.FREE3, X, None, o.n, 15, bks.F32, sym=True)
    assert np.array_equal(a, b)
    Z = factors(o.n, 5, 2, bks.F32)
    a = run(ctx, t, bks.FREE1, X, Z, o.m, 25, bks.F32)
    b = run(ctx, t, bks.FREE1, X, Z, o.m, 25, bks.F32)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("kind", ["empty", "single", "diagonal", "heavy_row", "ragged"])
def test_edge_cases(ctx, kind):
    rng = np.random.default_rng(5)
    if kind == "empty":
        m, n = 10, 4
        i = j = k = np.zeros(0, np.int32)
        v = np.zeros(0)
    elif kind == "single":
        m, n = 7, 3
        i, j, k, v = np.array([2]), np.array([5]), np.array([1]), np.array([1.5])
    elif kind == "diagonal":
        m, n = 50, 6
        i = j = rng.integers(0, m, 200)
        k = rng.integers(0, n, 200)
        key = np.unique(k * m + i)
        i = j = key % m
        k = key // m
        v = rng.standard_normal(i.shape[0])
    elif kind == "heavy_row":
        # one row holds more than 40% of the stored entries
        m, n = 5000, 50
        cnt = 30000
        i = np.full(cnt, 17)
        j = rng.integers(0, m, cnt)
        k = rng.integers(0, n, cnt)
        c2 = workloads.sparse_sym(m, n, 20000, seed=3, dtype=np.float64)
        i = np.concatenate([i, c2.i]); j = np.concatenate([j, c2.j]); k = np.concatenate([k, c2.k])
        v = rng.standard_normal(i.shape[0])
    else:
        m, n = 1031, 17  # not a multiple of any tile
        c = workloads.sparse_sym(m, n, 9000, zipf=1.1, seed=8, dtype=np.float64)
        i, j, k, v = c.i, c.j, c.k, c.val
    t = ctx.upload(m, n, i, j, k, np.asarray(v, np.float64), flags=bks.SUM_DUPLICATES)
    o = sptensor.from_coo(m, n, i, j, k, v)
    for prec in (bks.F32, bks.F64):
        X = factors(m, 3, 1, prec)
        Z = factors(n, 2, 2, prec)
        check(run(ctx, t, bks.FREE3, X, None, n, 6, prec, sym=True), ref.free3(o, X, sym_half=True), prec,
              absprod(o, "free3", X, sym=True))
        check(run(ctx, t, bks.FREE3, X, X[:, :2], n, 6, prec), ref.free3(o, X, X[:, :2]), prec,
              absprod(o, "free3", X, X[:, :2]))
        check(run(ctx, t, bks.FREE1, X, Z, m, 6, prec), ref.free1(o, X, Z), prec,
              absprod(o, "free1", X, Z))
        if t.npairs:
            check(run(ctx, t, bks.MODE3, None, Z, t.npairs, 2, prec), ref.mode3(o, Z)[2], prec,
                  absprod(o, "mode3", None, Z))
    assert abs(t.frob - np.sqrt(sptensor.frob2(o))) <= 1e-12 * max(1.0, t.frob)


def test_upload_from_device_arrays(ctx):
    """Coordinates and values given as device arrays (BKS_DEVICE_PTRS) build
    the same tensor as the host upload: same sizes, norm and pair pattern,
    and bitwise the same products for every op and precision."""
    c = workloads.sparse_sym(1031, 17, 9000, zipf=1.1, seed=8, dtype=np.float64)
    th = ctx.upload_coo(c)
    dev = [torch.tensor(a, dtype=torch.int32, device=DEV) for a in (c.i, c.j, c.k)]
    v = torch.tensor(c.val, dtype=torch.float64, device=DEV)
    torch.cuda.synchronize()
    td = ctx.upload(c.m, c.n, *dev, v)
    assert (td.nnz, td.npairs, td.frob) == (th.nnz, th.npairs, th.frob)
    for a, b in zip(td.pairs(), th.pairs()):
        np.testing.assert_array_equal(a, b)
    for prec in PRECS:
        X = factors(c.m, 4, 1, prec)
        Z = factors(c.n, 3, 2, prec)
        got = [(run(ctx, t_, bks.FREE3, X, None, c.n, 10, prec, sym=True),
                run(ctx, t_, bks.FREE1, X, Z, c.m, 12, prec),
                run(ctx, t_, bks.MODE3, None, Z, t_.npairs, 3, prec)) for t_ in (td, th)]
        for a, b in zip(*got):
            np.testing.assert_array_equal(a, b)
    with pytest.raises(ValueError):
        ctx.upload(c.m, c.n, dev[0].to(torch.int64), dev[1], dev[2], v)
    td.free()
    th.free()


def test_upload_errors(ctx):
    with pytest.raises(bks.BksError) as e:
        ctx.upload(5, 2, [0], [5], [0], np.array([1.0]))
    assert e.value.code == bks.EINDEX
    with pytest.raises(bks.BksError) as e:
        ctx.upload(5, 2, [0], [1], [0], np.array([np.inf]))
    assert e.value.code == bks.EVALUE
    with pytest.raises(bks.BksError) as e:
        ctx.upload(5, 2, [0, 1], [1, 0], [0, 0], np.array([1.0, 2.0]))
    assert e.value.code == bks.EDUP
    with pytest.raises(bks.BksError) as e:
        ctx.upload(5, 2, [0, 1], [1, 0], [0, 0], np.array([1.0, 2.0]), flags=bks.FULL_SYMMETRIC)
    assert e.value.code == bks.EASYM
    t = ctx.upload(5, 2, [0, 1, 3], [1, 0, 3], [0, 0, 1], np.array([1.0, 1.0, 2.0]),
                   flags=bks.FULL_SYMMETRIC)
    assert t.nnz == 2


def test_allocation_failure_is_reported(ctx, monkeypatch):
    # a device allocation forced to fail (BKS_FAIL_NEXT_ALLOC) comes back as
    # BKS_ENOMEM with a message, leaves nothing behind, and the ctx stays usable
    coo = workloads.sparse_sym(300, 20, 3000, seed=5, dtype=np.float32)
    monkeypatch.setenv("BKS_FAIL_NEXT_ALLOC", "1")
    with pytest.raises(bks.BksError) as e:
        ctx.upload_coo(coo)
    assert e.value.code == bks.ENOMEM
    assert "allocation" in str(e.value)
    monkeypatch.delenv("BKS_FAIL_NEXT_ALLOC", raising=False)
    t = ctx.upload_coo(coo)
    o = oracle_tensor(coo)
    X = factors(coo.m, 3, 7, bks.F32)
    check(run(ctx, t, bks.FREE3, X, None, coo.n, 6, bks.F32, sym=True),
          ref.free3(o, X, sym_half=True), bks.F32, absprod(o, "free3", X, sym=True))

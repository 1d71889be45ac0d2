"""GPU parity at the full workload sizes, on sampled outputs.

The C2-shaped planted tensor (20000 x 20000 x 2000, 2e6 stored), the
C3-shaped one (200000 x 200000 x 10000, 5e7 stored, the product sweep's) and
the C5-shaped one (1e6 x 1e6 x 500, 2e8 stored, power-law degrees) are
uploaded whole, and every product runs over the whole tensor in the launch
configuration the bench and the solver use: narrow widths 5, 10, 20, the
core product at k1 = 70 (C2), k1 = 190 (C3) and k1 = 580 (C5) on the matrix
cores, FP32 and FP64 accumulation.  The FP64 oracle then recomputes a
sample of output rows from exactly the entries those rows depend on (the
definitions of section "Multilinear tensor-matrix multiplication"): a FREE3 row k from slice k, a FREE1 row r from the entries
in row or column r, a MODE3 row from the entries of its stored pair.  The
samples include the longest slice, the heaviest row and the row of degree
rank 30, the row of degree rank 300 (split segments and
the fixed-order reduction tree; the heaviest row of the C3 law holds about
1e7 entries) and an empty row where one exists.

Tolerances as for the small cases: FP32 normwise 1e-5 over the sampled rows
plus row-wise 1e-5 on rows with norm >= 1e-3 of the largest, or, for a
cancellation-dominated row, the accumulation bound of parity_bounds; FP64
accumulation 1e-12."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import sptensor, ttmc as ref
from paper_2012_07595_amd import bks, workloads

import parity_bounds as pb

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def check_rows(got, want, prec, what, absw, L):
    """absw: the sampled rows of the product with |A| and |factors|; L: terms
    per output element (parity_bounds)."""
    assert np.all(np.isfinite(got)), f"{what}: unwritten output rows"
    tol = 1e-5 if prec == bks.F32 else 1e-12
    nw = np.linalg.norm(want)
    if nw == 0:
        assert np.abs(got).max() == 0, what
        return
    err = np.linalg.norm(got - want) / nw
    assert err <= tol, (what, err)
    ratio = pb.rows_ok(got, want, absw, L, tol, pb.U32 if prec == bks.F32 else pb.U64)
    assert ratio <= 1.0, (what, ratio)


def sub_tensor(coo, mask, k_map=None):
    """Oracle tensor of the selected stored entries (FP32 values promoted
    exactly); k_map renumbers the slices (FREE3 rows are per slice)."""
    k = coo.k[mask] if k_map is None else k_map[coo.k[mask]]
    n = coo.n if k_map is None else int(k_map.max()) + 1
    return sptensor.from_coo(coo.m, n, coo.i[mask], coo.j[mask], k,
                             coo.val[mask].astype(np.float64))


class Full:
    def __init__(self, ctx, coo, seed, nslices=10):
        self.coo = coo
        self.t = ctx.upload_coo(coo)
        rng = np.random.default_rng(seed)
        slen = np.bincount(coo.k, minlength=coo.n)
        nonempty = np.flatnonzero(slen)
        self.slices = np.unique(np.concatenate(
            [[int(np.argmax(slen))], rng.choice(nonempty, nslices - 1, replace=False)]))
        deg = np.bincount(np.concatenate([coo.i, coo.j]), minlength=coo.m)
        used = np.flatnonzero(deg)
        # heavy rows of degree rank 0, 30 and 300 (split into many chunks,
        # summed through the reduction tree) and random used rows
        by_deg = np.argsort(deg, kind="stable")[::-1]
        rows = [int(by_deg[300])] + list(rng.choice(used, 8, replace=False))
        empty = np.flatnonzero(deg == 0)
        if empty.size:
            rows.append(int(empty[0]))
        self.rows = np.unique(np.array(rows))
        self.rows_heavy = np.unique(np.append(self.rows, [int(by_deg[30]), int(by_deg[0])]))
        pi, pj = self.t.pairs()
        self.pairs = np.unique(rng.choice(pi.shape[0], 16, replace=False))
        self.pi, self.pj = pi, pj


def factor(rows, p, seed):
    return workloads.random_block(rows, p, seed).astype(np.float32).astype(np.float64)


def gpu(ctx, t, op, B1, B2, rows, q, prec, sym=False):
    dt = torch.float32 if prec == bks.F32 else torch.float64
    b1 = torch.tensor(B1, dtype=dt, device=DEV) if B1 is not None else None
    b2 = torch.tensor(B2, dtype=dt, device=DEV) if B2 is not None else None
    out = torch.full((rows, q), float("nan"), dtype=dt, device=DEV)
    ctx.ttmc(t, op, b1, b2, out, sym_half=sym, prec=prec)
    torch.cuda.synchronize()
    return out


def free3_sampled(ctx, F, px, py, prec, sym, seed):
    coo, t = F.coo, F.t
    X = factor(coo.m, px, seed)
    Y = None if sym else factor(coo.m, py, seed + 1)
    q = px * (px + 1) // 2 if sym else px * py
    out = gpu(ctx, t, bks.FREE3, X, Y, coo.n, q, prec, sym)
    got = out[torch.as_tensor(F.slices, device=DEV)].cpu().numpy().astype(np.float64)
    assert bool(torch.isfinite(out).all()), "unwritten FREE3 rows"
    del out
    k_map = np.full(coo.n, -1, np.int64)
    k_map[F.slices] = np.arange(F.slices.size)
    T = sub_tensor(coo, np.isin(coo.k, F.slices), k_map)
    print(f"[fullsize] FREE3 p=({px},{py}) sym={sym}: oracle slices over {T.i.size} stored "
          f"entries", flush=True)
    want = ref.free3(T, X, Y, sym_half=sym)
    absw = ref.free3(pb.abs_tensor(T), np.abs(X), None if Y is None else np.abs(Y), sym_half=sym)
    check_rows(got, want, prec, f"FREE3 sym={sym} p=({px},{py})", absw, pb.max_terms(T, "free3"))


def free1_sampled(ctx, F, py, pz, prec, seed, heavy=True):
    coo, t = F.coo, F.t
    rows = F.rows_heavy if heavy else F.rows
    Y = factor(coo.m, py, seed)
    Z = factor(coo.n, pz, seed + 1)
    out = gpu(ctx, t, bks.FREE1, Y, Z, coo.m, py * pz, prec)
    assert bool(torch.isfinite(out).all()), "unwritten FREE1 rows"
    got = out[torch.as_tensor(rows, device=DEV)].cpu().numpy().astype(np.float64)
    del out
    T = sub_tensor(coo, np.isin(coo.i, rows) | np.isin(coo.j, rows))
    print(f"[fullsize] FREE1 p=({py},{pz}): oracle rows over {T.i.size} stored entries", flush=True)
    want = ref.free1_rows(T, Y, Z, rows)
    absw = ref.free1_rows(pb.abs_tensor(T), np.abs(Y), np.abs(Z), rows)
    check_rows(got, want, prec, f"FREE1 p=({py},{pz})", absw, pb.max_terms(T, "free1"))


def mode3_sampled(ctx, F, pz, prec, seed):
    coo, t = F.coo, F.t
    Z = factor(coo.n, pz, seed)
    out = gpu(ctx, t, bks.MODE3, None, Z, t.npairs, pz, prec)
    assert bool(torch.isfinite(out).all()), "unwritten MODE3 rows"
    got = out[torch.as_tensor(F.pairs, device=DEV)].cpu().numpy().astype(np.float64)
    del out
    key = coo.i.astype(np.int64) * coo.m + coo.j
    want_keys = F.pi[F.pairs].astype(np.int64) * coo.m + F.pj[F.pairs]
    T = sub_tensor(coo, np.isin(key, want_keys))
    pi, pj, tt = ref.mode3(T, Z)
    ta = ref.mode3(pb.abs_tensor(T), np.abs(Z))[2]
    pos = {(int(a), int(b)): x for x, (a, b) in enumerate(zip(pi, pj))}
    sel = [pos[(int(F.pi[x]), int(F.pj[x]))] for x in F.pairs]
    check_rows(got, tt[sel], prec, f"MODE3 p={pz}", ta[sel], pb.max_terms(T, "mode3"))


@pytest.fixture(scope="module")
def ctx():
    c = bks.Ctx(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def c2(ctx):
    return Full(ctx, workloads.c2_planted(), 21)


@pytest.fixture(scope="module")
def c3(ctx):
    print("[fullsize] generating the C3-shaped tensor (5e7 stored)", flush=True)
    return Full(ctx, workloads.c3(), 31)


@pytest.fixture(scope="module")
def c5(ctx):
    print("[fullsize] generating the C5-shaped tensor (2e8 stored, Chung-Lu law)", flush=True)
    # C5 slices hold ~4e5 entries each: two sampled slices (the longest and
    # one more) keep the oracle's k1 = 580 products to seconds
    return Full(ctx, workloads.c5(), 51, nslices=2)


@pytest.mark.parametrize("prec", [bks.F32, bks.F64])
def test_c2_core_product(ctx, c2, prec):
    # the solver's core product at k1 = 70 (matrix cores in FP32)
    free3_sampled(ctx, c2, 70, 70, prec, True, 100)


@pytest.mark.parametrize("prec", [bks.F32, bks.F64])
def test_c2_narrow(ctx, c2, prec):
    free3_sampled(ctx, c2, 5, 5, prec, True, 110)
    free3_sampled(ctx, c2, 5, 4, prec, False, 120)
    free1_sampled(ctx, c2, 5, 5, prec, 130)
    mode3_sampled(ctx, c2, 5, prec, 140)


@pytest.mark.parametrize("p", [5, 10, 20])
def test_c3_sweep(ctx, c3, p):
    free3_sampled(ctx, c3, p, p, bks.F32, True, 200 + p)
    free3_sampled(ctx, c3, p, p, bks.F32, False, 300 + p)
    free1_sampled(ctx, c3, p, p, bks.F32, 400 + p)
    mode3_sampled(ctx, c3, p, bks.F32, 500 + p)


def test_c3_core_product(ctx, c3):
    # the rank-(10,10,10) solve's core product at k1 = 190
    free3_sampled(ctx, c3, 190, 190, bks.F32, True, 600)


def test_c5_core_product(ctx, c5):
    # the rank-(20,20,20) solve's core product at k1 = 580: 37 output tiles
    # per side, split over workgroups on the matrix cores
    free3_sampled(ctx, c5, 580, 580, bks.F32, True, 700)


def test_c5_narrow(ctx, c5):
    free3_sampled(ctx, c5, 20, 20, bks.F32, True, 710)
    free3_sampled(ctx, c5, 5, 4, bks.F32, False, 715)
    # the heaviest rows hold up to ~3e7 entries
    free1_sampled(ctx, c5, 5, 5, bks.F32, 720)
    free1_sampled(ctx, c5, 20, 20, bks.F32, 730)
    mode3_sampled(ctx, c5, 20, bks.F32, 740)


def test_c5_solve_two_restarts(ctx, c5):
    """The rank-(20,20,20) BKS(2,4) solve of the C5-shaped tensor (k1 = 580,
    k3 = 310, Newton systems of order 17000 on the device), two restarts
    from the bench's start in plain FP64 and in mixed precision.  The S-value
    gaps of this tensor at rank 20 are ~1e-4 of s_1 and below, so the
    subspaces are not determined well enough for an angle bar (parity
    unpinned: the angle and the ||F|| difference between the precisions are
    printed); what holds at any iterate is checked in both: sum s_i^2 =
    ||F||^2 in modes 1 and 3, ||F|| <= ||A|| and ||F|| non-decreasing."""
    t = c5.t
    U0, W0 = workloads.random_start(c5.coo.m, c5.coo.n, 20, 20, 2024)
    kw = dict(U0=U0, W0=W0, p=4, s=2, max_outer=2, tol=1e-11)
    out = {}
    for name, prec in (("fp64", bks.PREC_FP64), ("mixed", bks.PREC_MIXED)):
        print(f"[fullsize] C5 {name} solve, two restarts", flush=True)
        U, W, F, info, rc = ctx.solve(t, 20, 20, precision=prec, **kw)
        # two restarts end short of the tolerance: BKS_ENOTCONV, results written
        assert rc in (0, bks.ENOTCONV) and info.outer_iters == 2
        assert info.k1 == 580 and info.k3 == 310
        nF = float(np.linalg.norm(F))
        assert abs(nF - info.normF) <= 1e-12 * nF
        assert nF <= t.frob * (1 + 1e-12)
        s1 = np.array(info.svals1[:21])
        s3 = np.array(info.svals3[:21])
        assert abs(np.sum(s1[:20] ** 2) - nF ** 2) <= 1e-10 * nF ** 2
        assert abs(np.sum(s3[:20] ** 2) - nF ** 2) <= 1e-10 * nF ** 2
        h = np.array(info.normF_hist[:info.n_hist])
        assert np.all(h[1:] >= h[:-1] * (1 - (1e-12 if prec == bks.PREC_FP64 else 1e-5)))
        g1 = (s1[19] - s1[20]) / s1[0]
        g3 = (s3[19] - s3[20]) / s3[0]
        print(f"[fullsize] C5 {name}: |F| {nF:.12g} rel grad {info.rel_grad:.3e} gaps "
              f"{g1:.2e} {g3:.2e}", flush=True)
        out[name] = (U, W, nF)
    a = max(obks_distance(out["fp64"][0], out["mixed"][0]),
            obks_distance(out["fp64"][1], out["mixed"][1]))
    d = abs(out["mixed"][2] - out["fp64"][2]) / out["fp64"][2]
    print(f"[fullsize] C5 mixed vs FP64 after two restarts: angle {a:.1e}, |F| differs by "
          f"{d:.1e} relative (parity unpinned: gaps below 1e-3)", flush=True)


def obks_distance(Ua, Ub):
    from oracle import bks as obks
    return obks.subspace_distance(Ua, Ub)

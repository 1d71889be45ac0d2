"""GPU parity at the full workload sizes, on sampled outputs.

The C2-shaped planted tensor (20000 x 20000 x 2000, 2e6 stored, the bench's
default workload) and the C3-shaped one (200000 x 200000 x 10000, 5e7 stored,
the product sweep's) are uploaded whole, and every product runs over the whole
tensor in the launch configuration the bench and the solver use: narrow
widths 5, 10, 20, the core product at k1 = 70 (C2) and k1 = 190 (C3) on the
matrix cores, FP32 and FP64 accumulation.  The FP64 oracle then recomputes a
sample of output rows from exactly the entries those rows depend on (Section
2.2 definitions): a FREE3 row k from slice k, a FREE1 row r from the entries
in row or column r, a MODE3 row from the entries of its stored pair.  The
samples include the longest slice, the heaviest row and the row of degree
rank 30 (not at C3 width 20), the row of degree rank 300 (split segments and
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
    def __init__(self, ctx, coo, seed):
        self.coo = coo
        self.t = ctx.upload_coo(coo)
        rng = np.random.default_rng(seed)
        slen = np.bincount(coo.k, minlength=coo.n)
        nonempty = np.flatnonzero(slen)
        self.slices = np.unique(np.concatenate(
            [[int(np.argmax(slen))], rng.choice(nonempty, 9, replace=False)]))
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
    want = ref.free1(T, Y, Z)[rows]
    absw = ref.free1(pb.abs_tensor(T), np.abs(Y), np.abs(Z))[rows]
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
    # (the oracle's cost grows with p^2 x sampled entries: the heaviest rows
    # are left out at p = 20)
    free1_sampled(ctx, c3, p, p, bks.F32, 400 + p, heavy=p < 20)
    mode3_sampled(ctx, c3, p, bks.F32, 500 + p)


def test_c3_core_product(ctx, c3):
    # the rank-(10,10,10) solve's core product at k1 = 190
    free3_sampled(ctx, c3, 190, 190, bks.F32, True, 600)

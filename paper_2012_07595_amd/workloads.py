"""Seeded synthetic inputs for the (1,2)-symmetric sparse tensor workloads.

This module only draws inputs: coordinates, values, random start matrices and
arrival times. It performs none of the method's arithmetic (no contractions,
no orthogonalisation), so both the FP64 oracle and the HIP path can consume
the same inputs without sharing any computation.

The shapes and value laws follow the paper's experiments (section "Experiments"):
sparse (1,2)-symmetric tensors A in R^{m x m x n} whose mode-3 slices are
symmetric (Definition of a (1,2)-symmetric tensor, section "Notation"), with
power-law mode-1/2 indices (social-network and word co-occurrence tensors)
and uniform mode-3 indices.  Indices are 0-based.

Every stored entry is one distinct position (i, j, k) with i <= j; the full
tensor holds it at (i, j, k) and (j, i, k).
"""
from __future__ import annotations

import dataclasses
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


@dataclasses.dataclass
class SymCOO:
    """Stored upper-triangular entries of a (1,2)-symmetric tensor."""

    m: int
    n: int
    i: np.ndarray  # int32, i <= j
    j: np.ndarray  # int32
    k: np.ndarray  # int32
    val: np.ndarray  # float32 or float64

    @property
    def nnz(self) -> int:
        return int(self.i.shape[0])

    def astype(self, dtype) -> "SymCOO":
        return dataclasses.replace(self, val=self.val.astype(dtype))


def _zipf_labels(rng, m: int, size: int, s: float, perm: np.ndarray) -> np.ndarray:
    """Draw labels in [0, m): rank r (1-based) has probability ~ r^-s, then a
    fixed permutation maps ranks to labels so heavy rows are not at index 0.
    s == 0 gives the uniform law."""
    if s == 0.0:
        return rng.integers(0, m, size=size, dtype=np.int64)
    w = np.arange(1, m + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    u = rng.random(size)
    r = np.searchsorted(cdf, u, side="right")
    np.minimum(r, m - 1, out=r)
    return perm[r]


def sparse_sym(m: int, n: int, nnz: int, zipf: float = 0.0, values: str = "normal",
               seed: int = 0, dtype=np.float32) -> SymCOO:
    """Generator G(m, n, nnz, s, values): exactly ``nnz`` distinct stored
    positions (i <= j, k).  i and j are drawn from a truncated Zipf(s) law on
    the (permuted) row labels, k uniformly; positions are canonicalised to
    (min, max), deduplicated, oversampled until enough distinct positions
    exist, and a seeded subset of exactly ``nnz`` is kept.

    values: "normal" -> N(0,1); "abs" -> |N(0,1)|; "ones" -> 1.
    """
    if nnz < 0:
        raise ValueError("nnz must be >= 0")
    cap = (m * (m + 1) // 2) * n
    if nnz > cap:
        raise ValueError(f"nnz={nnz} exceeds the {cap} available positions")
    rng = np.random.default_rng(seed)
    perm = rng.permutation(m).astype(np.int64)
    keys = np.empty(0, dtype=np.int64)
    rounds = 0
    yield_est = 1.0
    piece = 4_000_000
    cdf = None
    if zipf != 0.0:
        w = np.arange(1, m + 1, dtype=np.float64) ** (-zipf)
        cdf = np.cumsum(w)
        cdf /= cdf[-1]

    def draw_piece(args):
        rnd, idx, d = args
        prng = np.random.default_rng([seed, rnd, idx])
        ab = []
        for _ in range(2):
            if cdf is None:
                ab.append(prng.integers(0, m, size=d, dtype=np.int64))
            else:
                r = np.searchsorted(cdf, prng.random(d), side="right")
                np.minimum(r, m - 1, out=r)
                ab.append(perm[r])
        kk = prng.integers(0, n, size=d, dtype=np.int64)
        a, b = ab
        return np.unique((kk * m + np.minimum(a, b)) * m + np.maximum(a, b))

    while keys.shape[0] < nnz:
        missing = nnz - keys.shape[0]
        # size the round by the distinct-position yield seen so far (power-law
        # indices repeat heavy (i, j) fibres, so most draws can be repeats)
        draw = int(min(400_000_000, max(1024, missing / max(yield_est, 0.02) * 1.2 + 64)))
        jobs = [(rounds, x, min(piece, draw - s0)) for x, s0 in enumerate(range(0, draw, piece))]
        with ThreadPoolExecutor(max_workers=_threads()) as ex:
            parts = list(ex.map(draw_piece, jobs))
        before = keys.shape[0]
        allk = np.concatenate([keys] + parts)
        allk.sort(kind="stable")  # merges the sorted runs
        keep = np.empty(allk.shape[0], dtype=bool)
        if allk.shape[0]:
            keep[0] = True
            np.not_equal(allk[1:], allk[:-1], out=keep[1:])
        keys = allk[keep]
        yield_est = max((keys.shape[0] - before) / draw, 1e-4)
        rounds += 1
        if rounds > 60:
            raise RuntimeError("could not draw enough distinct positions")
    if keys.shape[0] > nnz:
        keep = rng.choice(keys.shape[0], size=nnz, replace=False)
        keep.sort()
        keys = keys[keep]
    j = keys % m
    t = keys // m
    i = t % m
    k = t // m
    if values == "normal":
        v = rng.standard_normal(nnz)
    elif values == "abs":
        v = np.abs(rng.standard_normal(nnz))
    elif values == "ones":
        v = np.ones(nnz)
    else:
        raise ValueError(values)
    # shuffle the order so no consumer can rely on sorted input
    order = rng.permutation(nnz)
    return SymCOO(m, n, i[order].astype(np.int32), j[order].astype(np.int32),
                  k[order].astype(np.int32), v[order].astype(dtype))


def planted(m: int, n: int, core_diag, rows_per_col: int, slices_per_col: int,
            seed: int) -> SymCOO:
    """A planted (1,2)-symmetric tensor sum_t f_t u_t o u_t o w_t with a
    superdiagonal core f (``core_diag``) and factors that are orthonormal by
    construction: column t of U is N(0,1) on its own block of ``rows_per_col``
    random rows (disjoint across columns) scaled to unit length, and the same
    for W with ``slices_per_col`` slices.  Multilinear rank (r, r, r) with
    r = len(core_diag).  Returned as stored entries (i <= j)."""
    rng = np.random.default_rng(seed)
    r = len(core_diag)
    rows = rng.choice(m, size=r * rows_per_col, replace=False).reshape(r, rows_per_col)
    sl = rng.choice(n, size=r * slices_per_col, replace=False).reshape(r, slices_per_col)
    ii, jj, kk, vv = [], [], [], []
    for t in range(r):
        u = rng.standard_normal(rows_per_col)
        u /= np.sqrt(np.sum(u * u))
        w = rng.standard_normal(slices_per_col)
        w /= np.sqrt(np.sum(w * w))
        ridx = rows[t]
        for a in range(rows_per_col):
            for b in range(rows_per_col):
                if ridx[a] > ridx[b]:
                    continue
                for c in range(slices_per_col):
                    ii.append(ridx[a]); jj.append(ridx[b]); kk.append(sl[t, c])
                    vv.append(core_diag[t] * u[a] * u[b] * w[c])
    return SymCOO(m, n, np.asarray(ii, np.int32), np.asarray(jj, np.int32),
                  np.asarray(kk, np.int32), np.asarray(vv, np.float64))


def merge(a: SymCOO, b: SymCOO) -> SymCOO:
    """Union of two stored-entry sets of the same shape; values at common
    positions are added."""
    assert a.m == b.m and a.n == b.n
    m = a.m
    ka = (a.k.astype(np.int64) * m + a.i) * m + a.j
    kb = (b.k.astype(np.int64) * m + b.i) * m + b.j
    keys = np.concatenate([ka, kb])
    vals = np.concatenate([a.val.astype(np.float64), b.val.astype(np.float64)])
    uk, inv = np.unique(keys, return_inverse=True)
    v = np.zeros(uk.shape[0])
    np.add.at(v, inv, vals)
    j = uk % m
    t = uk // m
    return SymCOO(m, a.n, (t % m).astype(np.int32), j.astype(np.int32),
                  (t // m).astype(np.int32), v.astype(a.val.dtype))


def random_start(m: int, n: int, r: int, r3: int, seed: int):
    """N(0,1) start matrices (m x r, n x r3) for BKS and HOOI.  Both the oracle
    and the library orthonormalise them themselves."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((m, r)), rng.standard_normal((n, r3))


def random_block(rows: int, cols: int, seed: int, dtype=np.float64):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((rows, cols)).astype(dtype)


def dense_signal_noise(m: int, n: int, r: int, r3: int, rho: float, seed: int):
    """Example-1-like dense tensor (Example 1 of the Experiments section): an (r, r, r3) N(0,1) block,
    symmetrised in modes 1-2, placed in the leading corner of an m x m x n zero
    tensor, plus rho times a symmetrised N(0,1) noise tensor; then one random
    permutation applied to modes 1 and 2 and an independent one to mode 3.
    Returned as the stored entries (i <= j) of the dense tensor.  Symmetrising
    is done by averaging a block with its 1-2 transpose (input shaping only)."""
    rng = np.random.default_rng(seed)
    S = rng.standard_normal((r, r, r3))
    S = 0.5 * (S + S.transpose(1, 0, 2))
    N = rng.standard_normal((m, m, n))
    N = 0.5 * (N + N.transpose(1, 0, 2))
    A = rho * N
    A[:r, :r, :r3] += S
    p12 = rng.permutation(m)
    p3 = rng.permutation(n)
    A = A[np.ix_(p12, p12, p3)]
    iu, ju = np.triu_indices(m)
    i = np.repeat(iu, n)
    j = np.repeat(ju, n)
    k = np.tile(np.arange(n), iu.shape[0])
    v = A[i, j, k]
    return SymCOO(m, n, i.astype(np.int32), j.astype(np.int32), k.astype(np.int32), v)


# ---------------------------------------------------------------- configs
# Workloads shaped like the benchmark configurations.  Seeds are 1000 + index.

def c1(seed: int = 1000) -> SymCOO:
    """500 x 500 x 100: 5e4 uniform stored positions with N(0,1) values (FP64)
    plus a planted rank-(2,2,2) part with superdiagonal core (10, 5) whose
    factors live on 10 rows and 5 slices per column."""
    noise = sparse_sym(500, 100, 50_000, zipf=0.0, values="normal", seed=seed,
                       dtype=np.float64)
    plant = planted(500, 100, (10.0, 5.0), 10, 5, seed + 7)
    return merge(noise, plant)


def c2(seed: int = 1001) -> SymCOO:
    """20000 x 20000 x 2000, 2e6 stored, Zipf(1.3) modes 1-2, |N(0,1)| FP32."""
    return sparse_sym(20_000, 2_000, 2_000_000, zipf=1.3, values="abs", seed=seed)


def c2_planted(seed: int = 1001, m: int = 20_000, n: int = 2_000, nnz: int = 2_000_000,
               rows_per_col: int = 40, slices_per_col: int = 20) -> SymCOO:
    """The C2 law (20000 x 20000 x 2000, Zipf(1.3) modes 1-2, uniform mode 3,
    |N(0,1)| FP32) with about 82k of its 2e6 stored entries given to a planted
    rank-(5,5,5) part (superdiagonal core 3000, 2500, 2000, 1500, 1000; each
    factor column on 40 rows / 20 slices).  The plain law has a flat mode-3
    spectrum (uniform mode-3 indices), so its rank-(5,5,5) problem is
    ill-conditioned; the plant gives it separated S-values.  The size
    arguments give smaller tensors of the same law."""
    plant = planted(m, n, (3000.0, 2500.0, 2000.0, 1500.0, 1000.0), rows_per_col,
                    slices_per_col, seed + 7)
    noise = sparse_sym(m, n, nnz - plant.nnz, zipf=1.3, values="abs", seed=seed)
    return merge(noise.astype(np.float64), plant).astype(np.float32)


def c3(seed: int = 1002) -> SymCOO:
    """200000 x 200000 x 10000, 5e7 stored, Zipf(1.5) modes 1-2, |N(0,1)| FP32."""
    return sparse_sym(200_000, 10_000, 50_000_000, zipf=1.5, values="abs", seed=seed)


def c3_planted(seed: int = 1002) -> SymCOO:
    """The C3 law (200000 x 200000 x 10000, 5e7 stored, Zipf(1.5) modes 1-2,
    uniform mode 3, |N(0,1)| FP32) with a planted rank-(10,10,10) part
    (superdiagonal core 8000, 7500, ..., 3500; each factor column on 40 rows
    and 20 slices, ~82k stored entries).  Like the plain C2 law, the plain C3
    law has no separated rank-10 structure for BKS to converge to."""
    plant = planted(200_000, 10_000, tuple(8000.0 - 500.0 * x for x in range(10)), 40, 20,
                    seed + 7)
    noise = sparse_sym(200_000, 10_000, 50_000_000 - plant.nnz, zipf=1.5, values="abs",
                       seed=seed)
    return merge(noise.astype(np.float64), plant).astype(np.float32)


def chung_lu_sym(m: int, n: int, nnz: int, s: float, values: str = "abs", seed: int = 0,
                 dtype=np.float32) -> SymCOO:
    """Power-law degree generator: exactly ``nnz`` distinct stored positions
    (i <= j, k) of an m x m x n (1,2)-symmetric tensor whose row degrees
    follow a Zipf(s) law on the (permuted) row labels.

    Chung-Lu law: the node of rank r has weight w_r = r^-s, and every
    position (a <= b, k) is stored with probability min(1, c w_a w_b), with c
    chosen so that the expected count is nnz.  Pairs with c w_a w_b >= 1 are
    stored in all n slices (enumerated); for the rest, row a draws a Poisson
    number of positions with mean n c w_a (sum of w_b over its unsaturated
    partners b >= a), partners b from w restricted to those ranks, slices
    uniformly.  Repeated positions are removed, rounds are drawn until nnz
    distinct positions exist, and a seeded subset of exactly nnz is kept."""
    if nnz < 0:
        raise ValueError("nnz must be >= 0")
    rng = np.random.default_rng(seed)
    perm = rng.permutation(m).astype(np.int64)
    r = np.arange(1, m + 1, dtype=np.float64)
    w = r ** (-s)
    pre = np.concatenate([[0.0], np.cumsum(w)])          # pre[b] = sum_{b' <= b} w
    tot = pre[-1]

    def layout(c):
        J = np.minimum(np.floor((c * w) ** (1.0 / s)), m).astype(np.int64)
        a = np.arange(1, m + 1, dtype=np.int64)
        sat = np.maximum(0, J - a + 1)
        b0 = np.maximum(a, J + 1)
        lam = np.where(b0 <= m, n * c * w * (tot - pre[np.minimum(b0, m + 1) - 1]), 0.0)
        return J, sat, b0, lam

    lo, hi = 1e-12, 1e18
    for _ in range(200):
        mid = np.sqrt(lo * hi)
        _, sat, _, lam = layout(mid)
        if n * sat.sum() + lam.sum() < nnz:
            lo = mid
        else:
            hi = mid
    J, sat, b0, lam = layout(hi)

    def key(ra, rb, k):
        la, lb = perm[ra - 1], perm[rb - 1]
        return (k * m + np.minimum(la, lb)) * m + np.maximum(la, lb)

    parts = []
    for a in np.flatnonzero(sat > 0) + 1:
        bs = np.arange(a, J[a - 1] + 1, dtype=np.int64)
        kk = np.arange(n, dtype=np.int64)
        parts.append(key(np.full(bs.size * n, a), np.repeat(bs, n), np.tile(kk, bs.size)))
    keys = np.unique(np.concatenate(parts)) if parts else np.empty(0, np.int64)
    rows = np.arange(1, m + 1, dtype=np.int64)
    rounds = 0
    scale = 1.0
    while keys.shape[0] < nnz:
        cnt = rng.poisson(lam * scale)
        new = []
        step = 2_000_000
        # rows in blocks of about `step` samples
        cum = np.cumsum(cnt)
        start = 0
        while start < m:
            stop = int(np.searchsorted(cum, (cum[start - 1] if start else 0) + step, side="right"))
            stop = max(stop, start + 1)
            ra = np.repeat(rows[start:stop], cnt[start:stop])
            if ra.size:
                lo_w = pre[b0[ra - 1] - 1]
                u = lo_w + rng.random(ra.size) * (tot - lo_w)
                rb = np.minimum(np.searchsorted(pre, u, side="left"), m)
                rb = np.maximum(rb, b0[ra - 1])
                new.append(np.unique(key(ra, rb, rng.integers(0, n, size=ra.size, dtype=np.int64))))
            start = stop
        before = keys.shape[0]
        keys = np.unique(np.concatenate([keys] + new))
        got = keys.shape[0] - before
        rounds += 1
        if rounds > 20:
            raise RuntimeError("could not draw enough distinct positions")
        # next round: enough draws for the deficit at this round's yield
        scale = max(0.05, 1.2 * (nnz - keys.shape[0]) / max(got, 1)) * scale
    if keys.shape[0] > nnz:
        keep = rng.choice(keys.shape[0], size=nnz, replace=False)
        keep.sort()
        keys = keys[keep]
    j = keys % m
    t = keys // m
    i = t % m
    k = t // m
    if values == "normal":
        v = rng.standard_normal(nnz)
    elif values == "abs":
        v = np.abs(rng.standard_normal(nnz))
    elif values == "ones":
        v = np.ones(nnz)
    else:
        raise ValueError(values)
    order = rng.permutation(nnz)
    return SymCOO(m, n, i[order].astype(np.int32), j[order].astype(np.int32),
                  k[order].astype(np.int32), v[order].astype(dtype))


def c5(seed: int = 1004) -> SymCOO:
    """1e6 x 1e6 x 500, 2e8 stored, Zipf(1.6) mode-1/2 degrees (Chung-Lu law,
    chung_lu_sym), |N(0,1)| FP32."""
    return chung_lu_sym(1_000_000, 500, 200_000_000, 1.6, values="abs", seed=seed)


@dataclasses.dataclass
class Request:
    rid: int
    arrival_s: float
    m: int
    n: int
    nnz: int
    r: int
    seed: int


def p_princeton(seed: int = 1010) -> SymCOO:
    """Stand-in for the Princeton tensor (section "Experiments", Example 2; the data set
    is not used): 6593 x 6593 x 29, entry (l, m, v) = 1 when l and m are
    friends and one of them has flag v.  Friendships are 3.1e5 distinct
    pairs l != m drawn from a Zipf(1.0) law on the (permuted) node labels;
    every node gets one of the 29 flags uniformly.  An edge is stored once in
    each of its endpoints' flag slices: about 6.1e5 stored entries, about
    1.2e6 entries of the full tensor (the count the paper states)."""
    m, n, edges = 6593, 29, 310_000
    rng = np.random.default_rng(seed)
    perm = rng.permutation(m).astype(np.int64)
    keys = np.empty(0, np.int64)
    while keys.shape[0] < edges:
        a = _zipf_labels(rng, m, 2 * edges, 1.0, perm)
        b = _zipf_labels(rng, m, 2 * edges, 1.0, perm)
        ok = a != b
        keys = np.unique(np.concatenate([keys, np.minimum(a, b)[ok] * m + np.maximum(a, b)[ok]]))
    keys = np.sort(rng.choice(keys, size=edges, replace=False))
    i, j = keys // m, keys % m
    flag = rng.integers(0, n, size=m)
    two = flag[i] != flag[j]
    ii = np.concatenate([i, i[two]])
    jj = np.concatenate([j, j[two]])
    kk = np.concatenate([flag[i], flag[j][two]])
    order = rng.permutation(ii.shape[0])
    return SymCOO(m, n, ii[order].astype(np.int32), jj[order].astype(np.int32),
                  kk[order].astype(np.int32), np.ones(ii.shape[0], np.float32))


def p_reuters(seed: int = 1011) -> SymCOO:
    """Stand-in for the Reuters tensor (section "Experiments", Example 3; the data set
    is not used): 13332 x 13332 x 66 with 486,894 nonzeros of the full tensor
    (read as 243,447 stored (i <= j, k) positions), indices from a Zipf(1.0)
    law, positive integer weights from a Zipf(2) law."""
    coo = sparse_sym(13332, 66, 243_447, zipf=1.0, values="ones", seed=seed)
    rng = np.random.default_rng(seed + 1)
    return dataclasses.replace(coo, val=rng.zipf(2.0, size=coo.nnz).astype(np.float32))


def p_darpa(seed: int = 1012) -> SymCOO:
    """Stand-in for the 1998 DARPA tensor (section "Experiments", Example 4; the data
    set is not used; its nonzero count is not stated and is read as 1e6
    stored positions): 8891 x 8891 x 371, binary, indices from a Zipf(1.2)
    law, then every slice scaled to Frobenius norm 1 as in the paper."""
    coo = sparse_sym(8891, 371, 1_000_000, zipf=1.2, values="ones", seed=seed)
    # full-tensor squared norm of slice k: off-diagonal stored entries count twice
    w = np.where(coo.i == coo.j, 1.0, 2.0)
    norm2 = np.bincount(coo.k, weights=w, minlength=coo.n)
    scale = 1.0 / np.sqrt(np.maximum(norm2, 1.0))
    return dataclasses.replace(coo, val=scale[coo.k].astype(np.float32))


def c4_requests(count: int = 512, rate_per_s: float = 10.0, seed: int = 1003,
                m_range=(1_000, 100_000), n_range=(100, 5_000),
                nnz_range=(10_000, 5_000_000), ranks=(2, 3, 5, 8, 10)):
    """Serving trace: Poisson arrivals at ``rate_per_s``; per request I, K and
    nnz uniform on their ranges, r1 = r2 = r3 = r drawn from ``ranks``.  The
    tensor of request ``rid`` is ``sparse_sym(m, n, nnz, 1.3, 'abs', seed)``
    with seed 4000 + rid."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=count)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for q in range(count):
        m = int(rng.integers(m_range[0], m_range[1] + 1))
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        nnz = int(rng.integers(nnz_range[0], nnz_range[1] + 1))
        nnz = min(nnz, (m * (m + 1) // 2) * n // 4)
        r = int(rng.choice(ranks))
        out.append(Request(q, float(t[q]), m, n, nnz, r, 4000 + q))
    return out


def request_tensor(req: Request, plant: bool = True) -> SymCOO:
    """Tensor of a serving request.  With ``plant`` a rank-(r, r, r) part with
    separated S-values (superdiagonal core 5000, 4600, ..., above the noise's
    mean component; factors on 12 rows and 6 slices per column) replaces part
    of the entries: the plain law has a flat mode-3 spectrum, so its rank-r
    problems are ill-conditioned."""
    if not plant:
        return sparse_sym(req.m, req.n, req.nnz, zipf=1.3, values="abs", seed=req.seed)
    p = planted(req.m, req.n, tuple(5000.0 - 400.0 * x for x in range(req.r)), 12,
                min(6, req.n // max(req.r, 1)), req.seed + 100_000)
    base = sparse_sym(req.m, req.n, max(req.nnz - p.nnz, 0), zipf=1.3, values="abs", seed=req.seed)
    return merge(base.astype(np.float64), p).astype(np.float32)

"""Block-Krylov (BK) basis builders for (1,2)-symmetric tensors (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Two sequences of ON-blocks are built (section "Block-Krylov methods for (1,2)-symmetric tensors"): U-blocks for modes 1-2
and W-blocks for mode 3.  A new U-block comes from A.(Ubar_a, Wbar_b)_{2,3}
(Algorithm 3, mode 1); a new W-block from A.(Ubar_a, Ubar_b)_{1,2}, using the
upper-triangular mode-3 unfolding (triunfold_3) when a = b.

Which block pairs are multiplied is the variant (Tables 1-3):

  min-BK (Algorithm 4, Table 1): stage i uses (Ubar_{i-1}, Wbar_{i-1}) and
          (Ubar_{i-1}, Ubar_{i-1}).
  BK     (Table 3): stage 1 uses (U0, W0) and (U0, U0); stage t >= 2, with
          q = t - 1, uses for a = 0..q-1 the pairs (U_a, Wbar_q) and
          (Ubar_q, Wbar_a) for new U-blocks, then (Ubar_a, Ubar_q) for new
          W-blocks.  The diagonal pairs are omitted.
  max-BK  (Table 2): stage 1 as BK; later stages use every not yet used pair
          of whole blocks available at the start of the stage.

A bar means the first p columns of a block, except that U0 and W0 are always
used whole (section "Min-BK method").  A mode stops growing once its basis reaches the
mode size (section "BK method").
"""
from __future__ import annotations

import numpy as np

from . import ttmc
from .orth import orth_append


def stage_products(variant: str, stage: int, nu: int, nw: int, used_u: set, used_w: set):
    """Products of one stage as ('U', a, b) / ('W', a, b) block-index pairs.

    nu, nw: number of U- and W-blocks available at the start of the stage."""
    if stage == 1:
        return [("U", 0, 0), ("W", 0, 0)]
    if variant == "min":
        q = stage - 1
        return [("U", q, q), ("W", q, q)]
    if variant == "bk":
        q = stage - 1
        prods = []
        for a in range(q):
            prods.append(("U", a, q))
            prods.append(("U", q, a))
        for a in range(q):
            prods.append(("W", a, q))
        return prods
    if variant == "max":
        prods = []
        for s_ in range(1, max(nu, nw)):
            for a in range(s_):
                if a < nu and s_ < nw and (a, s_) not in used_u:
                    prods.append(("U", a, s_))
                if s_ < nu and a < nw and (s_, a) not in used_u:
                    prods.append(("U", s_, a))
            if s_ < nu and s_ < nw and (s_, s_) not in used_u:
                prods.append(("U", s_, s_))
        for s_ in range(nu):
            for a in range(s_ + 1):
                if (a, s_) not in used_w:
                    prods.append(("W", a, s_))
        return prods
    raise ValueError(variant)


def _bar(width: int, b: int, p: int | None) -> int:
    if b == 0 or p is None:
        return width
    return min(p, width)


def dims(variant: str, r: int, r3: int, p: int | None, stages: int, m: int = 10**12,
         n: int = 10**12):
    """Basis dimensions (k1, k3) after each stage, assuming no deflation.

    Returns a list of (k1, k3) per stage.  Used to check Tables 1-3."""
    uw = [r]
    ww = [r3]
    used_u, used_w = set(), set()
    out = []
    for t in range(1, stages + 1):
        prods = stage_products(variant, t, len(uw), len(ww), used_u, used_w)
        nuw, nww = [], []
        for kind, a, b in prods:
            if kind == "U":
                used_u.add((a, b))
                nuw.append(_bar(uw[a], a, p) * _bar(ww[b], b, p))
            else:
                used_w.add((a, b))
                pa, pb = _bar(uw[a], a, p), _bar(uw[b], b, p)
                nww.append(pa * (pa + 1) // 2 if a == b else pa * pb)
        # cap at the mode sizes
        for w in nuw:
            w = min(w, m - sum(uw))
            uw.append(w)
        for w in nww:
            w = min(w, n - sum(ww))
            ww.append(w)
        out.append((sum(uw), sum(ww)))
    return out


class Basis:
    """ON-blocks U_0, U_1, ... and W_0, W_1, ... with their concatenations
    X = [U_0 U_1 ...] and Z = [W_0 W_1 ...]."""

    def __init__(self, U0: np.ndarray, W0: np.ndarray):
        self.ub = [U0]
        self.wb = [W0]
        self.used_u = set()
        self.used_w = set()

    @property
    def X(self):
        return np.concatenate(self.ub, axis=1)

    @property
    def Z(self):
        return np.concatenate(self.wb, axis=1)

    def ubar(self, a: int, p: int | None):
        B = self.ub[a]
        return B if (a == 0 or p is None) else B[:, :p]

    def wbar(self, b: int, p: int | None):
        B = self.wb[b]
        return B if (b == 0 or p is None) else B[:, :p]


def run_stage(T, basis: Basis, variant: str, stage: int, p: int | None,
              tau: float = 1e-14):
    """Compute and append the new blocks of one stage (Algorithm 3 per product)."""
    prods = stage_products(variant, stage, len(basis.ub), len(basis.wb),
                           basis.used_u, basis.used_w)
    new_u, new_w = [], []
    for kind, a, b in prods:
        if kind == "U":
            basis.used_u.add((a, b))
            Y, Zb = basis.ubar(a, p), basis.wbar(b, p)
            new_u.append((Y, Zb))
        else:
            basis.used_w.add((a, b))
            new_w.append((a, b, basis.ubar(a, p), basis.ubar(b, p)))
    for Y, Zb in new_u:
        X = basis.X
        if Y.shape[1] == 0 or Zb.shape[1] == 0 or X.shape[1] >= T.m:
            basis.ub.append(np.zeros((T.m, 0)))
            continue
        B = ttmc.free1(T, Y, Zb)
        Q, _ = orth_append(X, B, T.m, tau)
        basis.ub.append(Q)
    for a, b, Ya, Yb in new_w:
        Z = basis.Z
        if Ya.shape[1] == 0 or Yb.shape[1] == 0 or Z.shape[1] >= T.n:
            basis.wb.append(np.zeros((T.n, 0)))
            continue
        if a == b:
            B = ttmc.free3(T, Ya, sym_half=True)
        else:
            B = ttmc.free3(T, Ya, Yb)
        Q, _ = orth_append(Z, B, T.n, tau)
        basis.wb.append(Q)

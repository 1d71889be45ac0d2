"""Row-wise acceptance bound shared by the FP32 product parity tests.

The target is a relative error of 1e-5 per call (normwise) and per output row
(rows with norm >= 1e-3 of the largest).  A row that is a sum of L terms of
mixed sign can be far smaller than the sum of its terms' magnitudes, and then
no FP32 accumulation meets 1e-5 relative: each rounding is relative to the
partial sums, not to the result.  For such a row the test takes the standard
probabilistic forward-error bound of an L-term sum, lambda sqrt(L) u times
the row of the same product taken with |A|, |X|, |Y| (u = 2^-24, lambda = 4:
exceeded with probability below 1e-3 per element under independent rounding
errors).  A row passes when its error is within the larger of the two.
"""
import numpy as np

from oracle import sptensor

U32 = 2.0 ** -24
U64 = 2.0 ** -53
LAMBDA = 4.0


def abs_tensor(T):
    """The same stored pattern with |values| (oracle representation)."""
    return sptensor.SymTensor(T.m, T.n, T.i, T.j, T.k, np.abs(T.a))


def max_terms(T, op):
    """Upper bound on the terms summed into one output element of `op`:
    twice the longest slice (FREE3), the largest row degree counting both
    orientations (FREE1), or the most slices of one stored pair (MODE3)."""
    if T.nnz == 0:
        return 1
    if op == "free3":
        return 2 * int(np.bincount(T.k, minlength=T.n).max())
    if op == "free1":
        off = T.i != T.j
        deg = np.bincount(np.concatenate([T.i, T.j[off]]), minlength=T.m)
        return int(deg.max())
    key = T.i * T.m + T.j
    return int(np.unique(key, return_counts=True)[1].max())


def rows_ok(got, want, absw, L, tol=1e-5, u=U32):
    """Largest ratio of a checked row's error to its allowance (<= 1 passes);
    u is the unit roundoff of the accumulation (U32, or U64 for products that
    accumulate in FP64, whose target is 1e-12)."""
    rn = np.linalg.norm(want, axis=1)
    big = rn >= 1e-3 * rn.max()
    err = np.linalg.norm(got - want, axis=1)[big]
    allow = np.maximum(tol * rn[big],
                       LAMBDA * np.sqrt(L) * u * np.linalg.norm(absw, axis=1)[big])
    return float((err / allow).max()) if err.size else 0.0

"""The binding's argument checks of Ctx.ttmc (CPU only: they run before any
library call).  The library sees raw pointers, so the binding refuses
operands whose dtype, device, layout or row count does not match the
product, and an output narrower than the product writes."""
import types

import pytest

from paper_2012_07595_amd import bks


class Fake:
    """Stands in for a 2-D device tensor: only what the checks read."""

    def __init__(self, rows, cols, esz=4, cuda=True, col_stride=1, row_stride=None,
                 floating=True):
        self.shape = (rows, cols)
        self.is_cuda = cuda
        self._esz = esz
        self._strides = (cols if row_stride is None else row_stride, col_stride)
        self._floating = floating

    def dim(self):
        return 2

    def stride(self, d):
        return self._strides[d]

    def element_size(self):
        return self._esz

    def is_floating_point(self):
        return self._floating


T = types.SimpleNamespace(m=100, n=7, npairs=50, h=None)


def call(op, B1, B2, out, sym=False, prec=bks.F32):
    # every refusal is raised before the library is touched (self is unused)
    bks.Ctx.ttmc(None, T, op, B1, B2, out, sym_half=sym, prec=prec)


@pytest.mark.parametrize("args,msg", [
    ((bks.FREE3, Fake(100, 5, cuda=False), None, Fake(7, 15)), "device"),
    ((bks.FREE3, Fake(100, 5, esz=8), None, Fake(7, 15)), "float32"),
    ((bks.FREE3, Fake(99, 5), None, Fake(7, 15)), "rows"),
    ((bks.FREE3, Fake(100, 5), None, Fake(7, 14)), "columns"),
    ((bks.FREE3, Fake(100, 5, col_stride=2), None, Fake(7, 15)), "unit column stride"),
    ((bks.FREE3, Fake(100, 5), Fake(100, 4), Fake(7, 19)), "columns"),
    ((bks.FREE1, Fake(100, 4), Fake(6, 5), Fake(100, 20)), "rows"),
    ((bks.FREE1, Fake(100, 4), None, Fake(100, 20)), "missing"),
    ((bks.FREE1, Fake(100, 4), Fake(7, 5), Fake(99, 20)), "rows"),
    ((bks.MODE3, None, Fake(7, 5), Fake(49, 5)), "rows"),
    ((bks.MODE3, None, Fake(7, 5, esz=4), Fake(50, 5, esz=8)), "float32"),
    ((7, Fake(100, 5), None, Fake(7, 15)), "unknown op"),
])
def test_ttmc_refuses_bad_operands(args, msg):
    op, B1, B2, out = args
    with pytest.raises(ValueError, match=msg):
        call(op, B1, B2, out, sym=(op == bks.FREE3 and B2 is None))


def test_ttmc_precision_sets_the_dtype():
    with pytest.raises(ValueError, match="float64"):
        call(bks.FREE1, Fake(100, 4), Fake(7, 5), Fake(100, 20), prec=bks.F64)

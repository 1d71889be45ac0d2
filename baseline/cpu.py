"""CPU baseline B (see the package docstring): build and call the C++/OpenMP
products, and run the oracle's BKS solve with them."""
from __future__ import annotations

import contextlib
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ttmc_omp.cpp")
LIB = os.path.join(HERE, "libttmc_omp.so")
_lib = None


def build() -> str:
    cmd = ["g++", "-O3", "-fopenmp", "-mavx2", "-mfma", "-fPIC", "-shared", SRC, "-o", LIB + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"baseline build failed: {' '.join(cmd)}\n{r.stderr}")
    os.replace(LIB + ".tmp", LIB)
    return LIB


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        lib = C.CDLL(LIB)
        p, i64, i32 = C.c_void_p, C.c_int64, C.c_int
        lib.cpu_free3.argtypes = [i64, p, p, p, p, p, i32, p, i32, i32, p]
        lib.cpu_free1.argtypes = [i64, p, p, p, p, p, i32, p, i32, p]
        lib.cpu_mode3.argtypes = [i64, p, p, p, p, i32, p]
        lib.cpu_threads.restype = C.c_int
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


class Layouts:
    """The sorted layouts of one oracle tensor (built once)."""

    def __init__(self, T):
        i, j, k, a = T.i, T.j, T.k, T.a
        o = np.lexsort((j, i, k))                      # slices, then (i, j)
        self.kptr = np.searchsorted(k[o], np.arange(T.n + 1)).astype(np.int64)
        self.ei, self.ej = i[o].astype(np.int32), j[o].astype(np.int32)
        self.ev = np.ascontiguousarray(a[o])
        off = i != j
        row = np.concatenate([i, j[off]]); col = np.concatenate([j, i[off]])
        kk = np.concatenate([k, k[off]]); v = np.concatenate([a, a[off]])
        o = np.lexsort((kk, col, row))
        self.rptr = np.searchsorted(row[o], np.arange(T.m + 1)).astype(np.int64)
        self.col, self.rk = col[o].astype(np.int32), kk[o].astype(np.int32)
        self.rv = np.ascontiguousarray(v[o])
        key = i * T.m + j
        o = np.lexsort((k, key))
        uk, first = np.unique(key[o], return_index=True)
        self.pptr = np.append(first, key.shape[0]).astype(np.int64)
        self.pi, self.pj = (uk // T.m), (uk % T.m)
        self.pk = k[o].astype(np.int32)
        self.pv = np.ascontiguousarray(a[o])


_cache: dict = {}


def layouts(T) -> Layouts:
    ent = _cache.get(id(T))
    if ent is None or ent[0] is not T:
        ent = (T, Layouts(T))
        _cache[id(T)] = ent
    return ent[1]


def free3(T, X, Y=None, sym_half=False):
    L, lib = layouts(T), load()
    X = np.ascontiguousarray(X, dtype=np.float64)
    same = Y is None
    Yc = X if same else np.ascontiguousarray(Y, dtype=np.float64)
    px, py = X.shape[1], Yc.shape[1]
    q = px * (px + 1) // 2 if sym_half else px * py
    out = np.empty((T.n, q))
    lib.cpu_free3(T.n, _p(L.kptr), _p(L.ei), _p(L.ej), _p(L.ev), _p(X), px, _p(Yc), py,
                  1 if sym_half else 0, _p(out))
    return out


def free1(T, Y, Z):
    L, lib = layouts(T), load()
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    out = np.empty((T.m, Y.shape[1] * Z.shape[1]))
    lib.cpu_free1(T.m, _p(L.rptr), _p(L.col), _p(L.rk), _p(L.rv), _p(Y), Y.shape[1], _p(Z),
                  Z.shape[1], _p(out))
    return out


def mode3(T, Z):
    L, lib = layouts(T), load()
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    out = np.empty((L.pi.shape[0], Z.shape[1]))
    lib.cpu_mode3(L.pi.shape[0], _p(L.pptr), _p(L.pk), _p(L.pv), _p(Z), Z.shape[1], _p(out))
    return L.pi, L.pj, out


@contextlib.contextmanager
def products():
    """The oracle's contractions replaced by these kernels for the duration."""
    from oracle import ttmc
    saved = (ttmc.free3, ttmc.free1, ttmc.mode3)
    ttmc.free3, ttmc.free1, ttmc.mode3 = free3, free1, mode3
    try:
        yield
    finally:
        ttmc.free3, ttmc.free1, ttmc.mode3 = saved


def bks_solve(T, *args, **kw):
    """The oracle's BKS solve with the C++/OpenMP products."""
    from oracle import bks
    with products():
        return bks.bks_solve(T, *args, **kw)


def threads() -> int:
    return load().cpu_threads()

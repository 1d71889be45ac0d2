"""ctypes binding of libbks (the C ABI in include/bks.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Device buffers are passed as raw pointers (torch tensors are used
for device memory and streams).  Loading fails loudly when the library has
not been built; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libbks.so")

OK, EINVAL, EINDEX, EVALUE, EASYM, ENOMEM, EDEVICE, ENOTFOUND, EDUP = 0, -1, -2, -3, -4, -5, -6, -7, -8
ECANCELED = -9
ENOTCONV = 1
F32, F64, F32IN_F64ACC = 0, 1, 2
FREE3, FREE1, MODE3 = 0, 1, 2
DEVICE_PTRS, SUM_DUPLICATES, FULL_SYMMETRIC = 1, 2, 4
SCALE_FROBENIUS, SCALE_LAMBDA_MAX = 8, 16
VARIANT = {"bk": 0, "min": 1, "max": 2}
PREC_FP64, PREC_MIXED = 0, 1

SYMBOLS = [
    "bks_ctx_create", "bks_ctx_destroy", "bks_last_error", "bks_version",
    "bks_ctx_profile", "bks_ctx_profile_read",
    "bks_tensor_upload", "bks_tensor_info", "bks_tensor_pairs", "bks_tensor_free",
    "bks_ttmc", "bks_ttmc_noalloc", "bks_solve", "hooi_solve",
    "bks_gtensor_upload", "bks_gttmc", "bks_gsolve",
    "bks_server_create", "bks_server_submit", "bks_server_submit_coo", "bks_server_poll",
    "bks_server_wait", "bks_server_cancel", "bks_server_now", "bks_server_destroy",
]


class BksError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libbks error {code}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("r", C.c_int), ("r3", C.c_int), ("s", C.c_int), ("p", C.c_int),
                ("variant", C.c_int), ("precision", C.c_int), ("tol", C.c_double),
                ("inner_tol", C.c_double), ("max_outer", C.c_int), ("hooi_warm", C.c_int),
                ("ng_max", C.c_int), ("U0", C.c_void_p), ("W0", C.c_void_p),
                ("seed", C.c_uint64), ("inner_start", C.c_int)]


class HooiParams(C.Structure):
    _fields_ = [("r", C.c_int), ("r3", C.c_int), ("precision", C.c_int), ("tol", C.c_double),
                ("max_iter", C.c_int), ("grad_every", C.c_int), ("U0", C.c_void_p),
                ("W0", C.c_void_p), ("seed", C.c_uint64)]


class Info(C.Structure):
    _fields_ = [("outer_iters", C.c_int), ("converged", C.c_int), ("k1", C.c_int),
                ("k3", C.c_int), ("rel_grad", C.c_double), ("normF", C.c_double),
                ("normA", C.c_double), ("svals1", C.c_double * 65), ("svals3", C.c_double * 65),
                ("t_expand", C.c_double), ("t_core", C.c_double), ("t_inner", C.c_double),
                ("t_step", C.c_double), ("t_total", C.c_double), ("n_hist", C.c_int),
                ("rel_hist", C.c_double * 512), ("normF_hist", C.c_double * 512),
                ("svals2", C.c_double * 65), ("fp64_from", C.c_int)]


class GParams(C.Structure):
    _fields_ = [("r1", C.c_int), ("r2", C.c_int), ("r3", C.c_int), ("s", C.c_int), ("p", C.c_int),
                ("precision", C.c_int), ("tol", C.c_double), ("inner_tol", C.c_double),
                ("max_outer", C.c_int), ("U0", C.c_void_p), ("V0", C.c_void_p),
                ("W0", C.c_void_p), ("seed", C.c_uint64)]


class ServerParams(C.Structure):
    _fields_ = [("max_active", C.c_int), ("host_workers", C.c_int),
                ("mem_budget_bytes", C.c_size_t)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int), ("done", C.c_int), ("t_submit", C.c_double),
                ("t_start", C.c_double), ("t_end", C.c_double), ("info", Info),
                ("footprint", C.c_size_t), ("dev_peak", C.c_size_t), ("_error", C.c_char * 160)]

    @property
    def error(self):
        return self._error.decode(errors="replace")


_lib = None


def load(path: str = LIBPATH):
    """Load libbks.so; raises if it is missing (build it with build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run paper_2012_07595_amd/build.py")
    lib = C.CDLL(path)
    vp, i64, i32p = C.c_void_p, C.c_int64, C.POINTER(C.c_int32)
    lib.bks_ctx_create.argtypes = [C.c_int, C.c_size_t, C.POINTER(vp)]
    lib.bks_ctx_destroy.argtypes = [vp]
    lib.bks_ctx_destroy.restype = None
    lib.bks_last_error.argtypes = [vp]
    lib.bks_last_error.restype = C.c_char_p
    lib.bks_version.restype = C.c_char_p
    lib.bks_ctx_profile.argtypes = [vp, C.c_int]
    lib.bks_ctx_profile_read.argtypes = [vp, C.c_int, C.c_char_p, C.c_int, C.POINTER(i64),
                                         C.POINTER(C.c_double), C.POINTER(C.c_double),
                                         C.POINTER(C.c_double)]
    lib.bks_tensor_upload.argtypes = [vp, i64, i64, i64, vp, vp, vp, vp, C.c_int, C.c_uint,
                                      C.POINTER(vp)]
    lib.bks_tensor_info.argtypes = [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64),
                                    C.POINTER(i64), C.POINTER(C.c_double), C.POINTER(C.c_size_t)]
    lib.bks_tensor_pairs.argtypes = [vp, i32p, i32p]
    lib.bks_tensor_free.argtypes = [vp]
    lib.bks_tensor_free.restype = None
    lib.bks_ttmc.argtypes = [vp, vp, C.c_int, vp, i64, C.c_int, vp, i64, C.c_int, C.c_int,
                             C.c_int, vp, i64, vp]
    lib.bks_ttmc_noalloc.argtypes = lib.bks_ttmc.argtypes
    lib.bks_gtensor_upload.argtypes = [vp, i64, i64, i64, i64, vp, vp, vp, vp, C.c_int, C.c_uint,
                                       C.POINTER(vp)]
    lib.bks_gttmc.argtypes = [vp, vp, C.c_int, vp, i64, C.c_int, vp, i64, C.c_int, C.c_int, vp,
                              i64, vp]
    lib.bks_gsolve.argtypes = [vp, vp, C.POINTER(GParams), vp, vp, vp, vp, C.POINTER(Info)]
    lib.bks_solve.argtypes = [vp, vp, C.POINTER(Params), vp, vp, vp, C.POINTER(Info)]
    lib.hooi_solve.argtypes = [vp, vp, C.POINTER(HooiParams), vp, vp, vp, C.POINTER(Info)]
    lib.bks_server_create.argtypes = [vp, C.POINTER(ServerParams), C.POINTER(vp)]
    lib.bks_server_submit.argtypes = [vp, vp, C.POINTER(Params), vp, vp, vp, C.POINTER(C.c_uint64)]
    lib.bks_server_submit_coo.argtypes = [vp, i64, i64, i64, vp, vp, vp, vp, C.POINTER(Params),
                                          vp, vp, vp, C.POINTER(C.c_uint64)]
    lib.bks_server_poll.argtypes = [vp, C.c_uint64, C.POINTER(Result)]
    lib.bks_server_wait.argtypes = [vp, C.c_uint64, C.POINTER(Result)]
    lib.bks_server_cancel.argtypes = [vp, C.c_uint64]
    lib.bks_server_now.argtypes = [vp]
    lib.bks_server_now.restype = C.c_double
    lib.bks_server_destroy.argtypes = [vp]
    lib.bks_server_destroy.restype = None
    _lib = lib
    return lib


def _ptr(a):
    """Raw pointer of a numpy array or torch tensor (no copy)."""
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return C.c_void_p(a.data_ptr())
    return a.ctypes.data_as(C.c_void_p)


class Ctx:
    def __init__(self, device: int = 0, mem_budget: int = 0):
        self.lib = load()
        h = C.c_void_p()
        rc = self.lib.bks_ctx_create(device, mem_budget, C.byref(h))
        if rc != OK:
            raise BksError(rc, "bks_ctx_create failed")
        self.h = h

    def check(self, rc):
        if rc < 0:
            raise BksError(rc, self.lib.bks_last_error(self.h).decode())
        return rc

    def close(self):
        if self.h:
            # tensors go before their context
            for t in list(getattr(self, "_tensors", [])):
                obj = t()
                if obj is not None:
                    obj.free()
            self.lib.bks_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile(self, enable=True):
        """Start (and reset) or stop event timing of the tensor products."""
        self.check(self.lib.bks_ctx_profile(self.h, 1 if enable else 0))

    def profile_read(self):
        """{class: (calls, ms, algorithmic bytes, flops)} of the recorded launches."""
        out = {}
        idx = 0
        name = C.create_string_buffer(128)
        calls, ms, by, fl = C.c_int64(), C.c_double(), C.c_double(), C.c_double()
        while True:
            rc = self.lib.bks_ctx_profile_read(self.h, idx, name, 128, C.byref(calls), C.byref(ms),
                                               C.byref(by), C.byref(fl))
            if rc == ENOTFOUND:
                return out
            self.check(rc)
            out[name.value.decode()] = (calls.value, ms.value, by.value, fl.value)
            idx += 1

    def upload(self, m, n, i, j, k, val, flags=0):
        """Upload coordinates: host arrays (converted to int32 and float32 /
        float64), or contiguous device tensors (int32 coordinates, float32 or
        float64 values) that the caller has finished writing, passed as device
        pointers (BKS_DEVICE_PTRS)."""
        if all(getattr(a, "is_cuda", False) for a in (i, j, k, val)):
            for a in (i, j, k):
                if a.element_size() != 4 or a.is_floating_point() or not a.is_contiguous():
                    raise ValueError("device coordinates must be contiguous int32 tensors")
            if not val.is_floating_point() or val.element_size() not in (4, 8) \
                    or not val.is_contiguous():
                raise ValueError("device values must be a contiguous float32/float64 tensor")
            nnz = int(i.numel())
            if j.numel() != nnz or k.numel() != nnz or val.numel() != nnz:
                raise ValueError("coordinate and value lengths differ")
            dt = F64 if val.element_size() == 8 else F32
            h = C.c_void_p()
            self.check(self.lib.bks_tensor_upload(self.h, m, n, nnz, _ptr(i), _ptr(j), _ptr(k),
                                                  _ptr(val), dt, flags | DEVICE_PTRS,
                                                  C.byref(h)))
            return self._track(Tensor(self, h))
        i = np.ascontiguousarray(i, dtype=np.int32)
        j = np.ascontiguousarray(j, dtype=np.int32)
        k = np.ascontiguousarray(k, dtype=np.int32)
        val = np.ascontiguousarray(val)
        dt = F64 if val.dtype == np.float64 else F32
        if dt == F32:
            val = np.ascontiguousarray(val, dtype=np.float32)
        h = C.c_void_p()
        self.check(self.lib.bks_tensor_upload(self.h, m, n, int(i.shape[0]), _ptr(i), _ptr(j),
                                              _ptr(k), _ptr(val), dt, flags, C.byref(h)))
        return self._track(Tensor(self, h))

    def _track(self, t):
        import weakref
        if not hasattr(self, "_tensors"):
            self._tensors = []
        self._tensors = [w for w in self._tensors if w() is not None] + [weakref.ref(t)]
        return t

    def upload_coo(self, coo, flags=0):
        return self.upload(coo.m, coo.n, coo.i, coo.j, coo.k, coo.val, flags)

    def ttmc(self, t, op, B1, B2, out, sym_half=False, prec=F32, stream=None, noalloc=False):
        """out <- product; B1, B2, out are 2-D row-major device tensors (rows
        with unit stride).  noalloc: through bks_ttmc_noalloc (no device
        allocation; workspace in the library's fixed scratch).  The shapes and dtypes are checked here against the
        tensor and the precision (ValueError), since the library sees raw
        pointers.  stream: a hipStream_t value; None means torch's current
        stream on out's device."""
        esz = 4 if prec == F32 else 8
        want_rows = {FREE3: (t.m, t.m, t.n), FREE1: (t.m, t.n, t.m),
                     MODE3: (None, t.n, t.npairs)}
        if op not in want_rows:
            raise ValueError(f"unknown op {op}")
        r1, r2, ro = want_rows[op]
        for name, a, rows in (("B1", B1, r1), ("B2", B2, r2), ("out", out, ro)):
            if a is None:
                continue
            if not getattr(a, "is_cuda", False):
                raise ValueError(f"{name} must be a device tensor")
            if a.dim() != 2 or a.stride(1) != 1 or a.stride(0) < a.shape[1]:
                raise ValueError(f"{name} must be 2-D with unit column stride")
            if not a.is_floating_point() or a.element_size() != esz:
                raise ValueError(f"{name} must be float{8 * esz} for precision {prec}")
            if rows is not None and a.shape[0] != rows:
                raise ValueError(f"{name} has {a.shape[0]} rows, the product needs {rows}")
        if out is None or (op != MODE3 and B1 is None) or (op in (FREE1, MODE3) and B2 is None):
            raise ValueError("missing operand")
        p1 = B1.shape[1] if B1 is not None else 0
        ld1 = B1.stride(0) if B1 is not None else 0
        p2 = B2.shape[1] if B2 is not None else 0
        ld2 = B2.stride(0) if B2 is not None else 0
        if op == FREE3:
            q = p1 * (p1 + 1) // 2 if sym_half else p1 * (p2 if B2 is not None else p1)
        else:
            q = p1 * p2 if op == FREE1 else p2
        if out.shape[1] < q:
            raise ValueError(f"out has {out.shape[1]} columns, the product writes {q}")
        if stream is None:
            import torch
            stream = torch.cuda.current_stream(out.device).cuda_stream
        s = C.c_void_p(stream) if stream else None
        fn = self.lib.bks_ttmc_noalloc if noalloc else self.lib.bks_ttmc
        self.check(fn(self.h, t.h, op, _ptr(B1), ld1, p1, _ptr(B2), ld2, p2,
                      1 if sym_half else 0, prec, _ptr(out), out.stride(0), s))

    def upload_general(self, l, m, n, i, j, k, val, flags=0):
        """bks_gtensor_upload from host arrays (int32 coordinates, float32 or
        float64 values); returns a Tensor with dims (l, m, n)."""
        i = np.ascontiguousarray(i, dtype=np.int32)
        j = np.ascontiguousarray(j, dtype=np.int32)
        k = np.ascontiguousarray(k, dtype=np.int32)
        val = np.ascontiguousarray(val)
        dt = F64 if val.dtype == np.float64 else F32
        if dt == F32:
            val = np.ascontiguousarray(val, dtype=np.float32)
        h = C.c_void_p()
        self.check(self.lib.bks_gtensor_upload(self.h, l, m, n, int(i.shape[0]), _ptr(i), _ptr(j),
                                               _ptr(k), _ptr(val), dt, flags, C.byref(h)))
        t = self._track(Tensor(self, h))
        t.dims = (l, m, n)
        return t

    def gttmc(self, t, mode, B1, B2, out, prec=F32, stream=None):
        """bks_gttmc: product of a general tensor with free mode `mode` (0, 1,
        2); B1, B2 the factors of the other two modes in mode order."""
        esz = 4 if prec == F32 else 8
        l, m, n = t.dims
        rows = {0: (m, n, l), 1: (l, n, m), 2: (l, m, n)}
        if mode not in rows:
            raise ValueError(f"mode must be 0, 1 or 2, not {mode}")
        for name, a, nr in zip(("B1", "B2", "out"), (B1, B2, out), rows[mode]):
            if not getattr(a, "is_cuda", False) or a.dim() != 2 or a.stride(1) != 1:
                raise ValueError(f"{name} must be a 2-D device tensor with unit column stride")
            if not a.is_floating_point() or a.element_size() != esz:
                raise ValueError(f"{name} must be float{8 * esz} for precision {prec}")
            if a.shape[0] != nr:
                raise ValueError(f"{name} has {a.shape[0]} rows, the product needs {nr}")
        if out.shape[1] < B1.shape[1] * B2.shape[1]:
            raise ValueError("out is narrower than the product")
        if stream is None:
            import torch
            stream = torch.cuda.current_stream(out.device).cuda_stream
        s = C.c_void_p(stream) if stream else None
        self.check(self.lib.bks_gttmc(self.h, t.h, mode, _ptr(B1), B1.stride(0), B1.shape[1],
                                      _ptr(B2), B2.stride(0), B2.shape[1], prec, _ptr(out),
                                      out.stride(0), s))

    def gsolve(self, t, r, U0=None, V0=None, W0=None, p=4, s=2, precision=PREC_FP64, tol=0.0,
               inner_tol=0.0, max_outer=0, seed=0):
        """bks_gsolve: returns (U, V, W, F, info, status); r = (r1, r2, r3)."""
        l, m, n = t.dims
        prm = GParams(r[0], r[1], r[2], s, p, precision, tol, inner_tol, max_outer, None, None,
                      None, seed)
        keep = []
        for name, X in (("U0", U0), ("V0", V0), ("W0", W0)):
            if X is not None:
                a = np.asfortranarray(X, dtype=np.float64)
                keep.append(a)
                setattr(prm, name, a.ctypes.data)
        U = np.zeros((l, r[0]), order="F")
        V = np.zeros((m, r[1]), order="F")
        W = np.zeros((n, r[2]), order="F")
        F = np.zeros(tuple(r), order="F")
        info = Info()
        rc = self.check(self.lib.bks_gsolve(self.h, t.h, C.byref(prm), _ptr(U), _ptr(V), _ptr(W),
                                            _ptr(F), C.byref(info)))
        return U, V, W, F, info, rc

    def solve(self, t, r, r3, U0=None, W0=None, p=4, s=2, variant="bk", precision=PREC_FP64,
              tol=0.0, inner_tol=0.0, max_outer=0, hooi_warm=-1, ng_max=0, seed=0,
              inner_start=0):
        """bks_solve: returns (U, W, F, info, status)."""
        m, n = t.m, t.n
        keep = []
        prm = Params(r, r3, s, p, VARIANT[variant], precision, tol, inner_tol, max_outer,
                     hooi_warm, ng_max, None, None, seed, inner_start)
        if U0 is not None:
            u = np.asfortranarray(U0, dtype=np.float64)
            w = np.asfortranarray(W0, dtype=np.float64)
            keep += [u, w]
            prm.U0 = u.ctypes.data
            prm.W0 = w.ctypes.data
        U = np.zeros((m, r), order="F")
        W = np.zeros((n, r3), order="F")
        F = np.zeros((r, r, r3), order="F")
        info = Info()
        rc = self.check(self.lib.bks_solve(self.h, t.h, C.byref(prm), _ptr(U), _ptr(W), _ptr(F),
                                           C.byref(info)))
        return U, W, F, info, rc

    def hooi(self, t, r, r3, U0=None, W0=None, precision=PREC_FP64, tol=0.0, max_iter=0,
             grad_every=0, seed=0):
        m, n = t.m, t.n
        prm = HooiParams(r, r3, precision, tol, max_iter, grad_every, None, None, seed)
        keep = []
        if U0 is not None:
            u = np.asfortranarray(U0, dtype=np.float64)
            w = np.asfortranarray(W0, dtype=np.float64)
            keep += [u, w]
            prm.U0 = u.ctypes.data
            prm.W0 = w.ctypes.data
        U = np.zeros((m, r), order="F")
        W = np.zeros((n, r3), order="F")
        F = np.zeros((r, r, r3), order="F")
        info = Info()
        rc = self.check(self.lib.hooi_solve(self.h, t.h, C.byref(prm), _ptr(U), _ptr(W), _ptr(F),
                                            C.byref(info)))
        return U, W, F, info, rc


class Server:
    """Continuous-batching BKS server (bks_server_*).  Output buffers are
    held here until the request completes."""

    def __init__(self, ctx: Ctx, max_active=4, host_workers=4, mem_budget=0):
        self.ctx = ctx
        self.lib = ctx.lib
        h = C.c_void_p()
        prm = ServerParams(max_active, host_workers, mem_budget)
        ctx.check(self.lib.bks_server_create(ctx.h, C.byref(prm), C.byref(h)))
        self.h = h
        self._out = {}

    def _params(self, r, r3, precision, U0, W0, p, s, tol, max_outer, seed):
        prm = Params(r, r3, s, p, 0, precision, tol, 0.0, max_outer, -1, 0, None, None, seed, 0)
        keep = []
        if U0 is not None:
            u = np.asfortranarray(U0, dtype=np.float64)
            w = np.asfortranarray(W0, dtype=np.float64)
            keep += [u, w]
            prm.U0 = u.ctypes.data
            prm.W0 = w.ctypes.data
        return prm, keep

    def submit(self, t, r, r3, precision=PREC_MIXED, U0=None, W0=None, p=4, s=2, tol=0.0,
               max_outer=0, seed=0, coo=None):
        """Submit a solve of tensor `t`, or of host coordinates `coo` (then t
        is None and the server uploads after admission).  Returns the id."""
        m, n = (t.m, t.n) if t is not None else (coo.m, coo.n)
        prm, keep = self._params(r, r3, precision, U0, W0, p, s, tol, max_outer, seed)
        U = np.zeros((m, r), order="F")
        W = np.zeros((n, r3), order="F")
        F = np.zeros((r, r, r3), order="F")
        rid = C.c_uint64()
        if t is not None:
            rc = self.lib.bks_server_submit(self.h, t.h, C.byref(prm), _ptr(U), _ptr(W), _ptr(F),
                                            C.byref(rid))
        else:
            i = np.ascontiguousarray(coo.i, np.int32)
            j = np.ascontiguousarray(coo.j, np.int32)
            k = np.ascontiguousarray(coo.k, np.int32)
            v = np.ascontiguousarray(coo.val, np.float32)
            rc = self.lib.bks_server_submit_coo(self.h, m, n, int(i.shape[0]), _ptr(i), _ptr(j),
                                                _ptr(k), _ptr(v), C.byref(prm), _ptr(U), _ptr(W),
                                                _ptr(F), C.byref(rid))
        if rc != OK:
            raise BksError(rc, "submit refused")
        # the tensor must outlive the request: hold it with the outputs
        self._out[rid.value] = (U, W, F, (keep, t))
        return rid.value

    def poll(self, rid):
        res = Result()
        self.ctx.check(self.lib.bks_server_poll(self.h, rid, C.byref(res)))
        return res

    def wait(self, rid):
        """Block until done; returns (U, W, F, result)."""
        res = Result()
        self.ctx.check(self.lib.bks_server_wait(self.h, rid, C.byref(res)))
        U, W, F, _ = self._out.pop(rid)
        return U, W, F, res

    def cancel(self, rid):
        """bks_server_cancel: returns the status code (0 taken or pending,
        ENOTFOUND, EINVAL if the request had finished)."""
        return self.lib.bks_server_cancel(self.h, rid)

    def now(self):
        return self.lib.bks_server_now(self.h)

    def close(self):
        if self.h:
            self.lib.bks_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tensor:
    def __init__(self, ctx: Ctx, h):
        self.ctx = ctx
        self.h = h
        m, n, nnz, npairs = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        fro = C.c_double()
        db = C.c_size_t()
        ctx.lib.bks_tensor_info(h, C.byref(m), C.byref(n), C.byref(nnz), C.byref(npairs),
                                C.byref(fro), C.byref(db))
        self.m, self.n, self.nnz, self.npairs = m.value, n.value, nnz.value, npairs.value
        self.frob = fro.value
        self.dev_bytes = db.value

    def pairs(self):
        pi = np.zeros(self.npairs, np.int32)
        pj = np.zeros(self.npairs, np.int32)
        self.ctx.check(self.ctx.lib.bks_tensor_pairs(self.h, pi.ctypes.data_as(C.POINTER(C.c_int32)),
                                                     pj.ctypes.data_as(C.POINTER(C.c_int32))))
        return pi, pj

    def free(self):
        if self.h:
            self.ctx.lib.bks_tensor_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

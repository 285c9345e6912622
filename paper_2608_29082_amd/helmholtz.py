"""Python binding of the complex Helmholtz entry points of libmgl.so (the C
ABI declared in include/mgh.h).

Argument marshalling only: every numerical step runs in the HIP library.
Complex vectors are torch complex tensors of shape (n, B) (complex64 for FP32
cycles, complex128 for FP64 cycles and solver-level vectors), whose memory
is the (real, imaginary) interleaved [n][B] layout the library expects.
There is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import binding as Bd

SMOOTHERS = {"jacobi": 0, "gmres": 1}
EXPORTED = ["mgh_num_params", "mgh_setup", "mgh_set_params", "mgh_vcycle", "mgh_fmg", "mgh_residual",
            "mgh_fgmres", "mgh_solve", "mgh_level_info", "mgh_destroy", "mgh_last_error"]


class _CCSR(C.Structure):
    _fields_ = [("nrows", C.c_int32), ("ncols", C.c_int32), ("nnz", C.c_int64),
                ("rowptr", C.POINTER(C.c_int32)), ("col", C.POINTER(C.c_int32)),
                ("re", C.POINTER(C.c_double)), ("im", C.POINTER(C.c_double))]


class _HHier(C.Structure):
    _fields_ = [("nlevels", C.c_int32), ("A", C.POINTER(_CCSR)), ("P", C.POINTER(Bd._CSR)),
                ("R", C.POINTER(Bd._CSR))]


class _HParams(C.Structure):
    _fields_ = [("KB", C.c_int32), ("KR", C.c_int32), ("KP", C.c_int32), ("smoother", C.POINTER(C.c_int32)),
                ("nu_pre", C.POINTER(C.c_int32)), ("nu_post", C.POINTER(C.c_int32)),
                ("gmres_steps", C.c_int32), ("values", C.POINTER(C.c_double))]


class _HOptions(C.Structure):
    _fields_ = [("precision", C.c_int32), ("nrhs", C.c_int32)]


_ready = False


def load_library():
    global _ready
    lib = Bd.load_library()
    if _ready:
        return lib
    vp = C.c_void_p
    lib.mgh_num_params.restype = C.c_int64
    lib.mgh_num_params.argtypes = [C.c_int32] * 4
    lib.mgh_setup.argtypes = [C.POINTER(_HHier), C.POINTER(_HParams), C.POINTER(_HOptions), vp, C.POINTER(vp)]
    lib.mgh_set_params.argtypes = [vp, C.POINTER(C.c_double), vp]
    lib.mgh_vcycle.argtypes = [vp, vp, vp, vp]
    lib.mgh_fmg.argtypes = [vp, vp, vp, vp]
    lib.mgh_residual.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.mgh_fgmres.argtypes = [vp, vp, vp, C.POINTER(Bd._KrylovOptions), C.POINTER(Bd.RhsInfo), vp]
    lib.mgh_solve.argtypes = [vp, vp, vp, C.c_double, C.c_int32, C.c_int32, C.POINTER(Bd.RhsInfo), vp]
    lib.mgh_level_info.argtypes = [vp, C.POINTER(C.c_int64)]
    lib.mgh_destroy.argtypes = [vp]
    lib.mgh_destroy.restype = None
    lib.mgh_last_error.restype = C.c_char_p
    for name in ("mgh_setup", "mgh_set_params", "mgh_vcycle", "mgh_fmg", "mgh_residual", "mgh_fgmres",
                 "mgh_solve", "mgh_level_info"):
        getattr(lib, name).restype = C.c_int
    _ready = True
    return lib


def _check(lib, status: int, what: str):
    if status != 0:
        raise Bd.MGError(status, f"{what}: {lib.mgh_last_error().decode()}")


def num_params(J: int, KB: int, KR: int, KP: int) -> int:
    return int(load_library().mgh_num_params(J, KB, KR, KP))


class _Host:
    """ctypes descriptors of a complex hierarchy (keeps the arrays alive)."""

    def __init__(self, A, P, R=None):
        self._keep = []
        J = len(A)
        arr = (_CCSR * J)()
        for k, m in enumerate(A):
            m = m.tocsr()
            m.sort_indices()
            rp = np.ascontiguousarray(m.indptr, dtype=np.int32)
            ci = np.ascontiguousarray(m.indices, dtype=np.int32)
            re = np.ascontiguousarray(m.data.real, dtype=np.float64)
            im = np.ascontiguousarray(m.data.imag, dtype=np.float64)
            self._keep += [rp, ci, re, im]
            arr[k] = _CCSR(m.shape[0], m.shape[1], m.nnz, rp.ctypes.data_as(C.POINTER(C.c_int32)),
                           ci.ctypes.data_as(C.POINTER(C.c_int32)), re.ctypes.data_as(C.POINTER(C.c_double)),
                           im.ctypes.data_as(C.POINTER(C.c_double)))
        self._keep.append(arr)
        Pa = self._real(P)
        Ra = self._real(R) if R is not None else C.POINTER(Bd._CSR)()
        self.h = _HHier(J, arr, Pa, Ra)

    def _real(self, mats):
        arr = (Bd._CSR * len(mats))()
        for k, m in enumerate(mats):
            m = m.tocsr()
            m.sort_indices()
            rp = np.ascontiguousarray(m.indptr, dtype=np.int32)
            ci = np.ascontiguousarray(m.indices, dtype=np.int32)
            va = np.ascontiguousarray(m.data, dtype=np.float64)
            self._keep += [rp, ci, va]
            arr[k] = Bd._CSR(m.shape[0], m.shape[1], m.nnz, rp.ctypes.data_as(C.POINTER(C.c_int32)),
                             ci.ctypes.data_as(C.POINTER(C.c_int32)), va.ctypes.data_as(C.POINTER(C.c_double)))
        self._keep.append(arr)
        return arr


class HelmholtzContext:
    """A set-up two-feature learnable V-cycle for complex A u = f on one GPU.

    A: complex scipy matrices (levels 0..J-1); P: real prolongations;
    plan: per level l < J-1 (kind, nu_pre, nu_post) with kind "jacobi" or
    "gmres"; params: flat float64 vector (include/mgh.h layout); v: GMRES
    steps of a GMRES smoothing step; precision "fp64" or "fp32".
    """

    def __init__(self, A, P, params, KB, KR, KP, plan, v=4, precision="fp64", nrhs=1, R=None, device=None,
                 stream=None):
        import torch
        self.torch = torch
        self.lib = load_library()
        self.device = torch.device(device or "cuda")
        self.J = len(A)
        self.n = [a.shape[0] for a in A]
        self.B = nrhs
        self.KB, self.KR, self.KP = KB, KR, KP
        self.precision = precision
        self.cycle_dtype = torch.complex128 if precision == "fp64" else torch.complex64
        self.nparams = num_params(self.J, KB, KR, KP)
        self._params = np.ascontiguousarray(params, dtype=np.float64)
        if self._params.size != self.nparams:
            raise ValueError(f"expected {self.nparams} parameters, got {self._params.size}")
        self._sm = np.ascontiguousarray([SMOOTHERS[p[0]] for p in plan], dtype=np.int32)
        self._pre = np.ascontiguousarray([p[1] for p in plan], dtype=np.int32)
        self._post = np.ascontiguousarray([p[2] for p in plan], dtype=np.int32)
        ip = C.POINTER(C.c_int32)
        self._p = _HParams(KB, KR, KP, self._sm.ctypes.data_as(ip), self._pre.ctypes.data_as(ip),
                           self._post.ctypes.data_as(ip), v, self._params.ctypes.data_as(C.POINTER(C.c_double)))
        self._o = _HOptions(Bd.PRECISIONS[precision], nrhs)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        host = _Host(A, P, R)
        h = C.c_void_p()
        _check(self.lib, self.lib.mgh_setup(C.byref(host.h), C.byref(self._p), C.byref(self._o), self._s(),
                                            C.byref(h)), "mgh_setup")
        self._h = h

    def _s(self):
        return C.c_void_p(self.stream.cuda_stream)

    def _vec(self, t, dtype, name):
        if (t.device.type != "cuda" or t.dtype != dtype or not t.is_contiguous()
                or tuple(t.shape) != (self.n[0], self.B)):
            raise ValueError(f"{name}: expected contiguous {dtype} CUDA tensor of shape ({self.n[0]}, {self.B}), "
                             f"got {t.dtype} {tuple(t.shape)} on {t.device}")
        return t

    def empty(self, dtype=None):
        return self.torch.empty((self.n[0], self.B), dtype=dtype or self.cycle_dtype, device=self.device)

    def set_params(self, values):
        self._params = np.ascontiguousarray(values, dtype=np.float64)
        if self._params.size != self.nparams:
            raise ValueError("wrong parameter count")
        self._p.values = self._params.ctypes.data_as(C.POINTER(C.c_double))
        _check(self.lib, self.lib.mgh_set_params(self._h, self._params.ctypes.data_as(C.POINTER(C.c_double)),
                                                 self._s()), "mgh_set_params")

    def vcycle(self, f, u):
        """u <- LMG(A, f, u) in place (cycle dtype)."""
        self._vec(f, self.cycle_dtype, "f")
        self._vec(u, self.cycle_dtype, "u")
        _check(self.lib, self.lib.mgh_vcycle(self._h, f.data_ptr(), u.data_ptr(), self._s()), "mgh_vcycle")
        return u

    def fmg(self, f, u):
        self._vec(f, self.cycle_dtype, "f")
        self._vec(u, self.cycle_dtype, "u")
        _check(self.lib, self.lib.mgh_fmg(self._h, f.data_ptr(), u.data_ptr(), self._s()), "mgh_fmg")
        return u

    def residual(self, f, u, want_r=True):
        c128 = self.torch.complex128
        self._vec(f, c128, "f")
        self._vec(u, c128, "u")
        r = self.empty(c128) if want_r else None
        norms = self.torch.empty(self.B, dtype=self.torch.float64, device=self.device)
        _check(self.lib, self.lib.mgh_residual(self._h, f.data_ptr(), u.data_ptr(),
                                               None if r is None else r.data_ptr(), norms.data_ptr(), self._s()),
               "mgh_residual")
        return r, norms

    def fgmres(self, f, u, restart=30, max_iter=200, rtol=1e-8, precond="vcycle", reorth=None,
               raise_on_failure=False) -> Bd.SolveInfo:
        c128 = self.torch.complex128
        self._vec(f, c128, "f")
        self._vec(u, c128, "u")
        o = Bd._KrylovOptions(restart, max_iter, rtol, Bd.PRECONDITIONERS[precond],
                              Bd.REORTH_DEFAULT if reorth is None else reorth)
        info = (Bd.RhsInfo * self.B)()
        st = self.lib.mgh_fgmres(self._h, f.data_ptr(), u.data_ptr(), C.byref(o), info, self._s())
        if st not in (0, 5, 6) or (raise_on_failure and st != 0):
            _check(self.lib, st, "mgh_fgmres")
        return Bd.SolveInfo(np.array([x.iters for x in info]), np.array([x.status for x in info]),
                            np.array([x.relres for x in info]), st)

    def solve(self, f, u, rtol=1e-8, max_cycles=1000, check_every=5, raise_on_failure=False) -> Bd.SolveInfo:
        """Stationary iteration u <- LMG(A, f, u) per column to rtol (FP64 contexts)."""
        c128 = self.torch.complex128
        self._vec(f, c128, "f")
        self._vec(u, c128, "u")
        info = (Bd.RhsInfo * self.B)()
        st = self.lib.mgh_solve(self._h, f.data_ptr(), u.data_ptr(), rtol, max_cycles, check_every, info, self._s())
        if st not in (0, 5, 6) or (raise_on_failure and st != 0):
            _check(self.lib, st, "mgh_solve")
        return Bd.SolveInfo(np.array([x.iters for x in info]), np.array([x.status for x in info]),
                            np.array([x.relres for x in info]), st)

    def level_info(self):
        n = (C.c_int64 * self.J)()
        _check(self.lib, self.lib.mgh_level_info(self._h, n), "mgh_level_info")
        return list(n)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.mgh_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def from_workload(w, precision="fp64", params=None, **kw) -> HelmholtzContext:
    """Context for a Helmholtz workload object (hier, plan, K orders, v)."""
    return HelmholtzContext(w.hier.A, w.hier.P, w.params if params is None else params, w.KB, w.KR, w.KP,
                            w.plan, v=w.v, precision=precision, nrhs=w.B, **kw)

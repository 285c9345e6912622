"""Python binding of libmgl.so (the C ABI declared in include/mgl.h).

Argument marshalling only: every numerical step runs in the HIP library.
Device vectors are torch tensors (torch supplies device memory and streams);
the hierarchy is handed over as host CSR arrays (scipy matrices).  There is no
CPU fallback: if the library cannot be loaded, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmgl.so")

STATUS = {0: "MG_OK", 1: "MG_ERR_INVALID_ARG", 2: "MG_ERR_SHAPE", 3: "MG_ERR_OOM", 4: "MG_ERR_HIP",
          5: "MG_ERR_NOT_CONVERGED", 6: "MG_ERR_DIVERGED", 7: "MG_ERR_STATE", 8: "MG_ERR_UNSUPPORTED"}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2}
BASES = {"monomial": 0, "chebyshev": 1}
AGGREGATIONS = {"mean": 0, "weighted": 1, "sym": 2}
FLAG_BACKWARD = 1
FLAG_NO_TAIL = 2
FLAG_NO_TILES = 4
FLAG_NO_COMPACT = 8

EXPORTED = ["mg_num_params", "mg_workspace_bytes", "mg_setup", "mg_set_params", "mg_vcycle",
            "mg_vcycle_backward", "mg_residual", "mg_residual_loss", "mg_refine_step", "mg_refine_step_backward",
            "mg_solve", "mg_level_info", "mg_timing_start", "mg_timing_read", "mg_square_hierarchy",
            "mg_host_hierarchy_view", "mg_host_hierarchy_free", "mg_destroy", "mg_last_error",
            "mg_fmg", "mg_fgmres_workspace_bytes", "mg_fgmres", "mg_fgmres_static", "mg_load_column",
            "mg_set_solver_options"]
KERNEL_FAMILIES = {"hop": 1, "resid": 2, "restrict": 3, "prolong": 4, "outer": 5, "krylov": 6, "conv": 7}
PRECONDITIONERS = {"none": 0, "vcycle": 1, "fmg": 2}
LOSS_KINDS = {"mean_rel_sq": 0, "resid_norm": 1}
# default threshold of the second Gram-Schmidt pass: run it for a vector when
# the first pass left less than a tenth of its norm (orthogonality to about
# ten units of roundoff per vector; 1/sqrt 2 is the "twice is enough" bound)
REORTH_DEFAULT = 0.1


class MGError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class _CSR(C.Structure):
    _fields_ = [("nrows", C.c_int32), ("ncols", C.c_int32), ("nnz", C.c_int64),
                ("rowptr", C.POINTER(C.c_int32)), ("col", C.POINTER(C.c_int32)),
                ("val", C.POINTER(C.c_double))]


class _Hier(C.Structure):
    _fields_ = [("nlevels", C.c_int32), ("A", C.POINTER(_CSR)), ("P", C.POINTER(_CSR)),
                ("R", C.POINTER(_CSR)), ("G", C.POINTER(_CSR)), ("ncolumn_values", C.c_int32),
                ("column_values", C.POINTER(C.POINTER(C.c_double)))]


class _Params(C.Structure):
    _fields_ = [("KB", C.c_int32), ("KR", C.c_int32), ("KP", C.c_int32), ("nu_pre", C.c_int32),
                ("nu_post", C.c_int32), ("values", C.POINTER(C.c_double)), ("basis", C.c_int32),
                ("aggregation", C.c_int32)]


class _Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("nrhs", C.c_int32), ("max_outer", C.c_int32),
                ("check_every", C.c_int32), ("rtol", C.c_double), ("diverge_factor", C.c_double),
                ("flags", C.c_int32)]


class _KrylovOptions(C.Structure):
    _fields_ = [("restart", C.c_int32), ("max_iter", C.c_int32), ("rtol", C.c_double), ("precond", C.c_int32),
                ("reorth", C.c_double)]


class RhsInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32), ("relres", C.c_double)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libmgl.so once; raises if it is missing (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is not built; run `python -m paper_2608_29082_amd.build`")
    lib = C.CDLL(path)
    vp, sz = C.c_void_p, C.c_size_t
    lib.mg_num_params.restype = C.c_int64
    lib.mg_num_params.argtypes = [C.c_int32] * 4
    lib.mg_workspace_bytes.argtypes = [C.POINTER(_Hier), C.POINTER(_Params), C.POINTER(_Options),
                                       C.POINTER(sz), C.POINTER(sz)]
    lib.mg_setup.argtypes = [C.POINTER(_Hier), C.POINTER(_Params), C.POINTER(_Options), vp, sz, vp,
                             C.POINTER(vp)]
    lib.mg_set_params.argtypes = [vp, C.POINTER(C.c_double), vp]
    lib.mg_load_column.argtypes = [vp, C.c_int32, C.POINTER(C.POINTER(C.c_double)), vp]
    lib.mg_set_solver_options.argtypes = [vp, C.c_int32, C.c_int32, C.c_double, C.c_double]
    lib.mg_vcycle.argtypes = [vp, vp, vp, vp, vp]
    lib.mg_vcycle_backward.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.mg_residual.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.mg_refine_step.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.mg_residual_loss.argtypes = [vp, C.c_int32, vp, vp, vp, vp, vp, vp, vp]
    lib.mg_refine_step_backward.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.mg_solve.argtypes = [vp, vp, vp, C.POINTER(RhsInfo), vp]
    lib.mg_level_info.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int32)]
    lib.mg_fmg.argtypes = [vp, vp, vp, vp]
    lib.mg_fgmres_workspace_bytes.argtypes = [vp, C.POINTER(_KrylovOptions), C.POINTER(sz)]
    lib.mg_fgmres.argtypes = [vp, vp, vp, C.POINTER(_KrylovOptions), vp, sz, C.POINTER(RhsInfo), vp]
    lib.mg_fgmres_static.argtypes = [vp, vp, vp, C.POINTER(_KrylovOptions), C.POINTER(RhsInfo), vp]
    lib.mg_timing_start.argtypes = [vp, C.c_int32, C.c_int32]
    lib.mg_timing_read.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.mg_square_hierarchy.argtypes = [C.c_int32, C.c_int32, C.POINTER(C.c_double), C.c_int32, C.POINTER(vp)]
    lib.mg_square_hierarchy.restype = C.c_int
    lib.mg_host_hierarchy_view.argtypes = [vp, C.POINTER(_Hier)]
    lib.mg_host_hierarchy_view.restype = C.c_int
    lib.mg_host_hierarchy_free.argtypes = [vp]
    lib.mg_host_hierarchy_free.restype = None
    lib.mg_destroy.argtypes = [vp]
    lib.mg_destroy.restype = None
    lib.mg_last_error.restype = C.c_char_p
    for name in ("mg_workspace_bytes", "mg_setup", "mg_set_params", "mg_load_column", "mg_set_solver_options",
                 "mg_vcycle", "mg_vcycle_backward",
                 "mg_residual", "mg_residual_loss", "mg_refine_step", "mg_refine_step_backward", "mg_solve", "mg_level_info",
                 "mg_timing_start", "mg_timing_read"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _check(status: int, what: str = ""):
    if status != 0:
        msg = _lib.mg_last_error().decode() if _lib is not None else ""
        raise MGError(status, f"{what}: {msg}")


def num_params(nlevels: int, KB: int, KR: int, KP: int) -> int:
    return int(load_library().mg_num_params(nlevels, KB, KR, KP))


class _HostHierarchy:
    """Keeps the numpy arrays behind the ctypes CSR descriptors alive."""

    def __init__(self, A, P, R=None, G=None):
        self._keep = []
        J = len(A)
        self.A = self._csr_array(A)
        self.P = self._csr_array(P)
        self.R = self._csr_array(R) if R is not None else None
        self.G = self._csr_array(G, pattern=True) if G is not None else None
        self.h = _Hier(J, self.A, self.P, self.R if self.R is not None else C.POINTER(_CSR)(),
                       self.G if self.G is not None else C.POINTER(_CSR)())

    def _csr_array(self, mats, pattern=False):
        arr = (_CSR * len(mats))()
        for k, m in enumerate(mats):
            m = m.tocsr()
            rp = np.ascontiguousarray(m.indptr, dtype=np.int32)
            ci = np.ascontiguousarray(m.indices, dtype=np.int32)
            va = np.ascontiguousarray(m.data, dtype=np.float64)
            self._keep += [rp, ci, va]
            arr[k] = _CSR(m.shape[0], m.shape[1], m.nnz,
                          rp.ctypes.data_as(C.POINTER(C.c_int32)), ci.ctypes.data_as(C.POINTER(C.c_int32)),
                          va.ctypes.data_as(C.POINTER(C.c_double)))
        self._keep.append(arr)
        return arr


def _level_values(src):
    """Per-level pointers to the CSR values of a column's operators: src is a
    SquareHierarchy (native arrays, no copy) or a list of scipy matrices A_l.
    Returns (pointer list, objects to keep alive)."""
    if isinstance(src, SquareHierarchy):
        return [src.view.A[l].val for l in range(src.nlevels)], [src]
    keep, ptrs = [], []
    for a in src:
        v = np.ascontiguousarray(a.tocsr().data, dtype=np.float64)
        keep.append(v)
        ptrs.append(v.ctypes.data_as(C.POINTER(C.c_double)))
    return ptrs, keep


def _level_nnz(src):
    if isinstance(src, SquareHierarchy):
        return [int(src.view.A[l].nnz) for l in range(src.nlevels)]
    return [int(a.nnz) for a in src]


class SquareHierarchy:
    """Native structured hierarchy (mg_square_hierarchy): host CSR levels owned
    by the library, usable directly by Context(native=...)."""

    def __init__(self, side: int, blocks, coarsest: int = 3):
        lib = load_library()
        b = np.ascontiguousarray(blocks, dtype=np.float64)
        nb = b.shape[0]
        h = C.c_void_p()
        st = lib.mg_square_hierarchy(side, nb, b.ctypes.data_as(C.POINTER(C.c_double)), coarsest, C.byref(h))
        if st != 0:
            raise MGError(st, f"mg_square_hierarchy(side={side})")
        self._h = h
        self._lib = lib
        self.view = _Hier()
        _check(lib.mg_host_hierarchy_view(h, C.byref(self.view)), "mg_host_hierarchy_view")
        self.nlevels = self.view.nlevels
        self.sizes = [self.view.A[l].nrows for l in range(self.nlevels)]

    def to_scipy(self):
        """Copies of the levels as scipy CSR matrices (A list, P list)."""
        import scipy.sparse as sp

        def conv(m):
            rp = np.ctypeslib.as_array(m.rowptr, shape=(m.nrows + 1,)).copy()
            ci = np.ctypeslib.as_array(m.col, shape=(max(m.nnz, 1),))[:m.nnz].copy()
            va = np.ctypeslib.as_array(m.val, shape=(max(m.nnz, 1),))[:m.nnz].copy()
            return sp.csr_matrix((va, ci, rp), shape=(m.nrows, m.ncols))
        J = self.nlevels
        return [conv(self.view.A[l]) for l in range(J)], [conv(self.view.P[l]) for l in range(J - 1)]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.mg_host_hierarchy_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


@dataclass
class SolveInfo:
    iters: np.ndarray
    status: np.ndarray
    relres: np.ndarray
    code: int


class Context:
    """A set-up learnable V-cycle on one GPU (wraps mg_ctx).

    A, P: lists of scipy sparse matrices (levels 0..J-1, 0 finest);
    params: flat float64 parameter vector; precision: "fp64", "fp32" or "bf16";
    basis: "monomial" or "chebyshev" (meaning of the convolution coefficients);
    aggregation: "mean", "weighted" (|a_ij| edge weights) or "sym" (symmetric
    normalisation), the graph operator of the convolutions.
    tail / tiles: allow the LDS-resident coarse tail / the fused K-hop
    convolution over LDS tiles (FP32/BF16 cycles with nrhs a multiple of 16).
    compact: let solve() narrow the cycle to the columns still iterating.
    columns: per-column operators (a batch of requests on one grid): a list of
    nrhs sources, each a SquareHierarchy or a list of scipy A_l on the pattern
    of the given A (or native) hierarchy; column b then solves with its own
    A_l^(b) (mg_hierarchy.ncolumn_values).
    """

    def __init__(self, A, P, params, KB, KR, KP, nu_pre=2, nu_post=2, precision="fp64", nrhs=1,
                 R=None, G=None, rtol=1e-8, max_outer=10000, check_every=10, diverge_factor=1e6,
                 backward=False, device=None, stream=None, workspace=True, tail=True, native=None,
                 basis="monomial", aggregation="mean", tiles=True, compact=True, columns=None):
        import torch
        self.torch = torch
        self.lib = load_library()
        self.device = torch.device(device or "cuda")
        self.KB, self.KR, self.KP = KB, KR, KP
        self.nu_pre, self.nu_post = nu_pre, nu_post
        self.precision = precision
        self.B = nrhs
        if native is not None:
            self.J = native.nlevels
            self.n = list(native.sizes)

            class _View:
                h = native.view
            self._hh = _View()
        else:
            self.J = len(A)
            self.n = [a.shape[0] for a in A]
            self._hh = _HostHierarchy(A, P, R, G)
        self.cycle_dtype = torch.float64 if precision == "fp64" else torch.float32
        self.nparams = num_params(self.J, KB, KR, KP)
        self._params = np.ascontiguousarray(params, dtype=np.float64)
        if self._params.size != self.nparams:
            raise ValueError(f"expected {self.nparams} parameters, got {self._params.size}")
        self.basis, self.aggregation = basis, aggregation
        self._p = _Params(KB, KR, KP, nu_pre, nu_post, self._params.ctypes.data_as(C.POINTER(C.c_double)),
                          BASES[basis], AGGREGATIONS[aggregation])
        self._o = _Options(PRECISIONS[precision], nrhs, max_outer, check_every, rtol, diverge_factor,
                           (FLAG_BACKWARD if backward else 0) | (0 if tail else FLAG_NO_TAIL) |
                           (0 if tiles else FLAG_NO_TILES) | (0 if compact else FLAG_NO_COMPACT))
        self._colkeep = None
        self.nnz = [int(self._hh.h.A[l].nnz) for l in range(self.J)]
        if columns is not None:
            if len(columns) != nrhs:
                raise ValueError("columns: one operator source per right-hand side")
            arr = (C.POINTER(C.c_double) * (self.J * nrhs))()
            keep = [arr]
            for b, src in enumerate(columns):
                if _level_nnz(src) != self.nnz:
                    raise ValueError(f"columns[{b}]: pattern sizes differ from the context's")
                ptrs, k = _level_values(src)
                if len(ptrs) != self.J:
                    raise ValueError("columns: wrong level count")
                keep += k
                for l in range(self.J):
                    arr[l * nrhs + b] = ptrs[l]
            hh = _Hier()
            C.memmove(C.byref(hh), C.byref(self._hh.h), C.sizeof(_Hier))
            hh.ncolumn_values = nrhs
            hh.column_values = arr
            self._colkeep = (hh, keep, self._hh)

            class _ColView:
                h = hh
            self._hh = _ColView()
        ws, ck = C.c_size_t(), C.c_size_t()
        _check(self.lib.mg_workspace_bytes(C.byref(self._hh.h), C.byref(self._p), C.byref(self._o),
                                           C.byref(ws), C.byref(ck)), "mg_workspace_bytes")
        self.workspace_bytes, self.ckpt_bytes = ws.value, ck.value
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device) if workspace else None
        h = C.c_void_p()
        _check(self.lib.mg_setup(C.byref(self._hh.h), C.byref(self._p), C.byref(self._o),
                                 _ptr(self._ws), self.workspace_bytes, self._s(), C.byref(h)), "mg_setup")
        self._h = h
        self._hh = None   # the library copied what it needs
        self._colkeep = None

    # ------------------------------------------------------------------ helpers
    def _s(self):
        return C.c_void_p(self.stream.cuda_stream)

    def _vec(self, t, dtype, name, n=None):
        n = self.n[0] if n is None else n
        if t is None:
            return None
        if t.device.type != "cuda" or t.dtype != dtype or not t.is_contiguous() or tuple(t.shape) != (n, self.B):
            raise ValueError(f"{name}: expected contiguous {dtype} CUDA tensor of shape ({n}, {self.B}), "
                             f"got {t.dtype} {tuple(t.shape)} on {t.device}")
        return t

    def empty(self, dtype=None):
        return self.torch.empty((self.n[0], self.B), dtype=dtype or self.cycle_dtype, device=self.device)

    def new_ckpt(self):
        return self.torch.empty(self.ckpt_bytes, dtype=self.torch.uint8, device=self.device)

    # ------------------------------------------------------------------ entry points
    def set_params(self, values):
        self._params = np.ascontiguousarray(values, dtype=np.float64)
        if self._params.size != self.nparams:
            raise ValueError("wrong parameter count")
        _check(self.lib.mg_set_params(self._h, self._params.ctypes.data_as(C.POINTER(C.c_double)), self._s()),
               "mg_set_params")

    def load_column(self, b: int, src):
        """mg_load_column: column b solves with the operators of `src` from now on
        (a SquareHierarchy or a list of scipy A_l on the context's pattern)."""
        nnz = _level_nnz(src)
        if nnz != self.nnz:
            raise ValueError(f"load_column: the source's pattern sizes {nnz} differ from the context's {self.nnz}")
        ptrs, keep = _level_values(src)
        arr = (C.POINTER(C.c_double) * len(ptrs))(*ptrs)
        _check(self.lib.mg_load_column(self._h, b, arr, self._s()), "mg_load_column")

    def set_solver_options(self, max_outer=None, check_every=None, rtol=None, diverge_factor=None):
        o = self._o
        o.max_outer = o.max_outer if max_outer is None else max_outer
        o.check_every = o.check_every if check_every is None else check_every
        o.rtol = o.rtol if rtol is None else rtol
        o.diverge_factor = o.diverge_factor if diverge_factor is None else diverge_factor
        _check(self.lib.mg_set_solver_options(self._h, o.max_outer, o.check_every, o.rtol, o.diverge_factor),
               "mg_set_solver_options")

    @property
    def params(self):
        return self._params.copy()

    def vcycle(self, f, u, ckpt=None):
        """u <- LMG(A, f, u) in place (cycle dtype)."""
        self._vec(f, self.cycle_dtype, "f")
        self._vec(u, self.cycle_dtype, "u")
        _check(self.lib.mg_vcycle(self._h, _ptr(f), _ptr(u), _ptr(ckpt), self._s()), "mg_vcycle")
        return u

    def vcycle_backward(self, ckpt, gu_out, want_gu=True, want_gf=True, want_gp=True):
        self._vec(gu_out, self.cycle_dtype, "gu_out")
        gu = self.empty() if want_gu else None
        gf = self.empty() if want_gf else None
        gp = self.torch.empty(self.nparams, dtype=self.torch.float64, device=self.device) if want_gp else None
        _check(self.lib.mg_vcycle_backward(self._h, _ptr(ckpt), _ptr(gu_out), _ptr(gu), _ptr(gf), _ptr(gp),
                                           self._s()), "mg_vcycle_backward")
        return gu, gf, gp

    def residual(self, f, u, want_r=True):
        self._vec(f, self.torch.float64, "f")
        self._vec(u, self.torch.float64, "u")
        r = self.empty(self.torch.float64) if want_r else None
        norms = self.torch.empty(self.B, dtype=self.torch.float64, device=self.device)
        _check(self.lib.mg_residual(self._h, _ptr(f), _ptr(u), _ptr(r), _ptr(norms), self._s()), "mg_residual")
        return r, norms

    def residual_loss(self, f, u, kind="mean_rel_sq", gseed=None, want_loss=True, want_gu=False, want_gf=False):
        """mg_residual_loss: (loss [1], dL/du, dL/df) as device float64 tensors (None
        where not requested).  kind "mean_rel_sq": mean_b ||r_b||^2/||f_b||^2;
        "resid_norm": sum_b ||r_b||_2.  gseed: device float64 tensor [1] scaling
        both gradients (None: 1)."""
        self._vec(f, self.torch.float64, "f")
        self._vec(u, self.torch.float64, "u")
        if gseed is not None and (gseed.device.type != "cuda" or gseed.dtype != self.torch.float64
                                  or gseed.numel() != 1 or not gseed.is_contiguous()):
            raise ValueError("gseed: expected a contiguous float64 CUDA tensor with one element")
        loss = self.torch.empty(1, dtype=self.torch.float64, device=self.device) if want_loss else None
        gu = self.empty(self.torch.float64) if want_gu else None
        gf = self.empty(self.torch.float64) if want_gf else None
        _check(self.lib.mg_residual_loss(self._h, LOSS_KINDS[kind], _ptr(f), _ptr(u), _ptr(gseed), _ptr(loss),
                                         _ptr(gu), _ptr(gf), self._s()), "mg_residual_loss")
        return loss, gu, gf

    def refine_step(self, f, u_in, u_out=None, ckpt=None):
        self._vec(f, self.torch.float64, "f")
        self._vec(u_in, self.torch.float64, "u_in")
        if u_out is None:
            u_out = self.empty(self.torch.float64)
        self._vec(u_out, self.torch.float64, "u_out")
        _check(self.lib.mg_refine_step(self._h, _ptr(f), _ptr(u_in), _ptr(u_out), _ptr(ckpt), self._s()),
               "mg_refine_step")
        return u_out

    def refine_step_backward(self, ckpt, gu_out, want_gu=True, want_gf=True, want_gp=True):
        self._vec(gu_out, self.torch.float64, "gu_out")
        gu = self.empty(self.torch.float64) if want_gu else None
        gf = self.empty(self.torch.float64) if want_gf else None
        gp = self.torch.empty(self.nparams, dtype=self.torch.float64, device=self.device) if want_gp else None
        _check(self.lib.mg_refine_step_backward(self._h, _ptr(ckpt), _ptr(gu_out), _ptr(gu), _ptr(gf), _ptr(gp),
                                                self._s()), "mg_refine_step_backward")
        return gu, gf, gp

    def solve(self, f, u, raise_on_failure=False) -> SolveInfo:
        self._vec(f, self.torch.float64, "f")
        self._vec(u, self.torch.float64, "u")
        info = (RhsInfo * self.B)()
        st = self.lib.mg_solve(self._h, _ptr(f), _ptr(u), info, self._s())
        if st not in (0, 5, 6) or (raise_on_failure and st != 0):
            _check(st, "mg_solve")
        return SolveInfo(np.array([x.iters for x in info]), np.array([x.status for x in info]),
                         np.array([x.relres for x in info]), st)

    def fmg(self, f, u):
        """u = FMG(f): nested iteration with one learnable cycle per level (cycle dtype)."""
        self._vec(f, self.cycle_dtype, "f")
        self._vec(u, self.cycle_dtype, "u")
        _check(self.lib.mg_fmg(self._h, _ptr(f), _ptr(u), self._s()), "mg_fmg")
        return u

    def fgmres_workspace_bytes(self, restart=30, precond="vcycle"):
        o = _KrylovOptions(restart, 1, 0.0, PRECONDITIONERS[precond], REORTH_DEFAULT)
        b = C.c_size_t()
        _check(self.lib.mg_fgmres_workspace_bytes(self._h, C.byref(o), C.byref(b)), "mg_fgmres_workspace_bytes")
        return b.value

    def fgmres(self, f, u, restart=30, max_iter=500, rtol=None, precond="vcycle", work=None, reorth=None,
               raise_on_failure=False) -> SolveInfo:
        """Flexible GMRES(restart) from u with the cycle (or FMG) as right preconditioner;
        iters counts FGMRES iterations per column.  work: optional uint8 device tensor
        of fgmres_workspace_bytes (else the library keeps its own).  reorth: second
        Gram-Schmidt pass threshold (default 0.1; 1/sqrt 2 "twice is enough"; 0 never,
        >= 1 always)."""
        self._vec(f, self.torch.float64, "f")
        self._vec(u, self.torch.float64, "u")
        o = _KrylovOptions(restart, max_iter, self._o.rtol if rtol is None else rtol, PRECONDITIONERS[precond],
                           REORTH_DEFAULT if reorth is None else reorth)
        info = (RhsInfo * self.B)()
        st = self.lib.mg_fgmres(self._h, _ptr(f), _ptr(u), C.byref(o), _ptr(work),
                                0 if work is None else work.numel(), info, self._s())
        if st not in (0, 5, 6) or (raise_on_failure and st != 0):
            _check(st, "mg_fgmres")
        return SolveInfo(np.array([x.iters for x in info]), np.array([x.status for x in info]),
                         np.array([x.relres for x in info]), st)

    def fgmres_static(self, f, u, restart=30, max_iter=500, rtol=None, precond="vcycle", reorth=None,
                      raise_on_failure=False) -> SolveInfo:
        """mg_fgmres_static: fgmres with the library's static per-GPU workspace
        (no device allocation; calls on one GPU must not overlap)."""
        self._vec(f, self.torch.float64, "f")
        self._vec(u, self.torch.float64, "u")
        o = _KrylovOptions(restart, max_iter, self._o.rtol if rtol is None else rtol, PRECONDITIONERS[precond],
                           REORTH_DEFAULT if reorth is None else reorth)
        info = (RhsInfo * self.B)()
        st = self.lib.mg_fgmres_static(self._h, _ptr(f), _ptr(u), C.byref(o), info, self._s())
        if st not in (0, 5, 6) or (raise_on_failure and st != 0):
            _check(st, "mg_fgmres_static")
        return SolveInfo(np.array([x.iters for x in info]), np.array([x.status for x in info]),
                         np.array([x.relres for x in info]), st)

    def level_info(self):
        n = (C.c_int64 * self.J)()
        w = (C.c_int32 * self.J)()
        _check(self.lib.mg_level_info(self._h, n, w), "mg_level_info")
        return list(n), list(w)

    def timing_start(self, family: str | None, level: int = -1):
        """Time every launch of one kernel family on one level (-1: all levels)."""
        _check(self.lib.mg_timing_start(self._h, KERNEL_FAMILIES[family] if family else 0, level),
               "mg_timing_start")

    def timing_read(self):
        """(launches, total_ms, total_algorithmic_bytes) of the timed family."""
        n, ms, by = C.c_int64(), C.c_double(), C.c_double()
        _check(self.lib.mg_timing_read(self._h, C.byref(n), C.byref(ms), C.byref(by)), "mg_timing_read")
        return n.value, ms.value, by.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.mg_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def from_hierarchy(hier, params, KB, KR, KP, **kw) -> Context:
    """Context from an object with A, P, R lists (e.g. a generated hierarchy)."""
    return Context(hier.A, hier.P, params, KB, KR, KP, R=getattr(hier, "R", None), **kw)

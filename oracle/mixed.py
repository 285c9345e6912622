"""Mixed-precision emulation of the learnable V-cycle -- TEST INFRASTRUCTURE ONLY.

Only the tests (and the benchmark's CPU-baseline leg) may import this module;
the GPU product path never calls it.  The parity target of every cycle stays
the FP64 oracle (oracle/lmg.py); this module predicts what the mixed-precision
solver does with its roundings, so that its iteration counts and its FP32
error are checked against something other than the GPU itself.

The solver of the stationary iteration u^m = u^{m-1} + B(f - A u^{m-1})
(Sec. 1) in refinement form: the residual f - A u, its norms and the update
are FP64; the correction B r is one learnable V-cycle (Alg. 2) from a zero
iterate computed in FP32 on fl32(r).  The cycle here is Alg. 2 in the paper's
order with every vector a float32 array (NumPy rounds each operation to
float32; SciPy's sparse products accumulate in float32), the coarsest level
solved with the FP64 inverse of A_J and rounded back to float32, and, for the
BF16-storage variant, the intermediates that the solver keeps in bfloat16
rounded to nearest-even bfloat16 where they are stored:
  * the Jacobi-scaled residual s = D^{-1}(f - A u) that enters Phi_B,
  * the output of Phi_R before the restriction R,
  * the interpolated correction P e_c before Phi_P,
on the levels listed in `bf16_levels` (the solver stores them so on the levels
whose convolutions run over LDS tiles; its LDS-resident coarse levels keep
FP32), while the convolution's hops, sums and updates stay float32.
Operation orders inside sums and fused multiply-adds are not reproduced: the
emulation agrees with any FP32 execution to a few units of float32 round-off
per operation, not bit for bit.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .lmg import OLevel, OParams, SolveResult


# ----------------------------------------------------------------------------- bfloat16
def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), returned as
    float32.  bfloat16 keeps the float32 sign and 8-bit exponent and the top 7
    fraction bits: add half an ulp of the kept part (0x7fff, plus one when the
    kept part is odd, which breaks ties towards even) and clear the low 16 bits.
    A NaN stays a (quiet) NaN; a carry out of the largest finite binade gives
    infinity, as rounding to nearest requires."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    bits = a.view(np.uint32).astype(np.uint64)
    nan = (bits & 0x7FFFFFFF) > 0x7F800000
    rounded = (bits + 0x7FFF + ((bits >> 16) & 1)) & 0xFFFF0000
    rounded = np.where(nan, (bits | 0x00400000) & 0xFFFF0000, rounded)
    return (rounded & 0xFFFFFFFF).astype(np.uint32).view(np.float32).reshape(a.shape)


# ----------------------------------------------------------------------------- float32 levels
@dataclass
class MLevel:
    A: sp.csr_matrix          # float32 copy of A_l
    Dinv: np.ndarray          # float32 1 / diag(A_l)
    G: sp.csr_matrix          # float32 0/1 graph (or the aggregation operator when Gw is set)
    inv_deg: np.ndarray | None   # float32 1/|N(i)| (None when G is an explicit aggregation operator)
    P: sp.csr_matrix | None
    R: sp.csr_matrix | None
    Ainv: np.ndarray | None   # FP64 inverse of the coarsest operator


def make_levels32(levels: list[OLevel]) -> list[MLevel]:
    """float32 copies of an oracle hierarchy (values rounded once, as the
    solver's FP32 copies are made at setup)."""
    out = []
    J = len(levels)
    for l, lv in enumerate(levels):
        f32 = lambda m: None if m is None else sp.csr_matrix(m, dtype=np.float32)
        if lv.Gw is not None:
            G, inv_deg = f32(lv.Gw), None
        else:
            G, inv_deg = f32(lv.G), lv.inv_deg.astype(np.float32)
        Ainv = np.linalg.inv(lv.A.toarray()) if l == J - 1 else None
        out.append(MLevel(f32(lv.A), lv.Dinv.astype(np.float32), G, inv_deg, f32(lv.P), f32(lv.R), Ainv))
    return out


def _mean32(lv: MLevel, y: np.ndarray) -> np.ndarray:
    if lv.inv_deg is None:
        return (lv.G @ y).astype(np.float32)
    return lv.inv_deg[:, None] * (lv.G @ y)


def graph_conv32(c: np.ndarray, lv: MLevel, x: np.ndarray) -> np.ndarray:
    """sum_k c_k M^k x by Horner's rule in float32 (power-series coefficients)."""
    c32 = np.asarray(c, dtype=np.float64).astype(np.float32)
    K = len(c32) - 1
    y = c32[K] * x
    for k in range(K - 1, -1, -1):
        y = _mean32(lv, y) + c32[k] * x
    return y.astype(np.float32)


def lmg32(levels: list[MLevel], prm: OParams, l: int, f: np.ndarray, u: np.ndarray | None,
          bf16_levels=()) -> np.ndarray:
    """Alg. 2 in float32 from the iterate u (None: zero), with the stored
    intermediates of the levels in bf16_levels rounded to bfloat16."""
    J = len(levels)
    lv = levels[l]
    f = np.asarray(f, dtype=np.float32)
    if l == J - 1:
        return (lv.Ainv @ f.astype(np.float64)).astype(np.float32)
    store = bf16_round if l in bf16_levels else (lambda v: v)
    scale = np.float32(prm.eta[l] * prm.theta[l])

    def smooth(u):
        r = f if u is None else f - lv.A @ u
        s = store(lv.Dinv[:, None] * r)
        w = scale * graph_conv32(prm.cB[l], lv, s)
        return w if u is None else u + w

    for _ in range(prm.nu_pre):
        u = smooth(u)
    r = f if u is None else f - lv.A @ u
    y = store(graph_conv32(prm.cR[l], lv, r))
    rc = (lv.R @ y).astype(np.float32)
    ec = lmg32(levels, prm, l + 1, rc, None, bf16_levels)
    x = store((lv.P @ ec).astype(np.float32))
    e = graph_conv32(prm.cP[l], lv, x)
    u = e if u is None else u + e
    for _ in range(prm.nu_post):
        u = smooth(u)
    return u.astype(np.float32)


def fmg32(levels: list[MLevel], prm: OParams, f: np.ndarray, bf16_levels=()) -> np.ndarray:
    """Full multigrid with one cycle per level (the oracle's fmg) in float32."""
    J = len(levels)
    fs = [np.asarray(f, dtype=np.float32)]
    for l in range(J - 1):
        store = bf16_round if l in bf16_levels else (lambda v: v)
        fs.append((levels[l].R @ store(graph_conv32(prm.cR[l], levels[l], fs[-1]))).astype(np.float32))
    u = lmg32(levels, prm, J - 1, fs[J - 1], None, bf16_levels)
    for l in range(J - 2, -1, -1):
        store = bf16_round if l in bf16_levels else (lambda v: v)
        u = graph_conv32(prm.cP[l], levels[l], store((levels[l].P @ u).astype(np.float32)))
        u = lmg32(levels, prm, l, fs[l], u, bf16_levels)
    return u


def solve_mixed(levels: list[OLevel], prm: OParams, f: np.ndarray, rtol: float = 1e-8,
                max_cycles: int = 10000, bf16_levels=(), levels32: list[MLevel] | None = None) -> SolveResult:
    """The refinement-form solver: per column, r = f - A u (FP64), stop at the
    first iterate with ||r|| <= rtol ||f||, else u += LMG_32(A, fl32(r), 0)."""
    A = levels[0].A
    lv32 = levels32 if levels32 is not None else make_levels32(levels)
    f = np.asarray(f, dtype=np.float64)
    u = np.zeros_like(f)
    fn = np.linalg.norm(f, axis=0)
    fn_safe = np.where(fn > 0, fn, 1.0)
    active = np.ones(f.shape[1], dtype=bool)
    iters = np.zeros(f.shape[1], dtype=np.int64)
    hist = []
    for _ in range(max_cycles):
        r = f - A @ u
        rel = np.linalg.norm(r, axis=0) / fn_safe
        hist.append(rel)
        active &= rel > rtol
        if not active.any():
            break
        idx = np.flatnonzero(active)
        e = lmg32(lv32, prm, 0, r[:, idx].astype(np.float32), None, bf16_levels)
        u[:, idx] += e.astype(np.float64)
        iters[idx] += 1
    rel = np.linalg.norm(f - A @ u, axis=0) / fn_safe
    return SolveResult(u, iters, rel, hist, rel <= rtol)

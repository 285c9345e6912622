"""FGMRES with the learnable cycle as preconditioner, and full multigrid -- TEST INFRASTRUCTURE ONLY.

The paper also uses the trained cycle as a preconditioner of flexible GMRES,
with a V-cycle or with full multigrid (nested iteration: start on the
coarsest level, interpolate, one V-cycle per level, using the same transfer
operators as the V-cycle) (Sec. 4.2, FGMRES and FMG paragraphs).  Plain NumPy
FP64, restated from the published algorithms (Saad's flexible GMRES with
right preconditioning and restarts, Givens rotations; nested iteration);
columns of f are solved independently.
"""
from __future__ import annotations

import numpy as np

from .lmg import OLevel, OParams, coarse_solve, graph_conv, lmg


def fmg(levels: list[OLevel], prm: OParams, f: np.ndarray) -> np.ndarray:
    """Full multigrid for A_0 u = f with one learnable V-cycle per level.

    Right-hand sides are carried down with the cycle's restriction
    f_{l+1} = R_l Phi_R,l(f_l); the coarsest level is solved exactly; each
    finer level starts from Phi_P,l(P_l u_{l+1}) and applies one LMG cycle.
    """
    J = len(levels)
    fs = [f]
    for l in range(J - 1):
        fs.append(levels[l].R @ graph_conv(prm.cR[l], levels[l], fs[-1], prm.basis))
    u = coarse_solve(levels[J - 1], fs[J - 1])
    for l in range(J - 2, -1, -1):
        u = graph_conv(prm.cP[l], levels[l], levels[l].P @ u, prm.basis)
        u = lmg(levels, prm, l, fs[l], u)
    return u


def fgmres(levels, prm: OParams, f: np.ndarray, restart: int = 20, rtol: float = 1e-8, max_iter: int = 1000,
           precond: str = "vcycle", A=None):
    """Flexible GMRES(restart) per column, right preconditioning z = C(v) with
    C one learnable V-cycle from zero ("vcycle"), full multigrid ("fmg"), the
    identity ("none") or the exact inverse ("exact").  Returns (u, iters,
    relres per column, residual-estimate history of column 0)."""
    A = levels[0].A if A is None else A
    n, B = f.shape
    if precond == "vcycle":
        C = lambda v: lmg(levels, prm, 0, v, np.zeros_like(v))
    elif precond == "fmg":
        C = lambda v: fmg(levels, prm, v)
    elif precond == "none":
        C = lambda v: v.copy()
    elif precond == "exact":
        Ad = A.toarray()
        C = lambda v: np.linalg.solve(Ad, v)
    else:
        raise ValueError(precond)
    u = np.zeros_like(f)
    iters = np.zeros(B, dtype=np.int64)
    relres = np.zeros(B)
    hist0 = []
    for b in range(B):
        x = np.zeros((n, 1))
        rhs = f[:, b:b + 1]
        bn = np.linalg.norm(rhs)
        if bn == 0:
            continue
        it = 0
        while it < max_iter:
            r = rhs - A @ x
            beta = np.linalg.norm(r)
            if beta <= rtol * bn:
                break
            V = [r / beta]
            Z = []
            H = np.zeros((restart + 1, restart))
            cs, sn = np.zeros(restart), np.zeros(restart)
            g = np.zeros(restart + 1)
            g[0] = beta
            j_done = 0
            for j in range(restart):
                z = C(V[j])
                Z.append(z)
                w = A @ z
                for i in range(j + 1):                  # modified Gram-Schmidt
                    H[i, j] = float(np.sum(w * V[i]))
                    w = w - H[i, j] * V[i]
                H[j + 1, j] = np.linalg.norm(w)
                V.append(w / H[j + 1, j] if H[j + 1, j] > 0 else w)
                for i in range(j):                      # previous rotations
                    t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                    H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                    H[i, j] = t
                d = np.hypot(H[j, j], H[j + 1, j])
                cs[j], sn[j] = H[j, j] / d, H[j + 1, j] / d
                H[j, j] = d
                H[j + 1, j] = 0.0
                g[j + 1] = -sn[j] * g[j]
                g[j] = cs[j] * g[j]
                it += 1
                j_done = j + 1
                if b == 0:
                    hist0.append(abs(g[j + 1]) / bn)
                if abs(g[j + 1]) <= rtol * bn or it >= max_iter:
                    break
            y = np.linalg.solve(np.triu(H[:j_done, :j_done]), g[:j_done])
            for k in range(j_done):
                x = x + y[k] * Z[k]
        u[:, b:b + 1] = x
        iters[b] = it
        relres[b] = np.linalg.norm(rhs - A @ x) / bn
    return u, iters, relres, hist0

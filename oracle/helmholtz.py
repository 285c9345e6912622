"""CPU complex128 oracle of the learnable V-cycle for the Helmholtz problem
(two features per node) -- TEST INFRASTRUCTURE ONLY.

Only the tests, the package's smoke check and the benchmark's CPU-baseline leg
may import this module.  The GPU product path never calls it.

Plain NumPy/SciPy code written from the paper:
  * complex solutions are carried as d = 2 node features (real part, imaginary
    part), and every graph convolution mixes them with 2 x 2 real weight
    matrices (Sec. 4.2, Helmholtz subsection: feature dimension 2, W_1 = I and
    W_2 = 0 at initialisation, off-diagonal entries trainable).  A convolution
    of order K is  Phi(x) = sum_k W_k (M^k x)  with M = D_g^{-1} A_g the
    neighbour mean acting on nodes and W_k acting on the two features of every
    node (K = 1 is SAGEConv with mean aggregation, Sec. 3.2; the K-order form is
    the polynomial-smoother remark of Sec. 3.3).  M and the W_k commute, so it
    is evaluated by Horner's rule  y = W_K x;  y <- M y + W_k x.
  * Jacobi smoothing (Sec. 3, learnable smoother with B_l = D_A^{-1}, the
    complex diagonal of A_l):  delta = theta D_A^{-1} (f - A u),
    u <- u + eta Phi_B(delta).
  * GMRES smoothing (Sec. 3, the Krylov-smoother form): the convolution makes
    the initial guess of v GMRES steps on A delta = r,
        r = f - A u,  delta_0 = theta Phi_B(r),
        u <- u + eta GMRES(A, r, delta_0, v).
    GMRES(A, r, x0, v) is the iterate of v steps of (unrestarted) GMRES with
    initial guess x0: x0 + V_v y with V_v an orthonormal basis of the Krylov
    space K_v(A, r - A x0) (Arnoldi, modified Gram-Schmidt, Hermitian inner
    product) and y minimising || beta e_1 - H y ||; a zero Arnoldi remainder
    (an invariant Krylov space) ends the steps early.
  * restriction r_c = R_l Phi_R(r) and prolongation u += Phi_P(P_l e_c) with
    Phi_R and Phi_P shared by all levels (Sec. 4.2, Helmholtz subsection);
  * the learnable V-cycle (Alg. 2) with per-level smoother kind and step
    counts, exact coarsest solve by dense complex LU;
  * full multigrid with one cycle per level and flexible GMRES with the cycle
    or FMG as right preconditioner (Sec. 4.2, FGMRES and FMG paragraphs),
    complex (Saad's FGMRES, Givens rotations).
Vectors are (n, B) complex arrays; the columns are independent.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


# ----------------------------------------------------------------------------- levels
@dataclass
class HLevel:
    A: sp.csr_matrix          # complex system matrix A_l
    Dinv: np.ndarray          # 1 / diag(A_l) (complex)
    M: sp.csr_matrix          # neighbour mean D_g^{-1} A_g on the graph of A_l
    P: sp.csr_matrix | None   # prolongation to this level from the next coarser one
    R: sp.csr_matrix | None   # restriction from this level to the next coarser one
    lu: tuple | None = None   # dense LU factors (coarsest level only)


def neighbour_mean(A: sp.csr_matrix) -> sp.csr_matrix:
    """M = D_g^{-1} A_g for the graph {(i, j): A_ij != 0, i != j} (Sec. 2.1)."""
    C = sp.coo_matrix(A)
    keep = (C.row != C.col) & (C.data != 0)
    n = A.shape[0]
    G = sp.csr_matrix((np.ones(int(keep.sum())), (C.row[keep], C.col[keep])), shape=(n, n))
    deg = np.asarray(G.sum(axis=1)).ravel()
    return sp.csr_matrix(sp.diags(np.where(deg > 0, 1.0 / np.where(deg > 0, deg, 1.0), 0.0)) @ G)


def make_levels(A_list, P_list, R_list=None) -> list[HLevel]:
    J = len(A_list)
    out = []
    for l in range(J):
        A = sp.csr_matrix(A_list[l]).astype(np.complex128)
        d = A.diagonal()
        Dinv = np.where(d != 0, 1.0 / np.where(d != 0, d, 1.0), 0.0)
        P = P_list[l] if l < J - 1 else None
        R = (R_list[l] if R_list is not None else sp.csr_matrix(P_list[l].T)) if l < J - 1 else None
        lu = sla.lu_factor(A.toarray()) if l == J - 1 else None
        out.append(HLevel(A, Dinv, neighbour_mean(A), P, R, lu))
    return out


# ----------------------------------------------------------------------------- parameters
@dataclass
class HParams:
    theta: np.ndarray          # [J-1]
    eta: np.ndarray            # [J-1]
    WB: list                   # [J-1] arrays (KB+1, 2, 2)
    WR: np.ndarray             # (KR+1, 2, 2), shared by all levels
    WP: np.ndarray             # (KP+1, 2, 2), shared by all levels
    plan: list                 # [J-1] (kind, nu_pre, nu_post), kind "jacobi" | "gmres"
    v: int = 4                 # GMRES steps of a GMRES smoothing step


def n_params(J: int, KB: int, KR: int, KP: int) -> int:
    return (J - 1) * (2 + 4 * (KB + 1)) + 4 * (KR + 1) + 4 * (KP + 1)


def unpack(flat, J: int, KB: int, KR: int, KP: int, plan, v: int = 4) -> HParams:
    """Flat layout: per level l < J-1  [theta_l, eta_l, W_B,l[0..KB] (2 x 2
    row-major each)], then W_R[0..KR], then W_P[0..KP]."""
    flat = np.asarray(flat, dtype=np.float64)
    assert flat.size == n_params(J, KB, KR, KP)
    per = 2 + 4 * (KB + 1)
    lv = flat[:(J - 1) * per].reshape(J - 1, per)
    rest = flat[(J - 1) * per:]
    return HParams(lv[:, 0].copy(), lv[:, 1].copy(),
                   [lv[l, 2:].reshape(KB + 1, 2, 2).copy() for l in range(J - 1)],
                   rest[:4 * (KR + 1)].reshape(KR + 1, 2, 2).copy(),
                   rest[4 * (KR + 1):].reshape(KP + 1, 2, 2).copy(), list(plan), v)


# ----------------------------------------------------------------------------- building blocks
def mix(W: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Apply the 2 x 2 real matrix W to the features (Re x, Im x) of every node."""
    xr, xi = x.real, x.imag
    return (W[0, 0] * xr + W[0, 1] * xi) + 1j * (W[1, 0] * xr + W[1, 1] * xi)


def conv(W: np.ndarray, lev: HLevel, x: np.ndarray) -> np.ndarray:
    """sum_k W_k (M^k x) by Horner's rule (W: (K+1, 2, 2))."""
    K = W.shape[0] - 1
    y = mix(W[K], x)
    for k in range(K - 1, -1, -1):
        y = (lev.M @ y) + mix(W[k], x)
    return y


def gmres_steps(A, r: np.ndarray, x0: np.ndarray, v: int) -> np.ndarray:
    """v steps of GMRES on A x = r from x0, column by column (module doc)."""
    out = np.array(x0, dtype=np.complex128, copy=True)
    for b in range(r.shape[1]):
        r0 = r[:, b] - A @ x0[:, b]
        beta = np.linalg.norm(r0)
        if beta == 0.0:
            continue
        V = [r0 / beta]
        H = np.zeros((v + 1, v), dtype=np.complex128)
        m = v
        for j in range(v):
            w = A @ V[j]
            for i in range(j + 1):
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] == 0.0:
                m = j + 1
                break
            V.append(w / H[j + 1, j])
        e1 = np.zeros(m + 1, dtype=np.complex128)
        e1[0] = beta
        y = np.linalg.lstsq(H[:m + 1, :m], e1, rcond=None)[0]
        out[:, b] = x0[:, b] + np.stack(V[:m], axis=1) @ y
    return out


def smooth(lev: HLevel, prm: HParams, l: int, f: np.ndarray, u: np.ndarray) -> np.ndarray:
    kind = prm.plan[l][0]
    r = f - lev.A @ u
    if kind == "jacobi":
        delta = prm.theta[l] * (lev.Dinv[:, None] * r)
        return u + prm.eta[l] * conv(prm.WB[l], lev, delta)
    if kind == "gmres":
        d0 = prm.theta[l] * conv(prm.WB[l], lev, r)
        return u + prm.eta[l] * gmres_steps(lev.A, r, d0, prm.v)
    raise ValueError(kind)


def coarse_solve(lev: HLevel, f: np.ndarray) -> np.ndarray:
    return sla.lu_solve(lev.lu, f)


def lmg(levels: list[HLevel], prm: HParams, l: int, f: np.ndarray, u: np.ndarray) -> np.ndarray:
    """One learnable V-cycle on level l (Alg. 2 with per-level smoothers)."""
    J = len(levels)
    lev = levels[l]
    if l == J - 1:
        return coarse_solve(lev, f)
    u = np.array(u, dtype=np.complex128, copy=True)
    for _ in range(prm.plan[l][1]):
        u = smooth(lev, prm, l, f, u)
    r = f - lev.A @ u
    rc = lev.R @ conv(prm.WR, lev, r)
    ec = lmg(levels, prm, l + 1, rc, np.zeros_like(rc))
    u = u + conv(prm.WP, lev, lev.P @ ec)
    for _ in range(prm.plan[l][2]):
        u = smooth(lev, prm, l, f, u)
    return u


def fmg(levels: list[HLevel], prm: HParams, f: np.ndarray) -> np.ndarray:
    """Full multigrid: f_{l+1} = R_l Phi_R(f_l); exact coarsest solve; on each
    finer level one cycle from Phi_P(P_l u_{l+1})."""
    J = len(levels)
    fs = [f]
    for l in range(J - 1):
        fs.append(levels[l].R @ conv(prm.WR, levels[l], fs[-1]))
    u = coarse_solve(levels[J - 1], fs[J - 1])
    for l in range(J - 2, -1, -1):
        u = conv(prm.WP, levels[l], levels[l].P @ u)
        u = lmg(levels, prm, l, fs[l], u)
    return u


def fgmres(levels, prm: HParams, f: np.ndarray, restart: int = 30, rtol: float = 1e-8, max_iter: int = 1000,
           precond: str = "vcycle"):
    """Complex flexible GMRES(restart) per column with right preconditioning
    z = C(v): one cycle from zero ("vcycle"), full multigrid ("fmg"), the
    identity ("none") or the exact inverse ("exact").  A restart starts from
    the true residual; a column stops at the first iteration whose residual
    estimate |g_{j+1}| meets rtol ||f|| and is done when its true residual
    does.  Returns (u, iters, relres per column, estimate history of column 0)."""
    A = levels[0].A
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
    u = np.zeros((n, B), dtype=np.complex128)
    iters = np.zeros(B, dtype=np.int64)
    relres = np.zeros(B)
    hist0 = []
    for b in range(B):
        x = np.zeros((n, 1), dtype=np.complex128)
        rhs = f[:, b:b + 1].astype(np.complex128)
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
            H = np.zeros((restart + 1, restart), dtype=np.complex128)
            cs = np.zeros(restart)
            sn = np.zeros(restart, dtype=np.complex128)
            g = np.zeros(restart + 1, dtype=np.complex128)
            g[0] = beta
            j_done = 0
            for j in range(restart):
                z = C(V[j])
                Z.append(z)
                w = A @ z
                for i in range(j + 1):                  # modified Gram-Schmidt
                    H[i, j] = np.vdot(V[i], w)
                    w = w - H[i, j] * V[i]
                H[j + 1, j] = np.linalg.norm(w)
                V.append(w / H[j + 1, j] if abs(H[j + 1, j]) > 0 else w)
                for i in range(j):                      # earlier rotations
                    t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                    H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
                    H[i, j] = t
                # complex Givens rotation: [c s; -conj(s) c] [a; b] = [rho; 0], c real
                a, bb = H[j, j], H[j + 1, j]
                d = np.hypot(abs(a), abs(bb))
                if abs(a) == 0:
                    cs[j], sn[j] = 0.0, 1.0
                else:
                    cs[j] = abs(a) / d
                    sn[j] = (a / abs(a)) * np.conj(bb) / d
                H[j, j] = cs[j] * a + sn[j] * bb
                H[j + 1, j] = 0.0
                g[j + 1] = -np.conj(sn[j]) * g[j]
                g[j] = cs[j] * g[j]
                it += 1
                j_done = j + 1
                if b == 0:
                    hist0.append(abs(g[j + 1]) / bn)
                if abs(g[j + 1]) <= rtol * bn or it >= max_iter:
                    break
            y = sla.solve_triangular(np.triu(H[:j_done, :j_done]), g[:j_done])
            for k in range(j_done):
                x = x + y[k] * Z[k]
        u[:, b:b + 1] = x
        iters[b] = it
        relres[b] = np.linalg.norm(rhs - A @ x) / bn
    return u, iters, relres, hist0

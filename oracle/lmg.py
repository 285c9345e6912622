"""CPU FP64 oracle of the learnable V-cycle -- TEST INFRASTRUCTURE ONLY.

Only the tests, the package's smoke check and the benchmark's CPU-baseline leg
may import this module.  The GPU product path never calls it.

Plain, slow, obviously-correct NumPy/SciPy code written from the paper:
  * neighbour mean  M = D_g^{-1} A_g  on the graph of A_l (Sec. 2.1; Sec. 3.2
    SAGEConv with mean aggregation; Sec. 3.3 eq. (graph-conv-matrix)),
  * a graph convolution of order K as the polynomial  sum_k c_k M^k x
    (K = 1 is SAGEConv with w1 = c_0, w2 = c_1; Sec. 3.3 remark on
    polynomial smoothers for the K-order case), evaluated by Horner's rule,
  * the learnable V-cycle LMG (Alg. 2) with B_l = D_A^{-1} (damped-Jacobi
    smoother of Sec. 2.3, eq. for the Jacobi update),
  * the classical V-cycle MG (Alg. 1), written separately,
  * the stationary iteration u^m = u^{m-1} + B (f - A u^{m-1}) with per-column
    stopping (Sec. 1).
Variants of the convolution (Sec. 3.2, other operators such as ChebConv;
Sec. 2.1, edge weights that encode matrix entries):
  * aggregation "weighted": G = D_w^{-1} W with W_ij = |A_ij| on the graph
    (|G_ij| for a given weighted graph), D_w = diag(sum_j W_ij);
  * aggregation "sym": G = D_g^{-1/2} A_g D_g^{-1/2} (the symmetric
    normalisation of the ChebConv layer);
  * basis "chebyshev": Phi(x) = sum_k c_k T_k(-G) x, T_k the Chebyshev
    polynomials evaluated by their three-term recurrence (the ChebConv layer
    with the rescaled Laplacian 2 L / lambda_max - I, L = I - G, lambda_max = 2).
Vectors are (n, B) arrays: B independent right-hand sides side by side.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


# ----------------------------------------------------------------------------- levels
@dataclass
class OLevel:
    A: sp.csr_matrix          # system matrix A_l
    Dinv: np.ndarray          # 1 / diag(A_l)
    G: sp.csr_matrix          # graph adjacency A_g (0/1), directed pairs stored both ways
    inv_deg: np.ndarray       # 1/|N(i)|, 0 for an isolated node
    P: sp.csr_matrix | None   # prolongation to this level from the next coarser one
    R: sp.csr_matrix | None   # restriction from this level to the next coarser one
    lu: tuple | None = None   # dense LU factors (coarsest level only)
    Gw: sp.csr_matrix | None = None   # aggregation operator for "weighted" / "sym" (None: mean)


def algebraic_graph(A: sp.csr_matrix) -> sp.csr_matrix:
    """E = {(i, j): A_ij != 0, i != j} (Sec. 2.1, algebraic construction)."""
    C = sp.coo_matrix(A)
    keep = (C.row != C.col) & (C.data != 0.0)
    n = A.shape[0]
    return sp.csr_matrix((np.ones(int(keep.sum())), (C.row[keep], C.col[keep])), shape=(n, n))


def aggregation_operator(A: sp.csr_matrix, G: sp.csr_matrix, Graw, aggregation: str):
    """The explicit operator G for the non-mean aggregations (see module doc)."""
    n = A.shape[0]
    if aggregation == "weighted":
        src = sp.coo_matrix(A if Graw is None else Graw)
        keep = (src.row != src.col) & (src.data != 0.0)
        W = sp.csr_matrix((np.abs(src.data[keep]), (src.row[keep], src.col[keep])), shape=(n, n))
        rs = np.asarray(W.sum(axis=1)).ravel()
        return sp.csr_matrix(sp.diags(np.where(rs > 0, 1.0 / np.where(rs > 0, rs, 1.0), 0.0)) @ W)
    if aggregation == "sym":
        deg = np.asarray(G.sum(axis=1)).ravel()
        isd = np.where(deg > 0, 1.0 / np.sqrt(np.where(deg > 0, deg, 1.0)), 0.0)
        return sp.csr_matrix(sp.diags(isd) @ G @ sp.diags(isd))
    raise ValueError(aggregation)


def make_levels(A_list, P_list, R_list=None, G_list=None, ghost_degree=None,
                aggregation: str = "mean") -> list[OLevel]:
    """Bundle a hierarchy.  R defaults to P^T (Sec. 2.2).  G defaults to the
    algebraic graph of A_l.  ghost_degree, if given, overrides |N(i)| by a
    constant (used only by the closed-form eigenvalue check).  aggregation:
    "mean" (default), "weighted" or "sym" (module doc)."""
    J = len(A_list)
    levels = []
    for l in range(J):
        A = sp.csr_matrix(A_list[l], dtype=np.float64)
        if G_list is None or G_list[l] is None:
            G = algebraic_graph(A)
        else:
            # a given pattern: its edges join distinct nodes, so the diagonal is not an edge
            Gc = sp.coo_matrix(G_list[l])
            off = Gc.row != Gc.col
            G = sp.csr_matrix((np.ones(int(off.sum())), (Gc.row[off], Gc.col[off])), shape=A.shape)
        G = sp.csr_matrix((np.ones(G.nnz), G.indices, G.indptr), shape=G.shape)
        deg = np.asarray(G.sum(axis=1)).ravel()
        if ghost_degree is not None:
            deg = np.full_like(deg, float(ghost_degree))
        inv_deg = np.where(deg > 0, 1.0 / np.where(deg > 0, deg, 1.0), 0.0)
        P = sp.csr_matrix(P_list[l]) if l < J - 1 else None
        if l < J - 1:
            R = sp.csr_matrix(P.T) if R_list is None or R_list[l] is None else sp.csr_matrix(R_list[l])
        else:
            R = None
        lu = sla.lu_factor(A.toarray()) if l == J - 1 else None
        Gw = None
        if aggregation != "mean":
            Graw = None if G_list is None or G_list[l] is None else sp.csr_matrix(G_list[l], dtype=np.float64)
            Gw = aggregation_operator(A, G, Graw, aggregation)
        levels.append(OLevel(A, 1.0 / A.diagonal(), G, inv_deg, P, R, lu, Gw))
    return levels


# ----------------------------------------------------------------------------- parameters
@dataclass
class OParams:
    theta: np.ndarray   # [J-1]
    eta: np.ndarray     # [J-1]
    cB: np.ndarray      # [J-1, KB+1]
    cR: np.ndarray      # [J-1, KR+1]
    cP: np.ndarray      # [J-1, KP+1]
    nu_pre: int = 2
    nu_post: int = 2
    basis: str = "monomial"   # or "chebyshev"


def unpack(flat, J: int, KB: int, KR: int, KP: int, nu_pre: int = 2, nu_post: int = 2,
           basis: str = "monomial") -> OParams:
    """Flat layout per level l: [theta, eta, cB[0..KB], cR[0..KR], cP[0..KP]]."""
    per = 2 + KB + 1 + KR + 1 + KP + 1
    p = np.asarray(flat, dtype=np.float64).reshape(J - 1, per)
    o = 2
    cB = p[:, o:o + KB + 1]; o += KB + 1
    cR = p[:, o:o + KR + 1]; o += KR + 1
    cP = p[:, o:o + KP + 1]
    return OParams(p[:, 0].copy(), p[:, 1].copy(), cB.copy(), cR.copy(), cP.copy(), nu_pre, nu_post, basis)


def pack(p: OParams) -> np.ndarray:
    return np.concatenate([p.theta[:, None], p.eta[:, None], p.cB, p.cR, p.cP], axis=1).ravel()


# ----------------------------------------------------------------------------- operators
def neighbour_mean(lv: OLevel, x: np.ndarray) -> np.ndarray:
    """(M x)_i = mean of x_j over j in N(i); 0 when N(i) is empty.  With a
    non-mean aggregation, the level's aggregation operator applied to x."""
    if lv.Gw is not None:
        return lv.Gw @ x
    return lv.inv_deg[:, None] * (lv.G @ x)


def graph_conv(c: np.ndarray, lv: OLevel, x: np.ndarray, basis: str = "monomial") -> np.ndarray:
    """Phi(x) = sum_{k=0..K} c_k M^k x, by Horner: y = c_K x; y = M y + c_k x.
    basis "chebyshev": Phi(x) = sum_k c_k T_k(-M) x with T_0 x = x,
    T_1 = -M x, T_{k+1} = -2 M T_k - T_{k-1}."""
    K = len(c) - 1
    if basis == "chebyshev":
        t_prev, t = x, -neighbour_mean(lv, x)
        y = c[0] * t_prev + (c[1] * t if K >= 1 else 0.0)
        for k in range(1, K):
            t_prev, t = t, -2.0 * neighbour_mean(lv, t) - t_prev
            y = y + c[k + 1] * t
        return y
    y = c[K] * x
    for k in range(K - 1, -1, -1):
        y = neighbour_mean(lv, y) + c[k] * x
    return y


def residual(lv: OLevel, f: np.ndarray, u: np.ndarray) -> np.ndarray:
    return f - lv.A @ u


def coarse_solve(lv: OLevel, f: np.ndarray) -> np.ndarray:
    """Exact solve A_J u = f by dense LU with partial pivoting."""
    return sla.lu_solve(lv.lu, f)


def smooth(lv: OLevel, l: int, prm: OParams, f, u):
    """delta = theta_l D_A^{-1} (f - A_l u);  u <- u + eta_l Phi_B(delta)."""
    delta = prm.theta[l] * (lv.Dinv[:, None] * residual(lv, f, u))
    return u + prm.eta[l] * graph_conv(prm.cB[l], lv, delta, prm.basis)


def lmg(levels: list[OLevel], prm: OParams, l: int, f: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Learnable V-cycle u = LMG(A_l, f, u, l, Theta) (Alg. 2); l = 0 is finest."""
    J = len(levels)
    lv = levels[l]
    if l == J - 1:
        return coarse_solve(lv, f)
    for _ in range(prm.nu_pre):
        u = smooth(lv, l, prm, f, u)
    r = residual(lv, f, u)
    rc = lv.R @ graph_conv(prm.cR[l], lv, r, prm.basis)
    ec = np.zeros((levels[l + 1].A.shape[0], f.shape[1]))
    ec = lmg(levels, prm, l + 1, rc, ec)
    e = graph_conv(prm.cP[l], lv, lv.P @ ec, prm.basis)
    u = u + e
    for _ in range(prm.nu_post):
        u = smooth(lv, l, prm, f, u)
    return u


def classical_mg(levels: list[OLevel], omega: float, nu: int, l: int, f, u):
    """Classical V-cycle MG (Alg. 1) with damped Jacobi B_l = omega D_A^{-1}."""
    J = len(levels)
    lv = levels[l]
    A = lv.A
    if l == J - 1:
        return np.linalg.solve(A.toarray(), f)
    d = A.diagonal()[:, None]
    for _ in range(nu):
        u = u + omega * (f - A @ u) / d
    rc = lv.R @ (f - A @ u)
    ec = classical_mg(levels, omega, nu, l + 1, rc, np.zeros((rc.shape[0], f.shape[1])))
    u = u + lv.P @ ec
    for _ in range(nu):
        u = u + omega * (f - A @ u) / d
    return u


# ----------------------------------------------------------------------------- solver
@dataclass
class SolveResult:
    u: np.ndarray
    iters: np.ndarray        # cycles applied per column
    relres: np.ndarray       # final ||f - A u|| / ||f|| per column
    history: list            # relres per cycle (array over columns)
    converged: np.ndarray


def solve(levels, prm: OParams, f: np.ndarray, rtol: float = 1e-8, max_cycles: int = 10000,
          u0: np.ndarray | None = None, cycle=None) -> SolveResult:
    """u^m = LMG(A, f, u^{m-1}) per column until ||f - A u^m|| <= rtol ||f||.

    A column stops (is frozen) at the first iterate that meets the tolerance,
    so its result does not depend on the other columns.  `cycle` may replace
    the learnable cycle (e.g. the classical one) for comparison.
    """
    A = levels[0].A
    u = np.zeros_like(f) if u0 is None else u0.copy()
    fn = np.linalg.norm(f, axis=0)
    fn_safe = np.where(fn > 0, fn, 1.0)
    active = np.ones(f.shape[1], dtype=bool)
    iters = np.zeros(f.shape[1], dtype=np.int64)
    hist = []
    cyc = cycle or (lambda ff, uu: lmg(levels, prm, 0, ff, uu))
    for _ in range(max_cycles):
        rel = np.linalg.norm(f - A @ u, axis=0) / fn_safe
        hist.append(rel)
        active &= rel > rtol
        if not active.any():
            break
        idx = np.flatnonzero(active)
        u[:, idx] = cyc(f[:, idx], u[:, idx])
        iters[idx] += 1
    rel = np.linalg.norm(f - A @ u, axis=0) / fn_safe
    return SolveResult(u, iters, rel, hist, rel <= rtol)

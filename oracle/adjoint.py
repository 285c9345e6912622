"""Hand-written reverse-mode adjoint of the learnable V-cycle -- TEST INFRASTRUCTURE ONLY.

Training the cycle (paper Sec. 3.1, Alg. 3) back-propagates a residual loss
through LMG.  This module computes, for one cycle u_out = LMG(A, f, u_in) and a
cotangent g = dL/du_out, the vector-Jacobian products dL/df, dL/du_in and
dL/dTheta, by running the steps of Alg. 2 backwards.  Every step of Alg. 2 is
linear in the vectors, so each reverse rule is a transpose:

  smoothing  delta = theta D^{-1}(f - A u), u' = u + eta Phi(delta):
      Phi_bar = eta g,  d eta += <g, Phi(delta)>,  d c_k += <Phi_bar, M^k delta>,
      delta_bar = sum_k c_k (M^T)^k Phi_bar,  d theta += <delta_bar, D^{-1}(f - A u)>,
      s = theta D^{-1} delta_bar,  f_bar += s,  u_bar = g - A^T s
  restriction r_c = R Phi_R(f - A u):  y = R^T r_c_bar, r_bar = Phi_R^T(y), ...
  prolongation u += Phi_P(P e_c):  e_c_bar = P^T Phi_P^T(g)
  coarsest   u = A_J^{-1} f:  f_bar = A_J^{-T} g
with M^T = A_g^T D_g^{-1}.  Inner products sum over all right-hand-side
columns.  Plain NumPy, FP64; shares no code with the GPU path.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .lmg import OLevel, OParams, graph_conv, neighbour_mean, residual, smooth, lmg


def neighbour_mean_T(lv: OLevel, y: np.ndarray) -> np.ndarray:
    """M^T y = A_g^T (D_g^{-1} y) (the aggregation operator's transpose)."""
    if lv.Gw is not None:
        return lv.Gw.T @ y
    return lv.G.T @ (lv.inv_deg[:, None] * y)


def _cheb_terms(op, x, K):
    """[T_0(-op) x, ..., T_K(-op) x] by the three-term recurrence."""
    ts = [x]
    if K >= 1:
        ts.append(-op(x))
    for _ in range(1, K):
        ts.append(-2.0 * op(ts[-1]) - ts[-2])
    return ts


def graph_conv_vjp(c: np.ndarray, lv: OLevel, x: np.ndarray, ybar: np.ndarray, basis: str = "monomial"):
    """For y = sum_k c_k M^k x (or sum_k c_k T_k(-M) x): returns (x_bar, c_bar).
    The transpose of a polynomial in M is the same polynomial in M^T."""
    K = len(c) - 1
    if basis == "chebyshev":
        tx = _cheb_terms(lambda v: neighbour_mean(lv, v), x, K)
        cbar = np.array([np.sum(ybar * t) for t in tx])
        tg = _cheb_terms(lambda v: neighbour_mean_T(lv, v), ybar, K)
        xbar = sum(c[k] * tg[k] for k in range(K + 1))
        return xbar, cbar
    cbar = np.zeros(K + 1)
    w = x
    for k in range(K + 1):
        cbar[k] = np.sum(ybar * w)
        if k < K:
            w = neighbour_mean(lv, w)
    xbar = np.zeros_like(ybar)
    z = ybar
    for k in range(K + 1):
        xbar = xbar + c[k] * z
        if k < K:
            z = neighbour_mean_T(lv, z)
    return xbar, cbar


def zero_grads(prm: OParams) -> OParams:
    return OParams(np.zeros_like(prm.theta), np.zeros_like(prm.eta), np.zeros_like(prm.cB),
                   np.zeros_like(prm.cR), np.zeros_like(prm.cP), prm.nu_pre, prm.nu_post, prm.basis)


def _smooth_vjp(lv, l, prm, f, u, g, grads):
    rs = lv.Dinv[:, None] * residual(lv, f, u)         # D^{-1}(f - A u)
    delta = prm.theta[l] * rs
    phi = graph_conv(prm.cB[l], lv, delta, prm.basis)
    grads.eta[l] += np.sum(g * phi)
    phibar = prm.eta[l] * g
    dbar, cbar = graph_conv_vjp(prm.cB[l], lv, delta, phibar, prm.basis)
    grads.cB[l] += cbar
    grads.theta[l] += np.sum(dbar * rs)
    s = prm.theta[l] * (lv.Dinv[:, None] * dbar)
    return s, g - lv.A.T @ s                           # (f_bar contribution, u_bar)


def lmg_vjp(levels, prm: OParams, l: int, f, u, g, grads: OParams):
    """Reverse of u_out = LMG(A_l, f, u, l).  Returns (f_bar, u_bar); adds the
    parameter gradients into `grads`."""
    J = len(levels)
    lv = levels[l]
    if l == J - 1:
        fbar = sla.lu_solve(lv.lu, g, trans=1)
        return fbar, np.zeros_like(u)
    # forward recomputation, keeping the states the reverse sweep needs
    pre = []
    for _ in range(prm.nu_pre):
        pre.append(u)
        u = smooth(lv, l, prm, f, u)
    r = residual(lv, f, u)
    rc = lv.R @ graph_conv(prm.cR[l], lv, r, prm.basis)
    ec = lmg(levels, prm, l + 1, rc, np.zeros((levels[l + 1].A.shape[0], f.shape[1])))
    pe = lv.P @ ec
    u = u + graph_conv(prm.cP[l], lv, pe, prm.basis)
    post = []
    for _ in range(prm.nu_post):
        post.append(u)
        u = smooth(lv, l, prm, f, u)
    # reverse sweep
    fbar = np.zeros_like(f)
    for up in reversed(post):
        s, g = _smooth_vjp(lv, l, prm, f, up, g, grads)
        fbar += s
    xbar, cbar = graph_conv_vjp(prm.cP[l], lv, pe, g, prm.basis)
    grads.cP[l] += cbar
    ecbar = lv.P.T @ xbar
    rcbar, _ = lmg_vjp(levels, prm, l + 1, rc, np.zeros_like(ec), ecbar, grads)
    rbar, cbar = graph_conv_vjp(prm.cR[l], lv, r, lv.R.T @ rcbar, prm.basis)
    grads.cR[l] += cbar
    fbar += rbar
    g = g - lv.A.T @ rbar
    for up in reversed(pre):
        s, g = _smooth_vjp(lv, l, prm, f, up, g, grads)
        fbar += s
    return fbar, g


def cycle_vjp(levels, prm: OParams, f, u, g):
    """Finest-level VJP; returns (f_bar, u_bar, grads)."""
    grads = zero_grads(prm)
    fbar, ubar = lmg_vjp(levels, prm, 0, f, u, g, grads)
    return fbar, ubar, grads


def unrolled_loss(levels, prm: OParams, f, cycles: int = 10, u0=None):
    """Alg. 3 forward unrolled: u^0 = 0 (or a given start, e.g. the random
    initial guess of Sec. 4.1), u^m = LMG(A, f, u^{m-1});
    L = mean_b ||f_b - A u_b^{cycles}||^2 / ||f_b||^2."""
    u = np.zeros_like(f) if u0 is None else np.array(u0, dtype=np.float64)
    for _ in range(cycles):
        u = lmg(levels, prm, 0, f, u)
    r = residual(levels[0], f, u)
    fn2 = np.sum(f * f, axis=0)
    return float(np.mean(np.sum(r * r, axis=0) / fn2))


def unrolled_loss_and_grad(levels, prm: OParams, f, cycles: int = 10, u0=None):
    """Loss of `unrolled_loss` and its gradient w.r.t. the parameters."""
    us = [np.zeros_like(f) if u0 is None else np.array(u0, dtype=np.float64)]
    for _ in range(cycles):
        us.append(lmg(levels, prm, 0, f, us[-1]))
    A = levels[0].A
    r = residual(levels[0], f, us[-1])
    fn2 = np.sum(f * f, axis=0)
    B = f.shape[1]
    loss = float(np.mean(np.sum(r * r, axis=0) / fn2))
    g = -(2.0 / B) * (A.T @ (r / fn2[None, :]))      # dL/du^{cycles}
    grads = zero_grads(prm)
    for m in range(cycles, 0, -1):
        _, g = lmg_vjp(levels, prm, 0, f, us[m - 1], g, grads)
    return loss, grads


def residual_loss_grads(A, f, u, kind: str = "mean_rel_sq"):
    """Alg. 3's residual loss (Sec. 3.1) and its gradients with respect to u and
    f, written out by hand.  With r_b = f_b - A u_b per column:
      mean_rel_sq: L = (1/B) sum_b ||r_b||^2 / ||f_b||^2,
          dL/du_b = -(2/B) A^T r_b / ||f_b||^2,
          dL/df_b = (2/B) (r_b / ||f_b||^2 - ||r_b||^2 f_b / ||f_b||^4)
          (the second term from the f-dependence of the denominator);
          a column with f_b = 0 contributes 0 and has zero gradients;
      resid_norm: L = sum_b ||r_b||_2, dL/du_b = -A^T r_b / ||r_b||,
          dL/df_b = r_b / ||r_b|| (zero where r_b = 0).
    Returns (L, gu, gf)."""
    f = np.asarray(f, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    B = f.shape[1]
    r = f - A @ u
    rn2 = np.sum(r * r, axis=0)
    fn2 = np.sum(f * f, axis=0)
    gu = np.zeros_like(f)
    gf = np.zeros_like(f)
    if kind == "mean_rel_sq":
        L = 0.0
        for b in range(B):
            if fn2[b] == 0.0:
                continue
            L += rn2[b] / fn2[b]
            gu[:, b] = -(2.0 / B) * (A.T @ r[:, b]) / fn2[b]
            gf[:, b] = (2.0 / B) * (r[:, b] / fn2[b] - rn2[b] * f[:, b] / fn2[b] ** 2)
        return L / B, gu, gf
    if kind == "resid_norm":
        rn = np.sqrt(rn2)
        for b in range(B):
            if rn[b] == 0.0:
                continue
            gu[:, b] = -(A.T @ r[:, b]) / rn[b]
            gf[:, b] = r[:, b] / rn[b]
        return float(np.sum(rn)), gu, gf
    raise ValueError(f"unknown loss kind {kind}")

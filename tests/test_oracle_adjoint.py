"""Pins of the oracle's hand-written adjoint (training through the cycle, Sec. 3.1).

The reverse sweep is checked against (a) PyTorch CPU autograd of a separately
written dense forward of Alg. 2 (power sums instead of Horner, dense matrices,
torch.linalg.solve for the coarsest level) and (b) central finite differences
in FP64 with step 1e-6.  The cycle is affine in (f, u), so the vector
products w.r.t. f and u are also checked by exact difference quotients.
"""
import numpy as np
import pytest
import torch

from mginputs import configs as C, hierarchy as H
from oracle import adjoint as AD
from oracle import lmg as O


def _problem(side=17, B=2, K=2, seed=0, nlevels=None):
    h = H.square_hierarchy(side, H.block_field(C.rng(8, 1, seed), 4, -1.5, 1.5), nlevels=nlevels)
    J = h.nlevels
    flat = C.random_params(J, K, K, K, seed=seed + 11, spread=0.2)
    f = C.rng(8, 2, seed).standard_normal((h.sizes[0], B))
    return h, J, flat, f


def _torch_unrolled_loss(h, J, K, flat_t, f_np, cycles, nu):
    """Independent dense torch forward of Alg. 2, unrolled `cycles` times."""
    dt = torch.float64
    A = [torch.tensor(a.toarray(), dtype=dt) for a in h.A]
    P = [torch.tensor(p.toarray(), dtype=dt) for p in h.P]
    Mm = []
    for a in A:
        adj = ((a != 0) & ~torch.eye(a.shape[0], dtype=torch.bool)).to(dt)
        deg = adj.sum(1)
        Mm.append(torch.where(deg[:, None] > 0, adj / deg.clamp(min=1)[:, None], torch.zeros_like(adj)))
    per = 2 + 3 * (K + 1)

    def prm(l, what):
        base = l * per
        if what == "theta":
            return flat_t[base]
        if what == "eta":
            return flat_t[base + 1]
        off = {"B": 2, "R": 2 + K + 1, "P": 2 + 2 * (K + 1)}[what]
        return flat_t[base + off: base + off + K + 1]

    def conv(c, l, x):
        out = c[0] * x
        w = x
        for k in range(1, len(c)):
            w = Mm[l] @ w
            out = out + c[k] * w
        return out

    def cycle(l, f, u):
        if l == J - 1:
            return torch.linalg.solve(A[l], f)
        d = torch.diagonal(A[l])[:, None]
        for _ in range(nu):
            u = u + prm(l, "eta") * conv(prm(l, "B"), l, prm(l, "theta") * (f - A[l] @ u) / d)
        rc = P[l].T @ conv(prm(l, "R"), l, f - A[l] @ u)
        ec = cycle(l + 1, rc, torch.zeros_like(rc))
        u = u + conv(prm(l, "P"), l, P[l] @ ec)
        for _ in range(nu):
            u = u + prm(l, "eta") * conv(prm(l, "B"), l, prm(l, "theta") * (f - A[l] @ u) / d)
        return u

    f = torch.tensor(f_np, dtype=dt)
    u = torch.zeros_like(f)
    for _ in range(cycles):
        u = cycle(0, f, u)
    r = f - A[0] @ u
    return torch.mean((r * r).sum(0) / (f * f).sum(0))


@pytest.mark.parametrize("K", [0, 1, 3])
def test_adjoint_matches_torch_autograd(K):
    h, J, flat, f = _problem(K=K, seed=K)
    lv = O.make_levels(h.A, h.P, h.R)
    prm = O.unpack(flat, J, K, K, K)
    loss, grads = AD.unrolled_loss_and_grad(lv, prm, f, cycles=3)
    flat_t = torch.tensor(flat, dtype=torch.float64, requires_grad=True)
    tl = _torch_unrolled_loss(h, J, K, flat_t, f, 3, 2)
    tl.backward()
    assert abs(loss - tl.item()) <= 1e-12 * abs(loss)
    g = O.pack(grads)
    gt = flat_t.grad.numpy()
    assert np.linalg.norm(g - gt) <= 1e-11 * np.linalg.norm(gt)


def test_adjoint_matches_central_fd():
    K = 2
    h, J, flat, f = _problem(K=K, seed=4)
    lv = O.make_levels(h.A, h.P, h.R)
    prm = O.unpack(flat, J, K, K, K)
    _, grads = AD.unrolled_loss_and_grad(lv, prm, f, cycles=3)
    g = O.pack(grads)
    step = 1e-6
    for i in range(len(flat)):
        fp, fm = flat.copy(), flat.copy()
        fp[i] += step
        fm[i] -= step
        Lp = AD.unrolled_loss(lv, O.unpack(fp, J, K, K, K), f, 3)
        Lm = AD.unrolled_loss(lv, O.unpack(fm, J, K, K, K), f, 3)
        fd = (Lp - Lm) / (2 * step)
        assert abs(fd - g[i]) <= 1e-5 * np.abs(g).max() + 1e-7 * abs(g[i]), (i, fd, g[i])


def test_vector_vjp_exact_difference_quotient():
    """LMG is affine in (f, u): <g, LMG(f + df, u + du) - LMG(f, u)> = <f_bar, df> + <u_bar, du>."""
    h, J, flat, f = _problem(side=33, K=3, seed=5, B=3)
    lv = O.make_levels(h.A, h.P, h.R)
    prm = O.unpack(flat, J, 3, 3, 3)
    gen = C.rng(8, 3, 0)
    u = gen.standard_normal(f.shape)
    g = gen.standard_normal(f.shape)
    df = gen.standard_normal(f.shape)
    du = gen.standard_normal(f.shape)
    fbar, ubar, _ = AD.cycle_vjp(lv, prm, f, u, g)
    lhs = np.sum(g * (O.lmg(lv, prm, 0, f + df, u + du) - O.lmg(lv, prm, 0, f, u)))
    rhs = np.sum(fbar * df) + np.sum(ubar * du)
    assert abs(lhs - rhs) <= 1e-11 * (abs(rhs) + np.linalg.norm(g) * np.linalg.norm(df))


@pytest.mark.parametrize("kind", ["mean_rel_sq", "resid_norm"])
def test_residual_loss_values_closed_form(kind):
    """The loss at iterates whose residual is known exactly: u = 0 gives r = f
    (L = 1 for the mean relative square, sum_b ||f_b|| for the norm), u = A^{-1} f
    gives r = 0 (L = 0, zero gradients), u = A^{-1} (f / 2) gives r = f / 2."""
    h = H.square_hierarchy(9)
    A = h.A[0].toarray()
    f = C.rng(6, 90, 0).standard_normal((A.shape[0], 3))
    fn = np.linalg.norm(f, axis=0)
    L0, _, gf0 = AD.residual_loss_grads(A, f, np.zeros_like(f), kind)
    want0 = 1.0 if kind == "mean_rel_sq" else fn.sum()
    assert abs(L0 - want0) <= 1e-14 * want0
    ustar = np.linalg.solve(A, f)
    L1, gu1, gf1 = AD.residual_loss_grads(A, f, ustar, kind)
    assert L1 <= 1e-24 if kind == "mean_rel_sq" else L1 <= 1e-12
    Lh, _, _ = AD.residual_loss_grads(A, f, np.linalg.solve(A, f / 2), kind)
    wanth = 0.25 if kind == "mean_rel_sq" else fn.sum() / 2
    assert abs(Lh - wanth) <= 1e-13 * wanth
    if kind == "mean_rel_sq":
        # at u = 0 the loss is 1 for every f, so dL/df vanishes (the two terms cancel)
        assert np.abs(gf0).max() <= 1e-15 * np.abs(f).max()
        assert np.abs(gu1).max() <= 1e-12


@pytest.mark.parametrize("kind", ["mean_rel_sq", "resid_norm"])
def test_residual_loss_gradients_match_torch_autograd_and_fd(kind):
    """Hand gradients against torch CPU autograd of the loss definition and
    against central differences; a zero right-hand side (mean_rel_sq) and a
    zero residual (resid_norm) take no part."""
    h = H.square_hierarchy(17, H.block_field(C.rng(6, 91, 1), 4, -1, 1))
    A = h.A[0].toarray()
    g = C.rng(6, 91, 0)
    f = g.standard_normal((A.shape[0], 3))
    u = g.standard_normal((A.shape[0], 3))
    if kind == "mean_rel_sq":
        f[:, 2] = 0.0
    else:
        f[:, 2] = 0.0
        u[:, 2] = 0.0          # r = 0 exactly
    L, gu, gf = AD.residual_loss_grads(A, f, u, kind)
    At = torch.tensor(A)
    ft = torch.tensor(f[:, :2], requires_grad=True)
    ut = torch.tensor(u[:, :2], requires_grad=True)
    r = ft - At @ ut
    if kind == "mean_rel_sq":
        Lt = ((r * r).sum(0) / (ft * ft).sum(0)).sum() / 3
    else:
        Lt = torch.sqrt((r * r).sum(0)).sum()
    Lt.backward()
    assert abs(L - Lt.item()) <= 1e-13 * abs(L)
    assert np.abs(gu[:, :2] - ut.grad.numpy()).max() <= 1e-12 * np.abs(gu).max()
    assert np.abs(gf[:, :2] - ft.grad.numpy()).max() <= 1e-12 * np.abs(gf).max()
    assert np.abs(gu[:, 2]).max() == 0.0 and np.abs(gf[:, 2]).max() == 0.0
    d = g.standard_normal(f.shape)
    d[:, 2] = 0.0
    eps = 1e-6
    for which, grad in (("u", gu), ("f", gf)):
        def Lat(s):
            ff, uu = (f, u + s * d) if which == "u" else (f + s * d, u)
            return AD.residual_loss_grads(A, ff, uu, kind)[0]
        fd = (Lat(eps) - Lat(-eps)) / (2 * eps)
        assert abs(fd - np.sum(grad * d)) <= 1e-6 * abs(fd)


def test_residual_loss_planted_mistake_fails_fd():
    """Dropping the denominator term of dL/df (a plausible slip) fails the
    central-difference check."""
    h = H.square_hierarchy(9)
    A = h.A[0].toarray()
    g = C.rng(6, 92, 0)
    f = g.standard_normal((A.shape[0], 2))
    u = g.standard_normal((A.shape[0], 2))
    L, gu, gf = AD.residual_loss_grads(A, f, u)
    r = f - A @ u
    wrong = (2.0 / 2) * r / np.sum(f * f, axis=0)
    d = g.standard_normal(f.shape)
    fd = (AD.residual_loss_grads(A, f + 1e-6 * d, u)[0] - AD.residual_loss_grads(A, f - 1e-6 * d, u)[0]) / 2e-6
    assert abs(fd - np.sum(gf * d)) <= 1e-6 * abs(fd)
    assert abs(fd - np.sum(wrong * d)) > 1e-3 * abs(fd)

"""Pins of the oracle's FGMRES and full multigrid (Sec. 4.2 usage as a
preconditioner): library GMRES, exact preconditioning, the Arnoldi
relation behind the residual estimate, and FMG's textbook accuracy."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from mginputs import configs as C, hierarchy as H
from oracle import krylov as KR
from oracle import lmg as O


def _levels(side=33, lo=-1.0, hi=1.0, seed=0):
    h = H.square_hierarchy(side, H.block_field(C.rng(7, 1, seed), 4, lo, hi))
    return h, O.make_levels(h.A, h.P, h.R)


def test_unpreconditioned_fgmres_matches_library_gmres():
    h, lv = _levels(17)
    J = h.nlevels
    prm = O.unpack(C.identity_params(J, 1, 1, 1), J, 1, 1, 1)
    f = C.rng(7, 2, 0).standard_normal((h.sizes[0], 1))
    n = h.sizes[0]
    u, it, rr, _ = KR.fgmres(lv, prm, f, restart=n, rtol=1e-10, max_iter=n, precond="none")
    x, info = spla.gmres(h.A[0], f[:, 0], rtol=1e-10, restart=n, maxiter=1, atol=0.0)
    assert info == 0
    assert rr[0] <= 1e-10
    assert np.linalg.norm(u[:, 0] - x) <= 1e-7 * np.linalg.norm(x)


def test_exact_preconditioner_converges_in_one_iteration():
    h, lv = _levels(17)
    J = h.nlevels
    prm = O.unpack(C.identity_params(J, 1, 1, 1), J, 1, 1, 1)
    f = C.rng(7, 2, 1).standard_normal((h.sizes[0], 2))
    u, it, rr, _ = KR.fgmres(lv, prm, f, restart=10, rtol=1e-12, precond="exact")
    assert np.all(it == 1) and np.all(rr <= 1e-12)


def test_residual_estimate_is_true_residual_and_learnable_preconditioner_helps():
    h, lv = _levels(33, -2, 2, seed=1)
    J = h.nlevels
    prm = O.unpack(C.random_params(J, 2, 2, 2, seed=5, spread=0.1), J, 2, 2, 2)
    f = C.rng(7, 2, 2).standard_normal((h.sizes[0], 1))
    u, it, rr, hist = KR.fgmres(lv, prm, f, restart=50, rtol=1e-10, precond="vcycle")
    assert rr[0] <= 1e-10 * 1.01
    assert abs(hist[-1] - rr[0]) <= 1e-3 * rr[0] + 1e-13
    stat = O.solve(lv, prm, f, rtol=1e-10)
    assert it[0] < stat.iters[0]


def test_fmg_with_classical_parameters_is_nested_iteration_of_alg1():
    """Identity parameters: FMG is nested iteration (exact coarsest solve,
    interpolation by P, one classical V-cycle of Alg. 1 per level)."""
    h, lv = _levels(33, -1, 1, seed=3)
    J = h.nlevels
    prm = O.unpack(C.identity_params(J, 2, 2, 2), J, 2, 2, 2)
    f = C.rng(7, 2, 4).standard_normal((h.sizes[0], 2))
    fs = [f]
    for l in range(J - 1):
        fs.append(h.R[l] @ fs[-1])
    u = np.linalg.solve(h.A[J - 1].toarray(), fs[J - 1])
    for l in range(J - 2, -1, -1):
        u = O.classical_mg(lv, 2.0 / 3.0, 2, l, fs[l], h.P[l] @ u)
    got = KR.fmg(lv, prm, f)
    assert np.abs(got - u).max() <= 1e-12 * np.abs(u).max()


def test_fmg_two_levels_starts_from_the_cycles_coarse_correction():
    """J = 2, random parameters: the FMG initial guess Phi_P P A_1^{-1} R Phi_R f
    is what one cycle without smoothing returns from u = 0, so FMG equals a
    V(2,2) cycle started there."""
    side = 9
    h = H.square_hierarchy(side, H.block_field(C.rng(7, 1, 9), 4, -1, 1), nlevels=2)
    lv = O.make_levels(h.A, h.P, h.R)
    flat = C.random_params(2, 3, 3, 3, seed=11, spread=0.3)
    prm = O.unpack(flat, 2, 3, 3, 3)
    prm0 = O.unpack(flat, 2, 3, 3, 3, nu_pre=0, nu_post=0)
    f = C.rng(7, 2, 5).standard_normal((h.sizes[0], 3))
    u0 = O.lmg(lv, prm0, 0, f, np.zeros_like(f))
    want = O.lmg(lv, prm, 0, f, u0)
    assert np.abs(KR.fmg(lv, prm, f) - want).max() <= 1e-13 * np.abs(want).max()


def test_fmg_error_shrinks_with_the_mesh():
    """Manufactured solution sin(pi x) sin(pi y), a = 1: one FMG pass with the
    classical cycle has a total error that falls by close to h^2 under
    refinement and stays within a small multiple of the discretisation error."""
    errs = []
    for side in (33, 65, 129):
        h = H.square_hierarchy(side)
        lv = O.make_levels(h.A, h.P, h.R)
        J = h.nlevels
        prm = O.unpack(C.identity_params(J, 1, 1, 1), J, 1, 1, 1)
        hh = 1.0 / (side - 1)
        xs = np.arange(1, side - 1) * hh
        X, Y = np.meshgrid(xs, xs, indexing="xy")
        uex = (np.sin(np.pi * X) * np.sin(np.pi * Y)).ravel()[:, None]
        f = hh * hh * 2 * np.pi ** 2 * uex
        udisc = spla.spsolve(h.A[0].tocsc(), f[:, 0])[:, None]
        u = KR.fmg(lv, prm, f)
        errs.append(np.abs(u - uex).max())
        assert np.abs(u - udisc).max() <= 12 * np.abs(udisc - uex).max()
    assert errs[0] / errs[1] >= 2.5 and errs[1] / errs[2] >= 2.8


def test_fmg_preconditioner_converges():
    h, lv = _levels(33, -2, 2, seed=2)
    J = h.nlevels
    prm = O.unpack(C.identity_params(J, 2, 2, 2), J, 2, 2, 2)
    f = C.rng(7, 2, 3).standard_normal((h.sizes[0], 1))
    u, it, rr, _ = KR.fgmres(lv, prm, f, restart=30, rtol=1e-8, precond="fmg")
    _, it_v, _, _ = KR.fgmres(lv, prm, f, restart=30, rtol=1e-8, precond="vcycle")
    assert rr[0] <= 1e-8 and it[0] <= it_v[0]

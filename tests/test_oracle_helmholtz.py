"""Pins of the Helmholtz (two-feature) oracle against facts fixed by the paper
and by the mathematics, not by the oracle's own formulas."""
import numpy as np
import pytest
import scipy.sparse as sp

from mginputs import configs as C
from mginputs import helmholtz as HZ
from oracle import helmholtz as OH


def small(side=17, k=6.0, J=3, B=3, seed=0):
    h = HZ.hierarchy(side, k, J)
    plan = HZ.smoother_plan(h)
    f = HZ.load_vectors(side, HZ.source_centres(B, C.rng(10, 2, seed)))
    return h, plan, f


def test_discretisation_is_complex_symmetric_and_consistent():
    """A = K - k^2 M - i k M_b: complex symmetric (not Hermitian); K has zero
    row sums; M integrates 1 to the area 1; M_b to the perimeter 4; on nested
    P1 meshes the Galerkin product P^T A_h P equals A_2h."""
    side, k = 17, 7.0
    K, M, Mb = HZ.matrices(side)
    one = np.ones(side * side)
    assert np.abs(K @ one).max() < 1e-12
    assert abs(one @ (M @ one) - 1.0) < 1e-13
    assert abs(one @ (Mb @ one) - 4.0) < 1e-13
    A = HZ.helmholtz_matrix(side, k)
    assert abs(A - A.T).max() == 0.0
    assert abs(A - A.conj().T).max() > 0.0
    P = HZ.prolongation(side)
    Ac = HZ.helmholtz_matrix((side + 1) // 2, k)
    assert abs(sp.csr_matrix(P.T @ A @ P) - Ac).max() < 1e-12
    # interpolation reproduces linear functions exactly
    pf, _ = HZ.mesh(side)
    pc, _ = HZ.mesh((side + 1) // 2)
    lin = lambda p: 0.3 + 2.0 * p[:, 0] - 1.5 * p[:, 1]
    assert np.abs(P @ lin(pc) - lin(pf)).max() < 1e-14


def test_smoother_plan_follows_kh():
    h = HZ.hierarchy(257, 16 * np.pi, 5)
    assert [round(h.kh(l), 3) for l in range(5)] == [0.196, 0.393, 0.785, 1.571, 3.142]
    assert [p[0] for p in HZ.smoother_plan(h)] == ["jacobi", "jacobi", "gmres", "gmres"]


def test_feature_mixing_with_complex_structured_weights_is_complex_multiplication():
    """With W_k = [[a_k, -b_k], [b_k, a_k]] the two-feature convolution is the
    complex polynomial sum_k (a_k + i b_k) M^k x (powers formed explicitly)."""
    h, _, _ = small()
    lev = OH.make_levels(h.A, h.P, h.R)[0]
    g = np.random.default_rng(3)
    x = g.standard_normal((lev.A.shape[0], 2)) + 1j * g.standard_normal((lev.A.shape[0], 2))
    K = 3
    a, b = g.standard_normal(K + 1), g.standard_normal(K + 1)
    W = np.stack([np.array([[a[k], -b[k]], [b[k], a[k]]]) for k in range(K + 1)])
    Md = lev.M.toarray()
    want = sum((a[k] + 1j * b[k]) * (np.linalg.matrix_power(Md, k) @ x) for k in range(K + 1))
    assert np.abs(OH.conv(W, lev, x) - want).max() < 1e-12


def test_feature_mixing_general_weights_as_real_feature_layers():
    """General weights: node features X = [Re x, Im x] (n x 2); the layer is
    sum_k (M^k X) W_k^T (a linear layer on the features of every node after
    k aggregations); feature 0 is the real part."""
    h, _, _ = small()
    lev = OH.make_levels(h.A, h.P, h.R)[0]
    g = np.random.default_rng(4)
    n = lev.A.shape[0]
    x = g.standard_normal(n) + 1j * g.standard_normal(n)
    W = g.standard_normal((3, 2, 2))
    X = np.stack([x.real, x.imag], axis=1)
    Md = lev.M.toarray()
    Y = sum(np.linalg.matrix_power(Md, k) @ X @ W[k].T for k in range(3))
    got = OH.conv(W, lev, x[:, None])[:, 0]
    assert np.abs(got.real - Y[:, 0]).max() < 1e-12 and np.abs(got.imag - Y[:, 1]).max() < 1e-12
    # W = [[0, 0], [1, 0]] copies the real part into the imaginary part
    cp = OH.conv(np.array([[[0.0, 0.0], [1.0, 0.0]]]), lev, x[:, None])[:, 0]
    assert np.array_equal(cp, 1j * x.real)


def test_gmres_steps_minimise_over_the_affine_krylov_space():
    """GMRES(A, r, x0, v) = argmin ||r - A x|| over x0 + span{r0, A r0, ...,
    A^{v-1} r0}, r0 = r - A x0 (brute force with the monomial basis)."""
    h, _, _ = small(side=9, k=9.0, J=2)
    A = h.A[0]
    Ad = A.toarray()
    n = Ad.shape[0]
    g = np.random.default_rng(5)
    r = g.standard_normal((n, 2)) + 1j * g.standard_normal((n, 2))
    x0 = 0.1 * (g.standard_normal((n, 2)) + 1j * g.standard_normal((n, 2)))
    for v in (1, 2, 4):
        got = OH.gmres_steps(A, r, x0, v)
        for b in range(2):
            r0 = r[:, b] - Ad @ x0[:, b]
            Kb = np.stack([np.linalg.matrix_power(Ad, j) @ r0 for j in range(v)], axis=1)
            y = np.linalg.lstsq(Ad @ Kb, r0, rcond=None)[0]
            want = x0[:, b] + Kb @ y
            assert np.linalg.norm(got[:, b] - want) <= 1e-9 * np.linalg.norm(want)
    # v = n: exact solve; r = A x0: x0 returned; A = I: exact after one step
    ex = OH.gmres_steps(A, r[:, :1], np.zeros((n, 1), complex), n)
    assert np.linalg.norm(Ad @ ex[:, 0] - r[:, 0]) <= 1e-8 * np.linalg.norm(r[:, 0])
    assert np.array_equal(OH.gmres_steps(A, A @ x0, x0, 3), x0)
    I = sp.identity(n, dtype=complex, format="csr")
    assert np.allclose(OH.gmres_steps(I, r, x0, 4), r, rtol=0, atol=1e-13)


def test_two_grid_jacobi_cycle_equals_its_error_propagation_matrix():
    """J = 2, Jacobi smoothing, identity convolutions: the cycle is
    u_out = E u + N f with E = S^post (I - P A_c^{-1} R A) S^pre and
    S = I - omega D^{-1} A (the classical two-grid operator, Sec. 2.2-2.3)."""
    h = HZ.hierarchy(17, 5.0, 2)
    plan = [("jacobi", 2, 1)]
    om = 0.6
    prm = OH.unpack(C.hz_identity_params(2, 1, 1, 1, plan, omega=om), 2, 1, 1, 1, plan)
    lev = OH.make_levels(h.A, h.P, h.R)
    A = h.A[0].toarray()
    n = A.shape[0]
    S = np.eye(n) - om * np.diag(1.0 / np.diag(A)) @ A
    P, R, Ac = h.P[0].toarray(), h.R[0].toarray(), h.A[1].toarray()
    CG = np.eye(n) - P @ np.linalg.solve(Ac, R @ A)
    E = S @ CG @ S @ S
    g = np.random.default_rng(6)
    u = g.standard_normal((n, 2)) + 1j * g.standard_normal((n, 2))
    x = g.standard_normal((n, 2)) + 1j * g.standard_normal((n, 2))
    f = A @ x
    got = OH.lmg(lev, prm, 0, f, u)
    # the cycle is consistent (x is a fixed point), so u_out - x = E (u - x)
    assert np.linalg.norm((got - x) - E @ (u - x)) <= 1e-10 * np.linalg.norm(u - x)


def test_gmres_level_with_zero_theta_is_the_classical_gmres_smoother():
    """Identity parameters on a GMRES level: each smoothing step is v GMRES
    steps from zero on the current residual equation (brute force)."""
    h = HZ.hierarchy(17, 20.0, 2)
    plan = [("gmres", 1, 0)]
    prm = OH.unpack(C.hz_identity_params(2, 1, 1, 1, plan), 2, 1, 1, 1, plan)
    prm.v = 3
    lev = OH.make_levels(h.A, h.P, h.R)
    A = h.A[0].toarray()
    n = A.shape[0]
    g = np.random.default_rng(7)
    f = g.standard_normal((n, 1)) + 1j * g.standard_normal((n, 1))
    u0 = np.zeros((n, 1), complex)
    got = OH.smooth(lev[0], prm, 0, f, u0)
    Kb = np.stack([np.linalg.matrix_power(A, j) @ f[:, 0] for j in range(3)], axis=1)
    want = Kb @ np.linalg.lstsq(A @ Kb, f[:, 0], rcond=None)[0]
    assert np.linalg.norm(got[:, 0] - want) <= 1e-9 * np.linalg.norm(want)


def test_fgmres_exact_and_unpreconditioned_limits():
    """The exact inverse as preconditioner converges in one iteration; without
    a preconditioner and with restart >= n, FGMRES is GMRES and reaches the
    solution of the system within n iterations."""
    h, plan, f = small(side=9, k=8.0, J=2, B=2)
    lev = OH.make_levels(h.A, h.P, h.R)
    prm = OH.unpack(C.hz_identity_params(2, 1, 1, 1, plan), 2, 1, 1, 1, plan)
    u, it, rr, _ = OH.fgmres(lev, prm, f, restart=5, precond="exact", rtol=1e-10)
    assert list(it) == [1, 1] and rr.max() < 1e-10
    n = h.sizes[0]
    u, it, rr, hist = OH.fgmres(lev, prm, f, restart=n, precond="none", rtol=1e-10, max_iter=n)
    assert it.max() <= n and rr.max() < 1e-9
    x = np.linalg.solve(h.A[0].toarray(), f)
    assert np.linalg.norm(u - x) <= 1e-8 * np.linalg.norm(x)
    assert all(a >= b - 1e-15 for a, b in zip(hist, hist[1:]))       # GMRES residuals never grow


def test_fgmres_estimate_matches_true_residual():
    """The Givens estimate |g_{j+1}| / ||f|| equals the true relative residual
    of the iterate built from the first j + 1 directions (no restart)."""
    h, plan, f = small(side=17, k=6.0, J=3, B=1)
    lev = OH.make_levels(h.A, h.P, h.R)
    prm = OH.unpack(C.hz_random_params(3, 1, 1, 1, plan, seed=2), 3, 1, 1, 1, plan)
    for mi in (3, 6):
        u, it, rr, hist = OH.fgmres(lev, prm, f, restart=40, precond="vcycle", max_iter=mi, rtol=1e-14)
        assert it[0] == mi
        assert abs(hist[-1] - rr[0]) <= 1e-8 * rr[0]


def test_learnable_cycle_solves_small_helmholtz_as_preconditioner():
    """V-cycle and FMG preconditioners with random near-identity weights
    (GMRES levels included) drive FGMRES to 1e-8 on every column, FMG in no
    more iterations than the V-cycle on the test and training sources."""
    w = C.helmholtz(33, 12.0, 4, B=2)
    lev = OH.make_levels(w.hier.A, w.hier.P, w.hier.R)
    assert [p[0] for p in w.plan] == ["jacobi", "gmres", "gmres"]
    prm = OH.unpack(w.params, 4, 1, 1, 1, w.plan)
    _, itv, rrv, _ = OH.fgmres(lev, prm, w.f, restart=30, precond="vcycle", max_iter=60)
    _, itf, rrf, _ = OH.fgmres(lev, prm, w.f, restart=30, precond="fmg", max_iter=60)
    assert rrv.max() <= 1e-8 and rrf.max() <= 1e-8
    assert (itf <= itv).all()
    prm2 = OH.unpack(C.hz_random_params(4, 1, 1, 1, w.plan, seed=3, spread=0.05), 4, 1, 1, 1, w.plan)
    _, it2, rr2, _ = OH.fgmres(lev, prm2, w.f, restart=30, precond="vcycle", max_iter=80)
    assert rr2.max() <= 1e-8


@pytest.mark.parametrize("mutation", ["transpose_mix", "no_conj", "drop_eta", "swap_R_P_conv"])
def test_planted_mistakes_are_caught(monkeypatch, mutation):
    """A plausible slip in the oracle fails at least one pin above."""
    import tests.test_oracle_helmholtz as T
    if mutation == "transpose_mix":
        orig = OH.mix
        monkeypatch.setattr(OH, "mix", lambda W, x: orig(W.T, x))
        checks = [T.test_feature_mixing_general_weights_as_real_feature_layers]
    elif mutation == "no_conj":
        monkeypatch.setattr(OH.np, "vdot", lambda a, b: np.sum(a * b))
        checks = [T.test_gmres_steps_minimise_over_the_affine_krylov_space]
    elif mutation == "drop_eta":
        orig_s = OH.smooth

        def bad(lev, prm, l, f, u):
            prm2 = OH.HParams(prm.theta, np.ones_like(prm.eta), prm.WB, prm.WR, prm.WP, prm.plan, prm.v)
            return orig_s(lev, prm2, l, f, u)
        monkeypatch.setattr(OH, "smooth", bad)
        checks = [_eta_pin]
    else:
        orig_l = OH.lmg

        def bad(levels, prm, l, f, u):
            prm2 = OH.HParams(prm.theta, prm.eta, prm.WB, prm.WP, prm.WR, prm.plan, prm.v)
            return orig_l(levels, prm2, l, f, u)
        monkeypatch.setattr(OH, "lmg", bad)
        checks = [_transfer_pin]
    failed = 0
    for c in checks:
        try:
            c()
        except AssertionError:
            failed += 1
    assert failed == len(checks)


def _eta_pin():
    """eta scales the whole smoothing correction: one Jacobi pre-smoothing
    step with eta = 1/2 moves u half as far as with eta = 1."""
    h = HZ.hierarchy(9, 3.0, 2)
    plan = [("jacobi", 1, 0)]
    lev = OH.make_levels(h.A, h.P, h.R)
    n = h.sizes[0]
    g = np.random.default_rng(8)
    f = g.standard_normal((n, 1)) + 0j
    u = np.zeros((n, 1), complex)
    p1 = OH.unpack(C.hz_identity_params(2, 1, 1, 1, plan), 2, 1, 1, 1, plan)
    p2 = OH.unpack(C.hz_identity_params(2, 1, 1, 1, plan), 2, 1, 1, 1, plan)
    p2.eta[:] = 0.5
    d1 = OH.smooth(lev[0], p1, 0, f, u)
    d2 = OH.smooth(lev[0], p2, 0, f, u)
    assert np.abs(d2 - 0.5 * d1).max() < 1e-15


def _transfer_pin():
    """Restriction applies Phi_R before R, prolongation applies Phi_P after P:
    a J = 2 cycle without smoothing is u + Phi_P(P A_c^{-1} R Phi_R(f - A u))
    (dense matrices, weight matrices applied to [Re, Im])."""
    h = HZ.hierarchy(9, 3.0, 2)
    plan = [("jacobi", 0, 0)]
    lev = OH.make_levels(h.A, h.P, h.R)
    g = np.random.default_rng(9)
    WR = np.array([[[1.0, 0.3], [-0.2, 0.9]]])
    WP = np.array([[[0.7, -0.4], [0.5, 1.1]]])
    prm = OH.HParams(np.zeros(1), np.ones(1), [np.eye(2)[None]], WR, WP, plan, 4)
    n = h.sizes[0]
    f = g.standard_normal((n, 1)) + 1j * g.standard_normal((n, 1))
    u = np.zeros((n, 1), complex)

    def lay(W, x):
        X = np.stack([x.real, x.imag], -1) @ W.T
        return X[..., 0] + 1j * X[..., 1]
    want = lay(WP[0], h.P[0] @ np.linalg.solve(h.A[1].toarray(), h.R[0] @ lay(WR[0], f)))
    got = OH.lmg(lev, prm, 0, f, u)
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()


def test_eta_and_transfer_pins():
    _eta_pin()
    _transfer_pin()


def test_fmg_two_level_closed_form():
    """Two-level FMG with no smoothing: the coarse solution
    u_1 = A_c^{-1} R Phi_R(f) is interpolated to u_0 = Phi_P(P u_1), and one
    cycle from u_0 adds Phi_P(P A_c^{-1} R Phi_R(f - A u_0)); dense matrices,
    the two-feature weights applied to [Re, Im]."""
    h = HZ.hierarchy(9, 3.0, 2)
    plan = [("jacobi", 0, 0)]
    lev = OH.make_levels(h.A, h.P, h.R)
    WR = np.array([[[1.1, 0.2], [-0.3, 0.8]]])
    WP = np.array([[[0.9, -0.1], [0.4, 1.2]]])
    prm = OH.HParams(np.zeros(1), np.ones(1), [np.eye(2)[None]], WR, WP, plan, 4)
    g = np.random.default_rng(11)
    n = h.sizes[0]
    f = g.standard_normal((n, 2)) + 1j * g.standard_normal((n, 2))

    def lay(W, x):
        X = np.stack([x.real, x.imag], -1) @ W.T
        return X[..., 0] + 1j * X[..., 1]
    A, P, R, Ac = h.A[0].toarray(), h.P[0].toarray(), h.R[0].toarray(), h.A[1].toarray()
    u1 = np.linalg.solve(Ac, R @ lay(WR[0], f))
    u0 = lay(WP[0], P @ u1)
    # the cycle from u0 adds Phi_P(P A_c^{-1} R Phi_R(f - A u0))
    want = u0 + lay(WP[0], P @ np.linalg.solve(Ac, R @ lay(WR[0], f - A @ u0)))
    got = OH.fmg(lev, prm, f)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()

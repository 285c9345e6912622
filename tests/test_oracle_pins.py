"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test pins a part of the oracle to something other than the oracle itself:
closed forms (eigenvalues of the learnable smoother, Sec. 3.3), textbook
properties (Galerkin orthogonality of the coarse-grid correction, O(h^2)
nodal error of P1 on a uniform mesh, symmetry of the V-cycle with a symmetric
smoother), exact rational brute force on a tiny grid, the classical V-cycle
(Alg. 1) that identity initialisation must recover (Sec. 3.4 and the recovery
remark of Sec. 3.3), and dense linear algebra on tiny grids.
"""
from fractions import Fraction
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

from mginputs import configs as C, hierarchy as H
from oracle import lmg as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def levels_of(h, **kw):
    return O.make_levels(h.A, h.P, h.R, **kw)


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


# ----------------------------------------------------------------------------- paper constants
def test_identity_initialisation_matches_paper_constants():
    """Identity initialisation W1 = I, W2 = 0, theta = omega, eta = 1 and the
    experiments' omega = 2/3 (Sec. 3.4, Sec. 4.1) as stored in the golden file."""
    with open(os.path.join(GOLDEN, "paper_constants.json")) as fh:
        g = json.load(fh)
    omega = g["omega_darcy"]["value"]
    p = O.unpack(C.identity_params(4, 2, 2, 2, omega), 4, 2, 2, 2)
    assert np.all(p.theta == omega) and np.all(p.eta == g["eta_init"]["value"])
    for c in (p.cB, p.cR, p.cP):
        assert np.all(c[:, 0] == g["w1_init"]["value"]) and np.all(c[:, 1:] == g["w2_init"]["value"])


# ----------------------------------------------------------------------------- P1 classical recovery
@pytest.mark.parametrize("problem", ["poisson", "blocks"])
def test_identity_params_recover_classical_vcycle(problem):
    """w1 = 1, w2 = 0, theta = omega, eta = 1 gives damped Jacobi, and identity
    transfer convolutions give plain R and P: LMG must equal Alg. 1."""
    if problem == "poisson":
        h = H.square_hierarchy(33)
    else:
        h = H.square_hierarchy(33, H.block_field(C.rng(9, 1, 0), 4, -2, 2))
    lv = levels_of(h)
    J = h.nlevels
    f = C.rng(9, 2, 0).standard_normal((h.sizes[0], 3))
    u = C.rng(9, 2, 1).standard_normal((h.sizes[0], 3))
    for K in (0, 1, 2, 3):
        prm = O.unpack(C.identity_params(J, K, K, K, 2 / 3), J, K, K, K)
        a = O.lmg(lv, prm, 0, f, u)
        b = O.classical_mg(lv, 2 / 3, 2, 0, f, u)
        assert rel(a, b) < 1e-14


def test_classical_poisson_33_converges_like_multigrid():
    """Config of the unit-square Poisson problem, 961 unknowns, 4 levels:
    classical V(2,2) reaches 1e-8 within 10-20 cycles (h-independent rate)."""
    w = C.poisson_unit()
    lv = levels_of(w.hier)
    prm = O.unpack(w.params, w.hier.nlevels, w.KB, w.KR, w.KP)
    res = O.solve(lv, prm, w.f, rtol=1e-8)
    assert res.converged.all() and 8 <= res.iters[0] <= 20
    hist = np.array(res.history)[:, 0]
    rates = hist[1:] / hist[:-1]
    assert rates[2:].max() < 0.35


# ----------------------------------------------------------------------------- P2 manufactured solution
def test_manufactured_solution_second_order():
    """-Lap u = 2 pi^2 sin(pi x) sin(pi y), P1 with lumped load: nodal max error O(h^2)."""
    errs, hs = [], []
    for side in (17, 33, 65, 129):
        h = H.square_hierarchy(side)
        hh = 1.0 / (side - 1)
        xs = np.arange(1, side - 1) * hh
        X, Y = np.meshgrid(xs, xs, indexing="xy")
        uex = (np.sin(np.pi * X) * np.sin(np.pi * Y)).ravel()[:, None]
        f = hh * hh * 2 * np.pi ** 2 * uex
        lv = levels_of(h)
        J = h.nlevels
        prm = O.unpack(C.identity_params(J, 1, 1, 1), J, 1, 1, 1)
        res = O.solve(lv, prm, f, rtol=1e-12)
        assert res.converged.all()
        errs.append(np.abs(res.u - uex).max())
        hs.append(hh)
    orders = np.log(np.array(errs[:-1]) / np.array(errs[1:])) / np.log(2)
    assert np.all((orders > 1.9) & (orders < 2.1)), orders


# ----------------------------------------------------------------------------- P5 closed-form eigenvalues
@pytest.mark.parametrize("coefs", [(1.0, 0.0), (0.9, 0.35), (1.1, -0.2, 0.3), (0.8, 0.1, -0.25, 0.2)])
def test_smoother_eigenvalues_closed_form(coefs):
    """With D_g = 4 I (ghost degree) on the 5-point Poisson matrix, D_A^{-1} A and
    D_g^{-1} A_g share the sine eigenbasis, and one learnable smoothing step maps
    the error mode v_pq to sigma v_pq with
    sigma = 1 - eta theta (sum_k c_k lam_hat^k) lam,  lam_hat = (cos p pi h + cos q pi h)/2,
    lam = 1 - lam_hat  (Sec. 3.3, eq. eigenvalue-S; K > 1 per the ChebConv remark)."""
    side = 17
    h = H.square_hierarchy(side)
    lv = levels_of(h, ghost_degree=4)
    J = h.nlevels
    K = len(coefs) - 1
    prm = O.unpack(C.identity_params(J, K, K, K), J, K, K, K)
    prm.theta[:] = 0.7
    prm.eta[:] = 0.9
    prm.cB[:] = np.array(coefs)
    hh = 1.0 / (side - 1)
    xs = np.arange(1, side - 1) * hh
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    for p, q in ((1, 1), (3, 5), (8, 2), (15, 15), (7, 14)):
        v = (np.sin(p * np.pi * X) * np.sin(q * np.pi * Y)).ravel()[:, None]
        lam_hat = 0.5 * (np.cos(p * np.pi * hh) + np.cos(q * np.pi * hh))
        lam = 1.0 - lam_hat
        poly = sum(c * lam_hat ** k for k, c in enumerate(coefs))
        sigma = 1.0 - 0.9 * 0.7 * poly * lam
        # error propagation: exact solution 0, f = 0, iterate u = v -> error -u
        out = O.smooth(lv[0], 0, prm, np.zeros_like(v), v)
        assert np.abs(out - sigma * v).max() < 1e-13


def test_graph_conv_equals_dense_power_sum():
    """Horner evaluation equals sum_k c_k (D_g^{-1} A_g)^k x with dense powers,
    and the neighbour mean is the mean over the matrix graph (Sec. 2.1)."""
    h = H.lshape_hierarchy(C.rng(4, 4, 7), target_nodes=60, refinements=1)
    lv = levels_of(h)[0]
    A = h.A[0].toarray()
    Ag = ((A != 0) & ~np.eye(len(A), dtype=bool)).astype(float)
    deg = Ag.sum(1)
    Mdense = Ag / deg[:, None]
    x = C.rng(9, 3, 0).standard_normal((len(A), 2))
    for c in ([0.7], [1.0, -0.4], [0.3, 0.2, -0.5], [1.2, 0.1, 0.05, -0.3]):
        want = sum(ck * np.linalg.matrix_power(Mdense, k) @ x for k, ck in enumerate(c))
        assert rel(O.graph_conv(np.array(c), lv, x), want) < 1e-14
    # the mean, node by node, from the definition
    i = 5
    nb = [j for j in range(len(A)) if j != i and A[i, j] != 0]
    assert abs(O.neighbour_mean(lv, x)[i, 0] - np.mean(x[nb, 0])) < 1e-15


# ----------------------------------------------------------------------------- P4 transfers / symmetry
def test_transfer_and_galerkin_properties():
    h = H.square_hierarchy(65, H.block_field(C.rng(9, 1, 1), 16, -2, 2))
    for l in range(h.nlevels - 1):
        assert (h.R[l] != h.P[l].T).nnz == 0
        Ac = h.A[l + 1]
        assert abs(Ac - Ac.T).max() == 0.0
        # P rows: coarse vertices copy (weight 1), midpoints average two ends;
        # an end on the Dirichlet boundary contributes 0 (two such ends: empty row)
        s = np.asarray(h.P[l].sum(axis=1)).ravel()
        assert set(np.unique(s)) <= {0.0, 0.5, 1.0}
        assert np.all(h.P[l].data == 0.5) or set(np.unique(h.P[l].data)) <= {0.5, 1.0}
    hc = H.square_hierarchy(65)
    hg = H.square_hierarchy(65, coarsening="geometric")
    for a, b in zip(hc.A, hg.A):
        assert (a != b).nnz == 0          # constant coefficient: Galerkin == rediscretisation


def _dense_B(lv, prm, n):
    """Columns of B_Theta: LMG(A, e_j, 0) (the cycle is linear in f at u = 0)."""
    return O.lmg(lv, prm, 0, np.eye(n), np.zeros((n, n)))


def test_cycle_symmetry_identity_vs_random():
    h = H.square_hierarchy(17, H.block_field(C.rng(9, 1, 2), 4, -1, 1))
    lv = levels_of(h)
    J, n = h.nlevels, h.sizes[0]
    prm = O.unpack(C.identity_params(J, 2, 2, 2), J, 2, 2, 2)
    Bm = _dense_B(lv, prm, n)
    assert np.abs(Bm - Bm.T).max() < 1e-13 * np.abs(Bm).max()
    prm = O.unpack(C.random_params(J, 2, 2, 2, seed=3), J, 2, 2, 2)
    Bm = _dense_B(lv, prm, n)
    assert np.abs(Bm - Bm.T).max() > 1e-3 * np.abs(Bm).max()


def test_two_level_coarse_correction_is_galerkin_orthogonal():
    """Without smoothing and with identity transfer convolutions, the exact
    two-level correction leaves an error A-orthogonal to range(P)."""
    h = H.square_hierarchy(33, H.block_field(C.rng(9, 1, 3), 8, -2, 2), nlevels=2)
    lv = levels_of(h)
    prm = O.unpack(C.identity_params(2, 1, 1, 1), 2, 1, 1, 1, nu_pre=0, nu_post=0)
    n = h.sizes[0]
    ustar = C.rng(9, 2, 5).standard_normal((n, 2))
    f = h.A[0] @ ustar
    u = C.rng(9, 2, 6).standard_normal((n, 2))
    e = ustar - O.lmg(lv, prm, 0, f, u)
    assert np.abs(h.P[0].T @ (h.A[0] @ e)).max() < 1e-11 * np.abs(h.A[0] @ (ustar - u)).max()


# ----------------------------------------------------------------------------- P3 brute force
def test_random_theta_affine_dense_and_rate():
    """Tiny grids, random Theta: (i) the cycle is u + B(f - A u) (Sec. 1);
    (ii) iterating it solves A u = f (dense solve); (iii) the observed rate is the
    spectral radius of I - B A."""
    h = H.square_hierarchy(17, H.block_field(C.rng(9, 1, 4), 4, -1, 1))
    lv = levels_of(h)
    J, n = h.nlevels, h.sizes[0]
    prm = O.unpack(C.random_params(J, 2, 2, 2, seed=1, spread=0.15), J, 2, 2, 2)
    Bm = _dense_B(lv, prm, n)
    A = h.A[0].toarray()
    g = C.rng(9, 2, 7)
    f, u = g.standard_normal((n, 3)), g.standard_normal((n, 3))
    assert rel(O.lmg(lv, prm, 0, f, u), u + Bm @ (f - A @ u)) < 1e-13
    E = np.eye(n) - Bm @ A
    rho = np.abs(np.linalg.eigvals(E)).max()
    assert rho < 1
    res = O.solve(lv, prm, f, rtol=1e-12)
    assert res.converged.all()
    ustar = np.linalg.solve(A, f)
    assert rel(res.u, ustar) < 1e-12 * np.linalg.cond(A)
    # error propagation: e_m = E^m e_0
    e = g.standard_normal((n, 1))
    norms = []
    for _ in range(60):
        e = O.lmg(lv, prm, 0, np.zeros_like(e), e)
        norms.append(np.linalg.norm(e))
    obs = (norms[-1] / norms[-21]) ** (1 / 20)
    assert abs(obs - rho) < 0.01 * rho


def _frac_cycle(A, P, theta, eta, cB, cR, cP, nu, l, f, u):
    """Alg. 2 in exact rational arithmetic on dense lists (tiny grids only).
    Graph convolutions are evaluated as explicit power sums."""
    n = len(A[l])
    J = len(A)

    def matvec(M, x):
        return [sum((M[i][j] * x[j] for j in range(len(x)) if M[i][j] != 0), Fraction(0)) for i in range(len(M))]

    def mean(x):
        out = []
        for i in range(n):
            nb = [x[j] for j in range(n) if j != i and A[l][i][j] != 0]
            out.append(sum(nb, Fraction(0)) / len(nb) if nb else Fraction(0))
        return out

    def conv(c, x):
        acc = [Fraction(0)] * n
        w = list(x)
        for k, ck in enumerate(c):
            if k:
                w = mean(w)
            acc = [a + ck * wi for a, wi in zip(acc, w)]
        return acc

    if l == J - 1:
        # Gauss-Jordan on [A | f]
        M = [row[:] + [f[i]] for i, row in enumerate(A[l])]
        for k in range(n):
            piv = next(i for i in range(k, n) if M[i][k] != 0)
            M[k], M[piv] = M[piv], M[k]
            for i in range(n):
                if i != k and M[i][k] != 0:
                    t = M[i][k] / M[k][k]
                    M[i] = [a - t * b for a, b in zip(M[i], M[k])]
        return [M[i][n] / M[i][i] for i in range(n)]

    def smooth_step(u):
        Au = matvec(A[l], u)
        d = [theta[l] * (f[i] - Au[i]) / A[l][i][i] for i in range(n)]
        ph = conv(cB[l], d)
        return [a + eta[l] * b for a, b in zip(u, ph)]

    for _ in range(nu):
        u = smooth_step(u)
    Au = matvec(A[l], u)
    r = [f[i] - Au[i] for i in range(n)]
    PT = [list(col) for col in zip(*P[l])]
    rc = matvec(PT, conv(cR[l], r))
    ec = _frac_cycle(A, P, theta, eta, cB, cR, cP, nu, l + 1, rc, [Fraction(0)] * len(rc))
    e = conv(cP[l], matvec(P[l], ec))
    u = [a + b for a, b in zip(u, e)]
    for _ in range(nu):
        u = smooth_step(u)
    return u


def test_exact_rational_cycle_tiny():
    """One learnable V(1,1) cycle on a 7 x 7 grid (3 levels) in exact rationals
    vs the FP64 oracle."""
    blocks = np.array([[1.0, 2.0], [3.0, 1.0]])
    h = H.square_hierarchy(9, blocks, nlevels=3)
    J = h.nlevels
    K = 2
    flat = C.identity_params(J, K, K, K).reshape(J - 1, -1)
    flat[:, 0] = [0.625, 0.75]
    flat[:, 1] = [1.125, 0.875]
    flat[:, 2:5] = [[1.0, 0.25, -0.125], [0.75, 0.5, 0.0625]]
    flat[:, 5:8] = [[1.25, -0.25, 0.125], [1.0, 0.125, 0.25]]
    flat[:, 8:11] = [[0.875, 0.375, -0.25], [1.0, -0.5, 0.125]]
    prm = O.unpack(flat.ravel(), J, K, K, K, nu_pre=1, nu_post=1)
    lv = levels_of(h)
    g = C.rng(9, 2, 8)
    f = g.standard_normal((h.sizes[0], 1))
    u = g.standard_normal((h.sizes[0], 1))
    want = O.lmg(lv, prm, 0, f, u)[:, 0]
    Fr = lambda M: [[Fraction(float(v)) for v in row] for row in M.toarray()]
    A = [Fr(a) for a in h.A]
    P = [Fr(p) for p in h.P]
    fr = lambda v: [Fraction(float(x)) for x in v]
    out = _frac_cycle(A, P, fr(prm.theta), fr(prm.eta), [fr(c) for c in prm.cB], [fr(c) for c in prm.cR],
                      [fr(c) for c in prm.cP], 1, 0, fr(f[:, 0]), fr(u[:, 0]))
    exact = np.array([float(x) for x in out])
    assert rel(want, exact) < 1e-14


# ----------------------------------------------------------------------------- P6 proposition
def test_proposition_learnable_smoothing_factor_not_worse():
    """min over (w1, w2, theta, eta) of rho(S_w) <= min over omega of rho(S_omega)
    (Sec. 3.3, Proposition), with S built column by column from the oracle."""
    h = H.square_hierarchy(9, H.block_field(C.rng(9, 1, 5), 2, -1, 1))
    lv = levels_of(h)
    J, n = h.nlevels, h.sizes[0]
    I = np.eye(n)

    def rho(theta, eta, c):
        prm = O.unpack(C.identity_params(J, 1, 1, 1), J, 1, 1, 1)
        prm.theta[0], prm.eta[0], prm.cB[0] = theta, eta, np.array(c)
        S = O.smooth(lv[0], 0, prm, np.zeros((n, n)), I)
        return np.abs(np.linalg.eigvals(S)).max()

    omegas = np.linspace(0.05, 1.2, 47)
    jac = [rho(w, 1.0, (1.0, 0.0)) for w in omegas]
    best_w = omegas[int(np.argmin(jac))]
    # the learnable family contains Jacobi, so its grid minimum cannot be larger
    grid = [rho(best_w, 1.0, (w1, w2)) for w1 in np.linspace(0.6, 1.4, 9) for w2 in np.linspace(-0.5, 0.5, 11)]
    assert min(grid) <= min(jac) + 1e-15
    # and Jacobi is the member with w1 = 1, w2 = 0 (eq. eigenvalue-jacobi):
    Dinv = 1.0 / h.A[0].diagonal()
    Sj = I - best_w * Dinv[:, None] * h.A[0].toarray()
    assert abs(np.abs(np.linalg.eigvals(Sj)).max() - min(jac)) < 1e-13


def test_given_graph_ignores_diagonal_and_adds_mesh_edges():
    """A given pattern defines N(i) without i itself (edges join distinct nodes,
    Sec. 2.1); the mean of node i is over exactly the listed neighbours."""
    h = H.square_hierarchy(9)
    A = h.A[0]
    n = A.shape[0]
    G = (A != 0).astype(float).tolil()
    G[0, n - 1] = 1.0
    G[n - 1, 0] = 1.0
    lv = O.make_levels(h.A, h.P, h.R, [sp.csr_matrix(G)] + [None] * (h.nlevels - 1))[0]
    x = np.arange(n, dtype=float)[:, None]
    nb0 = [j for j in range(n) if j != 0 and (A[0, j] != 0 or j == n - 1)]
    assert abs(O.neighbour_mean(lv, x)[0, 0] - np.mean(x[nb0, 0])) < 1e-15 * n
    assert lv.G.diagonal().sum() == 0


def test_generated_operators_exactly_symmetric():
    for h in (H.square_hierarchy(33, H.block_field(C.rng(9, 1, 9), 16, -3, 3)),
              H.lshape_hierarchy(C.rng(4, 4, 1), target_nodes=150, refinements=2)):
        for a in h.A:
            assert (a != a.T).nnz == 0

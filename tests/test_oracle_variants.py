"""Pins of the trainable parameterisations (shared Phi_R/Phi_P, LMG-RP,
LMG-RPS; Sec. 4.1) and of the Darcy input generator."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from mginputs import configs as C, darcy as D, hierarchy as H
from oracle import adjoint as AD
from oracle import lmg as O
from oracle import variants as V

J, K = 3, 2
NPHI = {"full": (J - 1) * (2 + 3 * (K + 1)), "shared": (J - 1) * (3 + K) + 2 * (K + 1),
        "rp": 2 * (K + 1), "rps": (J - 1) * (2 + K) + 2 * (K + 1)}


@pytest.mark.parametrize("name", ["shared", "rp", "rps"])
def test_expand_ties_and_fixes_what_the_paper_says(name):
    phi = C.rng(8, 1, 0).standard_normal(NPHI[name])
    p = V.expand(name, phi, J, K, K, K)
    assert np.all(p.cR == p.cR[0]) and np.all(p.cP == p.cP[0])      # one Phi_R, one Phi_P
    assert np.array_equal(p.cR[0], phi[-2 * (K + 1):-(K + 1)]) and np.array_equal(p.cP[0], phi[-(K + 1):])
    if name in ("rp", "rps"):
        assert np.all(p.theta == 2.0 / 3.0)                          # theta fixed at omega
    if name == "rp":                                                 # damped Jacobi smoother
        assert np.all(p.eta == 1.0) and np.all(p.cB[:, 0] == 1.0) and np.all(p.cB[:, 1:] == 0.0)


@pytest.mark.parametrize("name", ["full", "shared", "rp", "rps"])
def test_grad_phi_matches_central_differences(name):
    """The unrolled loss as a function of phi, differentiated by central
    differences, against grad_phi of the oracle's reverse sweep."""
    h = H.square_hierarchy(9, H.block_field(C.rng(8, 2, 0), 4, -1, 1))
    lv = O.make_levels(h.A, h.P, h.R)
    f = C.rng(8, 3, 0).standard_normal((h.sizes[0], 2))
    phi = C.rng(8, 4, 0).uniform(-0.2, 0.2, NPHI[name])
    # near the identity initialisation in each parameterisation
    if name in ("full", "shared"):
        phi += np.concatenate([[2 / 3, 1.0, 1.0, 0.0, 0.0] + ([1.0, 0.0, 0.0] * 2 if name == "full" else [])
                               for _ in range(J - 1)] + ([[1.0, 0, 0, 1.0, 0, 0]] if name == "shared" else []))
    elif name == "rps":
        phi += np.concatenate([[1.0, 1.0, 0.0, 0.0] for _ in range(J - 1)] + [[1.0, 0, 0, 1.0, 0, 0]])
    else:
        phi += np.array([1.0, 0, 0, 1.0, 0, 0])

    def loss(x):
        return AD.unrolled_loss(lv, V.expand(name, x, J, K, K, K), f, cycles=3)

    _, g = AD.unrolled_loss_and_grad(lv, V.expand(name, phi, J, K, K, K), f, cycles=3)
    gp = V.grad_phi(name, g, J, K, K, K)
    eps = 1e-6
    fd = np.array([(loss(phi + eps * e) - loss(phi - eps * e)) / (2 * eps) for e in np.eye(phi.size)])
    assert np.abs(fd - gp).max() <= 1e-6 * max(np.abs(gp).max(), 1e-12)


def test_darcy_uniform_conductivity_gives_the_linear_pressure():
    """k = 1, p = 1 at x = 0, p = 0 at x = 1, no flow top and bottom: the
    exact solution 1 - x is reproduced at the cell centres (TPFA is exact
    for linear pressures)."""
    n = 20
    A, b = D.tpfa(np.ones((n, n)))
    p = spla.spsolve(A.tocsc(), b)
    X, _ = D.cell_centres(n)
    assert np.abs(p - (1 - X.ravel())).max() <= 1e-12
    assert abs(A - A.T).max() == 0.0


def test_darcy_flux_balance_through_an_inclusion():
    """Mass conservation: the flux entering on the left equals the flux
    leaving on the right, for the paper's 1e-6 inclusion."""
    n = 40
    k = D.inclusion_field(n)
    A, b = D.tpfa(k)
    p = spla.spsolve(A.tocsc(), b).reshape(n, n)
    q_in = np.sum(2 * k[:, 0] * (1.0 - p[:, 0]))
    q_out = np.sum(2 * k[:, -1] * (p[:, -1] - 0.0))
    assert abs(q_in - q_out) <= 1e-10 * abs(q_in)


def test_darcy_aggregation_hierarchy():
    """Piecewise constant P: one unit entry per fine row; 100 cells give the
    paper's 7 levels down to 2 x 2; Galerkin products stay 5-point."""
    k = D.inclusion_field(100)
    h, b = D.darcy_hierarchy(k, 7)
    assert h.sizes == [10000, 2500, 625, 169, 49, 16, 4]
    for P in h.P:
        assert np.all(np.diff(P.indptr) == 1) and np.all(P.data == 1.0)
    for A in h.A:
        assert A.getnnz(axis=1).max() <= 5 and abs(A - A.T).max() == 0.0


def test_darcy_classical_cycle_converges():
    """Identity parameters (damped Jacobi, nu = 4, piecewise constant P)
    converge on the inclusion problem from a random start."""
    k = D.inclusion_field(40)
    h, b = D.darcy_hierarchy(k, 5)
    lv = O.make_levels(h.A, h.P, h.R)
    prm = O.unpack(C.identity_params(5, 1, 1, 1), 5, 1, 1, 1, 4, 4)
    u0 = C.rng(8, 5, 0).standard_normal((h.sizes[0], 1))
    res = O.solve(lv, prm, b[:, None], rtol=1e-8, u0=u0, max_cycles=500)
    assert res.converged.all() and res.iters[0] < 200

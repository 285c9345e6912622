"""Pins of the convolution variants: Chebyshev basis (the ChebConv layer of
Sec. 3.2 with the symmetric or random-walk normalisation) and weighted
aggregation (edge weights from matrix entries, Sec. 2.1)."""
import numpy as np
import numpy.polynomial.chebyshev as npc
import pytest
import scipy.sparse as sp

from mginputs import configs as C, hierarchy as H
from oracle import adjoint as AD
from oracle import lmg as O


def _lv(agg, side=9, coef=True):
    blocks = H.block_field(C.rng(8, 9, 0), 4, -1, 1) if coef else None
    h = H.square_hierarchy(side, blocks)
    return h, O.make_levels(h.A, h.P, h.R, aggregation=agg)


def test_chebyshev_sym_equals_spectral_evaluation():
    """S = D^-1/2 A_g D^-1/2 is symmetric: Phi = V diag(sum_k c_k T_k(-lam)) V^T,
    with the Chebyshev series evaluated by numpy (chebval) on the eigenvalues."""
    h, lv = _lv("sym")
    S = lv[0].Gw.toarray()
    assert np.allclose(S, S.T, atol=0)
    lam, V = np.linalg.eigh(S)
    c = np.array([0.7, -0.3, 0.2, 0.15])
    x = C.rng(8, 10, 0).standard_normal((S.shape[0], 2))
    want = V @ (npc.chebval(-lam, c)[:, None] * (V.T @ x))
    got = O.graph_conv(c, lv[0], x, "chebyshev")
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_chebyshev_mean_equals_power_series():
    """Random-walk normalisation: sum_k c_k T_k(-M) = sum_m a_m M^m with a the
    power-series coefficients of the Chebyshev series in -t (numpy cheb2poly),
    applied with dense matrix powers."""
    h, lv = _lv("mean")
    M = (sp.diags(lv[0].inv_deg) @ lv[0].G).toarray()
    c = np.array([0.5, 0.4, -0.25, 0.1])
    a = npc.cheb2poly(c) * (-1.0) ** np.arange(len(c))
    x = C.rng(8, 11, 0).standard_normal((M.shape[0], 3))
    want = sum(a[m] * np.linalg.matrix_power(M, m) @ x for m in range(len(a)))
    got = O.graph_conv(c, lv[0], x, "chebyshev")
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_sym_is_similar_to_the_mean():
    h, lv = _lv("sym")
    _, lm = _lv("mean")
    M = (sp.diags(lm[0].inv_deg) @ lm[0].G).toarray()
    d = 1.0 / lm[0].inv_deg
    S = lv[0].Gw.toarray()
    assert np.abs(S - np.diag(np.sqrt(d)) @ M @ np.diag(1 / np.sqrt(d))).max() <= 1e-14


def test_weighted_equals_mean_for_constant_coefficients_and_is_row_stochastic():
    """Constant coefficient: every off-diagonal entry of the 5-point stencil is
    the same, so weighting by |a_ij| is the plain mean; with variable
    coefficients the weighted operator differs but still averages (rows sum
    to one)."""
    _, lw = _lv("weighted", coef=False)
    _, lm = _lv("mean", coef=False)
    x = C.rng(8, 12, 0).standard_normal((lw[0].A.shape[0], 2))
    assert np.abs(O.neighbour_mean(lw[0], x) - O.neighbour_mean(lm[0], x)).max() <= 1e-15
    _, lw2 = _lv("weighted")
    _, lm2 = _lv("mean")
    one = np.ones((lw2[0].A.shape[0], 1))
    assert np.abs(O.neighbour_mean(lw2[0], one) - 1.0).max() <= 1e-14
    assert np.abs(O.neighbour_mean(lw2[0], x) - O.neighbour_mean(lm2[0], x)).max() > 1e-3


@pytest.mark.parametrize("agg,basis", [("sym", "chebyshev"), ("weighted", "monomial"), ("mean", "chebyshev"),
                                       ("weighted", "chebyshev")])
def test_variant_gradients_match_central_differences(agg, basis):
    h, lv = _lv(agg)
    J = h.nlevels
    flat = C.random_params(J, 2, 2, 2, seed=90, spread=0.2)
    f = C.rng(8, 13, 0).standard_normal((h.sizes[0], 2))
    prm = O.unpack(flat, J, 2, 2, 2, basis=basis)
    _, g = AD.unrolled_loss_and_grad(lv, prm, f, cycles=3)
    gflat = O.pack(g)
    eps = 1e-6
    for i in range(flat.size):
        e = np.zeros_like(flat)
        e[i] = eps
        fd = (AD.unrolled_loss(lv, O.unpack(flat + e, J, 2, 2, 2, basis=basis), f, 3)
              - AD.unrolled_loss(lv, O.unpack(flat - e, J, 2, 2, 2, basis=basis), f, 3)) / (2 * eps)
        assert abs(fd - gflat[i]) <= 1e-6 * np.abs(gflat).max(), (i, fd, gflat[i])


def test_planted_recurrence_sign_error_is_caught():
    """A Chebyshev evaluation with T_1 = +S x (sign error) disagrees with the
    spectral pin, so the pin would catch it."""
    h, lv = _lv("sym")
    S = lv[0].Gw.toarray()
    lam, V = np.linalg.eigh(S)
    c = np.array([0.7, -0.3, 0.2, 0.15])
    x = C.rng(8, 10, 0).standard_normal((S.shape[0], 1))
    want = V @ (npc.chebval(-lam, c)[:, None] * (V.T @ x))
    t0, t1 = x, S @ x
    bad = c[0] * t0 + c[1] * t1
    for k in range(1, 3):
        t0, t1 = t1, 2 * S @ t1 - t0
        bad = bad + c[k + 1] * t1
    assert np.abs(bad - want).max() > 1e-3

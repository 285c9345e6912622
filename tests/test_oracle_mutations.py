"""The pins must catch plausible oracle mistakes.

Each case plants one mistake in the CPU oracle (monkeypatched, in this process
only) and checks that at least one pin then fails.
"""
import numpy as np
import pytest

from oracle import adjoint as AD
from oracle import lmg as O

import tests.test_oracle_adjoint as TA
import tests.test_oracle_pins as TP


def _fails(*tests):
    for t, args in tests:
        try:
            t(*args)
        except AssertionError:
            return True
    return False


def _transposed_mean(lv, x):
    return lv.G.T @ (lv.inv_deg[:, None] * x)


def _reversed_horner(c, lv, x, basis="monomial"):
    K = len(c) - 1
    y = c[0] * x
    for k in range(1, K + 1):
        y = O.neighbour_mean(lv, y) + c[k] * x
    return y


def _smooth_no_theta(lv, l, prm, f, u):
    delta = lv.Dinv[:, None] * O.residual(lv, f, u)
    return u + prm.eta[l] * O.graph_conv(prm.cB[l], lv, delta)


def _smooth_sign(lv, l, prm, f, u):
    delta = prm.theta[l] * (lv.Dinv[:, None] * (lv.A @ u - f))
    return u + prm.eta[l] * O.graph_conv(prm.cB[l], lv, delta)


def _smooth_phi_before_scale(lv, l, prm, f, u):
    # applies the convolution to the raw residual and B afterwards (wrong order)
    r = O.residual(lv, f, u)
    return u + prm.eta[l] * prm.theta[l] * lv.Dinv[:, None] * O.graph_conv(prm.cB[l], lv, r)


PIN_FORWARD = [
    (TP.test_smoother_eigenvalues_closed_form, ((0.9, 0.35),)),
    (TP.test_smoother_eigenvalues_closed_form, ((1.1, -0.2, 0.3),)),
    (TP.test_graph_conv_equals_dense_power_sum, ()),
    (TP.test_exact_rational_cycle_tiny, ()),
    (TP.test_identity_params_recover_classical_vcycle, ("blocks",)),
    (TP.test_two_level_coarse_correction_is_galerkin_orthogonal, ()),
    (TP.test_manufactured_solution_second_order, ()),
]


@pytest.mark.parametrize("target,name,impl", [
    (O, "neighbour_mean", _transposed_mean),
    (O, "graph_conv", _reversed_horner),
    (O, "smooth", _smooth_no_theta),
    (O, "smooth", _smooth_sign),
    (O, "smooth", _smooth_phi_before_scale),
])
def test_forward_mutation_is_caught(monkeypatch, target, name, impl):
    monkeypatch.setattr(target, name, impl)
    # modules that imported the name directly see the mutation too
    if hasattr(AD, name):
        monkeypatch.setattr(AD, name, impl)
    assert _fails(*PIN_FORWARD)


def test_transfer_mutations_are_caught(monkeypatch):
    orig = O.lmg

    def lmg_no_phiR(levels, prm, l, f, u):
        saved = prm.cR.copy()
        prm.cR[:] = 0.0
        prm.cR[:, 0] = 1.0
        try:
            return orig(levels, prm, l, f, u)
        finally:
            prm.cR[:] = saved

    monkeypatch.setattr(O, "lmg", lmg_no_phiR)
    assert _fails((TP.test_exact_rational_cycle_tiny, ()))
    monkeypatch.undo()

    def make_levels_half_R(A, P, R=None, G=None, ghost_degree=None):
        lv = O.make_levels(A, P, R, G, ghost_degree)
        for x in lv[:-1]:
            x.R = 0.5 * x.R
        return lv

    monkeypatch.setattr(TP, "levels_of", lambda h, **kw: make_levels_half_R(h.A, h.P, h.R, **kw))
    assert _fails((TP.test_two_level_coarse_correction_is_galerkin_orthogonal, ()),
                  (TP.test_identity_params_recover_classical_vcycle, ("blocks",)))


@pytest.mark.parametrize("which", ["meanT", "theta_grad", "ubar_sign"])
def test_adjoint_mutation_is_caught(monkeypatch, which):
    if which == "meanT":
        monkeypatch.setattr(AD, "neighbour_mean_T", lambda lv, y: O.neighbour_mean(lv, y))
    elif which == "theta_grad":
        orig = AD._smooth_vjp

        def no_theta(lv, l, prm, f, u, g, grads):
            t = grads.theta[l]
            out = orig(lv, l, prm, f, u, g, grads)
            grads.theta[l] = t
            return out
        monkeypatch.setattr(AD, "_smooth_vjp", no_theta)
    else:
        orig = AD._smooth_vjp

        def flipped(lv, l, prm, f, u, g, grads):
            s, gu = orig(lv, l, prm, f, u, g, grads)
            return s, 2 * g - gu                      # g + A^T s instead of g - A^T s
        monkeypatch.setattr(AD, "_smooth_vjp", flipped)
    assert _fails((TA.test_adjoint_matches_torch_autograd, (1,)), (TA.test_adjoint_matches_torch_autograd, (3,)))

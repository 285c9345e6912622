"""GPU parity of the Darcy workload (cell-centred, piecewise constant
interpolation, nu = 4; Sec. 4.1) and of the trainable parameterisations
(shared Phi_R/Phi_P, LMG-RP, LMG-RPS) against the oracle."""
import numpy as np
import pytest

from mginputs import configs as C, darcy as D
from oracle import adjoint as AD
from oracle import lmg as O
from oracle import variants as V
from tests.gpu_util import ctx_for, oracle_levels, oracle_params, elem_rel, to_dev, to_np

pytestmark = pytest.mark.gpu


def _darcy(n=40, J=5, k=None):
    return D.darcy_hierarchy(D.inclusion_field(n) if k is None else k, J)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_darcy_cycle_matches_oracle(prec, tol):
    import torch
    h, b = _darcy()
    J = h.nlevels
    flat = C.random_params(J, 3, 3, 3, seed=80, spread=0.2)
    u = C.rng(9, 7, 0).standard_normal((h.sizes[0], 3))
    f = np.repeat(b[:, None], 3, axis=1)
    want = O.lmg(oracle_levels(h), oracle_params(flat, J, 3, nu=(4, 4)), 0, f, u)
    ctx = ctx_for(h, flat, 3, 3, prec, nu=(4, 4))
    ud = to_dev(u, ctx.cycle_dtype)
    ctx.vcycle(to_dev(f, ctx.cycle_dtype), ud)
    err = elem_rel(to_np(ud), want)
    print(f"darcy {prec} cycle rel {err:.2e}", flush=True)
    assert err <= tol


@pytest.mark.parametrize("field", ["inclusion", "two-regions", "channels", "random-80"])
def test_darcy_fields_solve_from_random_start(field):
    """The paper's full-size Darcy setting (100 x 100 cells, 7 levels, random
    initial iterate) and the test-field stand-ins: FP32 cycles in FP64
    refinement reach 1e-8 (host FP64 residual)."""
    import torch
    k = {"inclusion": lambda: D.inclusion_field(100), "two-regions": lambda: D.two_regions_field(100),
         "channels": lambda: D.channels_field(100),
         "random-80": lambda: D.random_field(C.rng(9, 1, 0), 40, 80)}[field]()
    h, b = D.darcy_hierarchy(k, 7)
    J = h.nlevels
    B = 4
    f = np.repeat(b[:, None], B, axis=1)
    u0 = C.rng(9, 2, 100).standard_normal((h.sizes[0], B))
    ctx = ctx_for(h, C.identity_params(J, 3, 3, 3), 3, B, "fp32", nu=(4, 4), max_outer=5000)
    u = to_dev(u0, torch.float64)
    info = ctx.solve(to_dev(f, torch.float64), u)
    rr = np.linalg.norm(f - h.A[0] @ to_np(u), axis=0) / np.linalg.norm(f, axis=0)
    print(f"darcy {field}: cycles {info.iters} relres {rr.max():.2e}", flush=True)
    assert info.code == 0 and rr.max() <= 1e-8 * (1 + 1e-3)


@pytest.mark.parametrize("name", ["full", "shared", "rp", "rps"])
def test_variant_gradient_matches_oracle(name):
    """Unrolled-loss gradient with respect to the trainable vector phi of each
    parameterisation: torch autograd through params.Variant and the library's
    reverse sweep (FP64) against the oracle's grad_phi."""
    import torch
    from paper_2608_29082_amd import autograd as AG
    from paper_2608_29082_amd import params as PR
    h, b = _darcy()
    J, K, B = h.nlevels, 2, 3
    var = PR.Variant(name, J, K, K, K)
    g = C.rng(9, 8, 0)
    phi0 = var.initial() + g.uniform(-0.1, 0.1, var.nphi)
    f = np.repeat(b[:, None], B, axis=1)
    u0 = g.standard_normal((h.sizes[0], B))
    ctx = ctx_for(h, var.expand(phi0), K, B, "fp64", nu=(4, 4), backward=True)
    phi = torch.tensor(phi0, dtype=torch.float64, requires_grad=True)
    L = AG.unrolled_loss(ctx, var.expand(phi), to_dev(f, torch.float64), cycles=4, u0=to_dev(u0, torch.float64))
    L.backward()
    Lo, go = AD.unrolled_loss_and_grad(oracle_levels(h), V.expand(name, phi0, J, K, K, K, nu_pre=4, nu_post=4), f,
                                       cycles=4, u0=u0)
    want = V.grad_phi(name, go, J, K, K, K)
    err = elem_rel(phi.grad.numpy(), want)
    print(f"variant {name}: loss {L.item():.6e} vs {Lo:.6e}, grad rel {err:.2e}", flush=True)
    assert abs(L.item() - Lo) <= 1e-10 * Lo
    assert err <= 1e-9

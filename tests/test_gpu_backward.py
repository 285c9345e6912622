"""GPU reverse sweep (training through the cycle) against the oracle's
hand-written adjoint and central finite differences in FP64."""
import numpy as np
import pytest

from mginputs import configs as C, hierarchy as H
from oracle import adjoint as AD
from oracle import lmg as O
from tests.gpu_util import ctx_for, oracle_levels, oracle_params, elem_rel, small_cases, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("case", ["poisson33", "blocks65", "lshape"])
@pytest.mark.parametrize("K", [0, 1, 3])
def test_vcycle_backward_matches_oracle_vjp(case, K):
    import torch
    hier = dict(small_cases())[case]
    J = hier.nlevels
    flat = C.random_params(J, K, K, K, seed=K + 3)
    g = C.rng(5, 1, K)
    B = 3
    f = g.standard_normal((hier.sizes[0], B))
    u = g.standard_normal((hier.sizes[0], B))
    gu = g.standard_normal((hier.sizes[0], B))
    fbar, ubar, grads = AD.cycle_vjp(oracle_levels(hier), oracle_params(flat, J, K), f, u, gu)
    ctx = ctx_for(hier, flat, K, B, "fp64", backward=True)
    ck = ctx.new_ckpt()
    ud = to_dev(u, torch.float64)
    ctx.vcycle(to_dev(f, torch.float64), ud, ckpt=ck)
    gin, gf, gp = ctx.vcycle_backward(ck, to_dev(gu, torch.float64))
    torch.cuda.synchronize()
    want_u = O.lmg(oracle_levels(hier), oracle_params(flat, J, K), 0, f, u)
    assert elem_rel(to_np(ud), want_u) <= 1e-12
    e = (elem_rel(to_np(gf), fbar), elem_rel(to_np(gin), ubar), elem_rel(to_np(gp), O.pack(grads)))
    print(case, K, e, flush=True)
    assert max(e) <= 1e-10


def test_refine_step_backward_matches_oracle():
    """u_out = u + C(f - A u): gu_in = gu - A C^T gu, gf = C^T gu."""
    import torch
    hier = dict(small_cases())["blocks65"]
    J = hier.nlevels
    flat = C.random_params(J, 2, 2, 2, seed=7)
    g = C.rng(5, 2, 0)
    f = g.standard_normal((hier.sizes[0], 2))
    u = g.standard_normal((hier.sizes[0], 2))
    gu = g.standard_normal((hier.sizes[0], 2))
    lv = oracle_levels(hier)
    prm = oracle_params(flat, J, 2)
    r = f - hier.A[0] @ u
    rbar, _, grads = AD.cycle_vjp(lv, prm, r, np.zeros_like(u), gu)
    want_gu = gu - hier.A[0].T @ rbar
    ctx = ctx_for(hier, flat, 2, 2, "fp64", backward=True)
    ck = ctx.new_ckpt()
    ctx.refine_step(to_dev(f, torch.float64), to_dev(u, torch.float64), ckpt=ck)
    gin, gf, gp = ctx.refine_step_backward(ck, to_dev(gu, torch.float64))
    torch.cuda.synchronize()
    assert elem_rel(to_np(gf), rbar) <= 1e-10
    assert elem_rel(to_np(gin), want_gu) <= 1e-10
    assert elem_rel(to_np(gp), O.pack(grads)) <= 1e-10


def test_unrolled_training_gradient_fd_fp64():
    """Loss mean_b ||f_b - A u^m||^2/||f_b||^2 after m unrolled refinement steps
    (FP64 context): autograd through the library vs central FD, step 1e-6."""
    import torch
    from paper_2608_29082_amd import autograd as AG
    w = C.block_diffusion(3, 65, -2, 2, B=4, K=3, precision="fp64")
    J = w.hier.nlevels
    flat = C.random_params(J, 3, 3, 3, seed=12, spread=0.1)
    ctx = ctx_for(w.hier, flat, 3, 4, "fp64", backward=True)
    f = to_dev(w.f, torch.float64)

    def loss_at(p, grad=False):
        theta = torch.tensor(p, dtype=torch.float64, device="cuda", requires_grad=grad)
        L = AG.unrolled_loss(ctx, theta, f, cycles=4)
        if grad:
            L.backward()
            return L.item(), theta.grad.cpu().numpy()
        return L.item()

    L0, gr = loss_at(flat, True)
    lo = O.make_levels(w.hier.A, w.hier.P, w.hier.R)
    Lo, go = AD.unrolled_loss_and_grad(lo, O.unpack(flat, J, 3, 3, 3), w.f, cycles=4)
    assert abs(L0 - Lo) <= 1e-10 * Lo
    assert elem_rel(gr, O.pack(go)) <= 1e-8
    step = 1e-6
    idx = np.argsort(-np.abs(gr))[:12]
    for i in idx:
        pp, pm = flat.copy(), flat.copy()
        pp[i] += step
        pm[i] -= step
        fd = (loss_at(pp) - loss_at(pm)) / (2 * step)
        assert abs(fd - gr[i]) <= 1e-5 * np.abs(gr).max(), (i, fd, gr[i])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("kind", ["mean_rel_sq", "resid_norm"])
def test_residual_loss_matches_oracle(kind, prec):
    """mg_residual_loss (loss, dL/du, dL/df scaled by a cotangent seed) against
    the oracle's hand gradients, element by element, with a column that takes
    no part (f = 0; for the norm also u = 0, so r = 0 exactly) and B = 5; then
    the same through the autograd node with gradients for f and u."""
    import torch
    from paper_2608_29082_amd import autograd as AG
    hier = dict(small_cases())["blocks65"]
    J = hier.nlevels
    A = hier.A[0]
    B = 5
    g = C.rng(5, 40, 0)
    f = g.standard_normal((hier.sizes[0], B))
    u = g.standard_normal((hier.sizes[0], B))
    f[:, 3] = 0.0
    if kind == "resid_norm":
        u[:, 3] = 0.0
    L, gu, gf = AD.residual_loss_grads(A, f, u, kind)
    ctx = ctx_for(hier, C.identity_params(J, 1, 1, 1), 1, B, prec, backward=True)
    seed = torch.tensor([0.7], dtype=torch.float64, device="cuda")
    fd_, ud_ = to_dev(f, torch.float64), to_dev(u, torch.float64)
    Ld, gud, gfd = ctx.residual_loss(fd_, ud_, kind=kind, gseed=seed, want_gu=True, want_gf=True)
    e = (abs(Ld.item() - L) / L, elem_rel(to_np(gud), 0.7 * gu), elem_rel(to_np(gfd), 0.7 * gf))
    print(f"{kind} {prec}: loss rel {e[0]:.1e}, gu {e[1]:.1e}, gf {e[2]:.1e}", flush=True)
    assert e[0] <= 1e-14 and e[1] <= 1e-13 and e[2] <= 1e-13
    assert float(gud[:, 3].abs().max()) == 0.0 and float(gfd[:, 3].abs().max()) == 0.0
    ft = fd_.clone().requires_grad_(True)
    ut = ud_.clone().requires_grad_(True)
    Lt = AG.ResidualLoss.apply(ctx, ft, ut, kind)
    (3.0 * Lt).backward()
    assert abs(Lt.item() - L) <= 1e-14 * L
    assert elem_rel(to_np(ut.grad), 3.0 * gu) <= 1e-13
    assert elem_rel(to_np(ft.grad), 3.0 * gf) <= 1e-13
    ctx.close()


def test_residual_loss_du_needs_backward_context():
    """dL/du uses A^T = A, which only a context set up for the reverse sweep has
    checked: without MG_FLAG_BACKWARD the call is refused; the loss alone works."""
    import torch
    from paper_2608_29082_amd.binding import MGError
    hier = dict(small_cases())["poisson33"]
    J = hier.nlevels
    ctx = ctx_for(hier, C.identity_params(J, 1, 1, 1), 1, 2, "fp64")
    f = to_dev(C.rng(5, 41, 0).standard_normal((hier.sizes[0], 2)), torch.float64)
    L, _, _ = ctx.residual_loss(f, torch.zeros_like(f))
    assert abs(L.item() - 1.0) <= 1e-15
    with pytest.raises(MGError):
        ctx.residual_loss(f, torch.zeros_like(f), want_gu=True)
    ctx.close()

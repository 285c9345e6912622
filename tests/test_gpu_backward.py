"""GPU reverse sweep (training through the cycle) against the oracle's
hand-written adjoint and central finite differences in FP64."""
import numpy as np
import pytest

from mginputs import configs as C, hierarchy as H
from oracle import adjoint as AD
from oracle import lmg as O
from tests.gpu_util import ctx_for, oracle_levels, oracle_params, rel, small_cases, to_dev, to_np

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
    assert rel(to_np(ud), want_u) <= 1e-12
    e = (rel(to_np(gf), fbar), rel(to_np(gin), ubar), rel(to_np(gp), O.pack(grads)))
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
    assert rel(to_np(gf), rbar) <= 1e-10
    assert rel(to_np(gin), want_gu) <= 1e-10
    assert rel(to_np(gp), O.pack(grads)) <= 1e-10


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
    assert rel(gr, O.pack(go)) <= 1e-8
    step = 1e-6
    idx = np.argsort(-np.abs(gr))[:12]
    for i in idx:
        pp, pm = flat.copy(), flat.copy()
        pp[i] += step
        pm[i] -= step
        fd = (loss_at(pp) - loss_at(pm)) / (2 * step)
        assert abs(fd - gr[i]) <= 1e-5 * np.abs(gr).max(), (i, fd, gr[i])

"""Parity at the workloads' full sizes, in the launch configurations the
benchmark and the training CLI use."""
import numpy as np
import pytest

from mginputs import configs as C
from oracle import adjoint as AD
from oracle import lmg as O
from tests.gpu_util import ctx_for, oracle_levels, oracle_params, elem_rel, to_dev, to_np

pytestmark = pytest.mark.gpu


def test_training_257_gradient_full_size_fd_and_oracle():
    """257 x 257, 7 levels, 32 rhs, K = 3 (84 parameters), 10 unrolled V(2,2)
    refinement steps, FP64 context: autograd through the library against the
    oracle's gradient and against central finite differences (step 1e-6)."""
    import torch
    from paper_2608_29082_amd import autograd as AG
    w = C.training_257()
    J = w.hier.nlevels
    flat = C.random_params(J, 3, 3, 3, seed=40, spread=0.1)
    ctx = ctx_for(w.hier, flat, 3, w.B, "fp64", backward=True)
    f = to_dev(w.f, torch.float64)

    def loss(p, grad=False):
        th = torch.tensor(p, dtype=torch.float64, requires_grad=grad)
        L = AG.unrolled_loss(ctx, th, f, cycles=10)
        if grad:
            L.backward()
            return L.item(), th.grad.numpy().copy()
        return L.item()

    L0, g = loss(flat, True)
    Lo, go = AD.unrolled_loss_and_grad(oracle_levels(w.hier), O.unpack(flat, J, 3, 3, 3), w.f, cycles=10)
    go = O.pack(go)
    print(f"loss gpu {L0:.6e} oracle {Lo:.6e}; grad rel {elem_rel(g, go):.2e}", flush=True)
    assert abs(L0 - Lo) <= 1e-9 * Lo
    assert elem_rel(g, go) <= 1e-7
    step = 1e-6
    for i in list(np.argsort(-np.abs(g))[:6]) + [0, 1, 2 + 1, 2 + 3 + 1 + 2]:
        pp, pm = flat.copy(), flat.copy()
        pp[i] += step
        pm[i] -= step
        fd = (loss(pp) - loss(pm)) / (2 * step)
        assert abs(fd - g[i]) <= 1e-5 * np.abs(g).max(), (i, fd, g[i])


def test_training_257_fp32_gradient_close_to_fp64():
    """The FP32 context (the training configuration) gives the FP64 gradient to
    the accuracy of FP32 cycles."""
    import torch
    from paper_2608_29082_amd import autograd as AG
    w = C.training_257()
    J = w.hier.nlevels
    flat = C.random_params(J, 3, 3, 3, seed=41, spread=0.1)
    grads = {}
    for prec in ("fp64", "fp32"):
        ctx = ctx_for(w.hier, flat, 3, w.B, prec, backward=True)
        th = torch.tensor(flat, dtype=torch.float64, requires_grad=True)
        L = AG.unrolled_loss(ctx, th, to_dev(w.f, torch.float64), cycles=10)
        L.backward()
        grads[prec] = th.grad.numpy().copy()
    assert elem_rel(grads["fp32"], grads["fp64"]) <= 1e-3


def test_lshape_full_size_cycle_and_mixed_solve():
    """L-shape, ~196k unknowns, 5 levels, anisotropic: one FP64 cycle with
    random parameters matches the oracle; the FP32 solve reaches 1e-8."""
    import torch
    w = C.lshape_aniso()
    h = w.hier
    J = h.nlevels
    flat = C.random_params(J, 3, 3, 3, seed=42, spread=0.15)
    g = C.rng(4, 9, 0)
    u = g.standard_normal((h.sizes[0], 1))
    want = O.lmg(oracle_levels(h), oracle_params(flat, J, 3), 0, w.f, u)
    ctx = ctx_for(h, flat, 3, 1, "fp64")
    ud = to_dev(u, torch.float64)
    ctx.vcycle(to_dev(w.f, torch.float64), ud)
    kappa = np.linalg.cond(h.A[-1].toarray())
    err = elem_rel(to_np(ud), want)
    print(f"lshape fp64 cycle rel {err:.2e} (kappa(A_J) = {kappa:.1e})", flush=True)
    assert err <= max(1e-12, 50 * kappa * np.finfo(float).eps)
    ctx32 = ctx_for(h, C.identity_params(J, 3, 3, 3), 3, 1, "fp32", max_outer=20000)
    f = to_dev(w.f, torch.float64)
    x = torch.zeros_like(f)
    info = ctx32.solve(f, x)
    rr = np.linalg.norm(w.f - h.A[0] @ to_np(x)) / np.linalg.norm(w.f)
    print(f"lshape fp32 solve: {info.iters[0]} cycles, relres {rr:.2e}", flush=True)
    assert info.code == 0 and rr <= 1e-8


def test_diffusion_513_bench_configuration_cycle():
    """The benchmark's configuration (513 x 513, 64 rhs, FP32 cycles with the
    shipped trained parameters, LDS coarse tail): one cycle from zero against
    the FP64 oracle, whole vectors."""
    import torch
    from paper_2608_29082_amd import params as PR
    w = C.diffusion_513(B=64)
    h = w.hier
    J = h.nlevels
    theta, meta = PR.load(PR.default_file("diffusion-513", 3))
    flat = PR.map_levels(theta, meta["J"], J, 3, 3, 3)
    ctx = ctx_for(h, flat, 3, 64, "fp32")
    f = to_dev(w.f, torch.float64)
    e = torch.zeros_like(f)
    ctx.refine_step(f, torch.zeros_like(f), e)          # e = LMG_32(A, f, 0)
    want = O.lmg(oracle_levels(h), oracle_params(flat, J, 3), 0, w.f, np.zeros_like(w.f))
    err = elem_rel(to_np(e), want)
    print(f"513 fp32 bench-config cycle rel {err:.2e}", flush=True)
    assert err <= 2e-5

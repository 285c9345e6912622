"""torch.autograd wrappers of the HIP forward and reverse sweeps (training, paper Sec. 3.1).

Training unrolls refinement steps  u^m = u^{m-1} + LMG(A, f - A u^{m-1}, 0)
(Alg. 3's forward pass in the form the solver uses) and minimises a residual
loss with Rprop (Sec. 3.1).  Each step is one autograd node whose forward
calls mg_refine_step with a per-call checkpoint and whose backward calls
mg_refine_step_backward.  Parameters must not change between a node's forward
and backward (a new training step sets them first).
"""
from __future__ import annotations

import numpy as np
import torch


class RefineStep(torch.autograd.Function):
    """u_out = u + LMG_p(A, f - A u, 0) with gradients for (theta, f, u)."""

    @staticmethod
    def forward(ac, mg, theta, f, u):
        ck = mg.new_ckpt()
        out = mg.refine_step(f.contiguous(), u.contiguous(), ckpt=ck)
        ac.mg, ac.ck = mg, ck
        ac.theta_device = theta.device
        return out

    @staticmethod
    def backward(ac, gout):
        need = ac.needs_input_grad
        gu, gf, gp = ac.mg.refine_step_backward(ac.ck, gout.contiguous(), want_gu=need[3], want_gf=need[2],
                                                 want_gp=need[1])
        ac.ck = None
        if gp is not None:
            gp = gp.to(ac.theta_device)
        return None, gp, gf, gu


class VCycle(torch.autograd.Function):
    """u_out = LMG(A, f, u) in the context's cycle precision (Alg. 2)."""

    @staticmethod
    def forward(ac, mg, theta, f, u):
        ck = mg.new_ckpt()
        out = u.detach().clone().contiguous()
        mg.vcycle(f.contiguous(), out, ckpt=ck)
        ac.mg, ac.ck = mg, ck
        ac.theta_device = theta.device
        return out

    @staticmethod
    def backward(ac, gout):
        need = ac.needs_input_grad
        gu, gf, gp = ac.mg.vcycle_backward(ac.ck, gout.contiguous(), want_gu=need[3], want_gf=need[2],
                                           want_gp=need[1])
        ac.ck = None
        if gp is not None:
            gp = gp.to(ac.theta_device)
        return None, gp, gf, gu


class ResidualLoss(torch.autograd.Function):
    """Alg. 3's residual loss through mg_residual_loss: kind "mean_rel_sq"
    L = mean_b ||f_b - A u_b||^2 / ||f_b||^2 (the training workload's loss) or
    "resid_norm" L = sum_b ||f_b - A u_b||_2.  The loss, both gradients and
    their scaling by the incoming cotangent are computed by the library in
    FP64; this node only passes tensors."""

    @staticmethod
    def forward(ac, mg, f, u, kind="mean_rel_sq"):
        f, u = f.contiguous(), u.contiguous()
        loss, _, _ = mg.residual_loss(f, u, kind=kind)
        ac.mg, ac.kind = mg, kind
        ac.save_for_backward(f, u)
        return loss.reshape(())

    @staticmethod
    def backward(ac, g):
        f, u = ac.saved_tensors
        need = ac.needs_input_grad
        seed = g.detach().to(device=f.device, dtype=torch.float64).reshape(1).contiguous()
        _, gu, gf = ac.mg.residual_loss(f, u, kind=ac.kind, gseed=seed, want_loss=False, want_gu=need[2],
                                        want_gf=need[1])
        return None, gf, gu, None


def unrolled_loss(mg, theta: torch.Tensor, f: torch.Tensor, cycles: int = 10, u0=None,
                  kind: str = "mean_rel_sq") -> torch.Tensor:
    """Loss after `cycles` refinement steps from u0 (zero by default)."""
    mg.set_params(theta.detach().double().cpu().numpy())
    u = torch.zeros_like(f) if u0 is None else u0
    for _ in range(cycles):
        u = RefineStep.apply(mg, theta, f, u)
    return ResidualLoss.apply(mg, f, u, kind)


def train_rprop(mg, theta0, f, cycles: int = 10, steps: int = 100, lr: float = 0.01, tol: float = 1e-6,
                etas=(0.5, 1.2), step_sizes=(1e-6, 50.0), frozen=None, log=None):
    """Rprop on the unrolled residual loss (Sec. 3.1; learning rate 0.01 and at
    most 100 epochs as in Sec. 4).  Stops when L / L^0 <= tol.  `frozen`: a
    boolean mask of parameters kept fixed.  Returns (theta, losses)."""
    theta = torch.tensor(np.asarray(theta0, dtype=np.float64), requires_grad=True)
    opt = torch.optim.Rprop([theta], lr=lr, etas=etas, step_sizes=step_sizes)
    mask = None if frozen is None else torch.tensor(np.asarray(frozen, dtype=bool))
    losses = []
    for it in range(steps):
        opt.zero_grad()
        L = unrolled_loss(mg, theta, f, cycles)
        L.backward()
        if mask is not None:
            theta.grad[mask] = 0.0
        losses.append(L.item())
        if log:
            log(it, losses[-1])
        if losses[-1] <= tol * losses[0]:
            break
        opt.step()
    mg.set_params(theta.detach().numpy())
    return theta.detach().numpy().copy(), losses

"""Train the learnable V-cycle (paper Sec. 3.1) with the HIP forward and reverse sweeps.

    python -m paper_2608_29082_amd.train --workload training-257 --steps 100 --out theta.npy
    python -m paper_2608_29082_amd.train --workload darcy-100 --variant rp --out rp.npy

Block-diffusion workloads (a piecewise constant on 16 x 16 blocks):
  training-257   257 x 257 grid, 7 levels, log10 a ~ U(-2, 2), 32 rhs
  diffusion-513  513 x 513 grid, 8 levels, log10 a ~ U(-3, 3), 32 rhs
  serving-<side> the serving distribution at one grid size
Loss: mean over fields and right-hand sides of ||f - A u^(10)||^2 / ||f||^2
after 10 unrolled refinement steps (cycle precision as chosen, FP64 iterate
and residual), minimised with Rprop from the identity initialisation
(Sec. 3.1; Sec. 3.4; learning rate 0.01, at most 100 epochs, Sec. 4).
--fields N trains on N coefficient fields at once (the right-hand sides are
split between them), seeds --field-seed .. --field-seed + N - 1.  --init starts
Rprop from a saved parameter file.  The result is the parameter set of the
lowest loss seen (--keep-last: the last iterate).  Held-out right-hand sides, on the training fields and
on held-out fields, are then solved to 1e-8 with the trained and with the
identity parameters, and the cycle counts are reported.

Darcy workload (Sec. 4.1): darcy-100 is the cell-centred pressure equation on
100 x 100 cells with the 1e-6 inclusion on [0.4, 0.6]^2, p = 1 / 0 on the
left / right, no flow on top and bottom, f = 0; piecewise constant
interpolation, Galerkin coarse operators, 7 levels, nu = 4, omega = 2/3.  The
right-hand side comes from the boundary data and every column starts from its
own seeded random iterate.  Evaluation: the training field and stand-ins for
the paper's three test fields (two low-conductivity regions at contrast 1e4,
two high-conductivity channels at contrast 1e6, a smooth random field given on
40 x 40 and used on 80 x 80 cells), each solved to 1e-8 from a random start.

--variant selects the trainable parameterisation (params.Variant): full,
shared (one Phi_R and one Phi_P for all levels), rp (LMG-RP: only the shared
Phi_R, Phi_P; damped Jacobi smoother) or rps (LMG-RPS: shared Phi_R, Phi_P
plus Phi_B,l and eta_l; theta_l = omega fixed).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

WORKLOADS = {"training-257": (3, 257, -2.0, 2.0), "diffusion-513": (2, 513, -3.0, 3.0),
             "diffusion-129": (3, 129, -2.0, 2.0)}
# serving distribution (log10 a ~ U(-2, 2)); training fields use seeds from
# 900000 on, disjoint from the request streams' fields
for _side in (65, 129, 257, 513, 1025):
    WORKLOADS[f"serving-{_side}"] = (5, _side, -2.0, 2.0)
DARCY = {"darcy-100": (9, 100, 7)}


def darcy_problems(wid, n, J, B, seed_base):
    """[(name, hierarchy, f (n x B), u0 (n x B))]: training field first, then
    the three test-field stand-ins."""
    from mginputs import configs as C
    from mginputs import darcy as D
    fields = [("train-inclusion", D.inclusion_field(n), J), ("I-two-regions", D.two_regions_field(n), J),
              ("II-channels", D.channels_field(n), J),
              ("III-random-80", D.random_field(C.rng(wid, 1, 0), 40, 80), J)]
    out = []
    for k, (name, kf, Jf) in enumerate(fields):
        h, b = D.darcy_hierarchy(kf, Jf)
        f = np.repeat(b[:, None], B, axis=1)
        u0 = C.rng(wid, 2, seed_base + k).standard_normal((h.sizes[0], B))
        out.append((name, h, f, u0))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="training-257", choices=sorted(WORKLOADS) + sorted(DARCY))
    ap.add_argument("--variant", default="full", choices=["full", "shared", "rp", "rps"])
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--cycles", type=int, default=10)
    ap.add_argument("--lr", type=float, default=0.01)
    ap.add_argument("--K", type=int, default=3)
    ap.add_argument("--B", type=int, default=32)
    ap.add_argument("--fields", type=int, default=1)
    ap.add_argument("--field-seed", type=int, default=0, help="seed of the first training field")
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--init", default=None, help="start from this parameter file (.npy) instead of the identity")
    ap.add_argument("--keep-last", action="store_true",
                    help="keep the last Rprop iterate instead of the parameters of the lowest loss seen")
    ap.add_argument("--out", default=None)
    ap.add_argument("--eval-B", type=int, default=8)
    ap.add_argument("--eval-fields", type=int, default=2)
    args = ap.parse_args(argv)

    import torch
    from mginputs import configs as C
    from mginputs import hierarchy as H
    from paper_2608_29082_amd import autograd as AG
    from paper_2608_29082_amd import binding as Bd
    from paper_2608_29082_amd import params as PR

    K = args.K
    darcy = args.workload in DARCY
    nu = 4 if darcy else 2
    if darcy:
        wid, n_cells, J = DARCY[args.workload]
        Bt = max(1, args.B)
        probs = darcy_problems(wid, n_cells, J, Bt, 100)
        hiers = [probs[0][1]]
        fs_np, u0s_np = [probs[0][2]], [probs[0][3]]
        Bf = Bt
    else:
        wid, side, lo, hi = WORKLOADS[args.workload]
        hiers = []
        for k in range(args.fields):
            fseed = args.field_seed + k + (900000 if args.workload.startswith("serving") else 0)
            blocks = H.block_field(C.rng(wid, 1, fseed), 16, lo, hi)
            hiers.append(H.square_hierarchy(side, blocks))
        J = hiers[0].nlevels
        Bf = max(1, args.B // args.fields)
        n0 = hiers[0].sizes[0]
        # training right-hand sides: seeds disjoint from the benchmark's (index 0)
        fs_np = [C.rng(wid, 2, 5000 + k).standard_normal((n0, Bf)) for k in range(args.fields)]
        u0s_np = [None] * args.fields
    var = PR.Variant(args.variant, J, K, K, K)
    theta0 = PR.identity(J, K, K, K)
    ctxs = [Bd.Context(h.A, h.P, theta0, K, K, K, nu_pre=nu, nu_post=nu, precision=args.precision, nrhs=Bf,
                       backward=True) for h in hiers]
    dev = lambda a: None if a is None else torch.tensor(a, dtype=torch.float64, device="cuda")
    fs = [dev(a) for a in fs_np]
    u0s = [dev(a) for a in u0s_np]

    start = None
    if args.init:
        start, _ = PR.load(args.init)
        if start.size != theta0.size:
            raise SystemExit(f"{args.init}: {start.size} parameters, expected {theta0.size}")
    phi = torch.tensor(var.initial(start), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Rprop([phi], lr=args.lr, etas=(0.5, 1.2), step_sizes=(1e-6, 50.0))
    losses = []
    best_loss, best_phi, best_step = float("inf"), None, -1
    t0 = time.time()
    for it in range(args.steps):
        opt.zero_grad()
        theta = var.expand(phi)
        L = sum(AG.unrolled_loss(c, theta, f, args.cycles, u0=u0) for c, f, u0 in zip(ctxs, fs, u0s)) / len(ctxs)
        L.backward()
        losses.append(L.item())
        # the parameters of the lowest loss seen are the result (a Rprop run can leave a good
        # region late in training; the loss of an unrolled divergent cycle grows without bound)
        if np.isfinite(losses[-1]) and losses[-1] < best_loss:
            best_loss, best_phi, best_step = losses[-1], phi.detach().clone(), it
        if it % 10 == 0:
            print(f"# step {it} loss {losses[-1]:.4e} ({time.time() - t0:.1f}s)", file=sys.stderr, flush=True)
        if losses[-1] <= 1e-6 * losses[0]:
            break
        opt.step()
    train_s = time.time() - t0
    final_phi = best_phi if (best_phi is not None and not args.keep_last) else phi.detach()
    theta_np = var.expand(final_phi.numpy().copy())
    for c in ctxs:
        c.close()

    def cycles(h, params, f_np, u0_np=None):
        c = Bd.Context(h.A, h.P, params, K, K, K, nu_pre=nu, nu_post=nu, precision=args.precision,
                       nrhs=f_np.shape[1], max_outer=8000, check_every=10)
        fd = torch.tensor(f_np, dtype=torch.float64, device="cuda")
        u = torch.zeros_like(fd) if u0_np is None else torch.tensor(u0_np, dtype=torch.float64, device="cuda")
        info = c.solve(fd, u)
        c.close()
        return {"mean": float(info.iters.mean()), "max": int(info.iters.max()), "code": int(info.code)}

    evals = []
    if darcy:
        for name, h, f_np, u0_np in probs:
            evals.append({"field": name, "identity": cycles(h, theta0, f_np[:, :args.eval_B], u0_np[:, :args.eval_B]),
                          "trained": cycles(h, theta_np, f_np[:, :args.eval_B], u0_np[:, :args.eval_B])})
            print(f"# eval {evals[-1]}", file=sys.stderr, flush=True)
    else:
        eval_fields = [("train", hiers[0])]
        for k in range(args.eval_fields):
            blocks = H.block_field(C.rng(wid, 1, 950000 + k), 16, lo, hi)
            eval_fields.append((f"heldout{k}", H.square_hierarchy(side, blocks)))
        f_eval = C.rng(wid, 2, 7000).standard_normal((hiers[0].sizes[0], args.eval_B))
        for name, h in eval_fields:
            evals.append({"field": name, "identity": cycles(h, theta0, f_eval), "trained": cycles(h, theta_np, f_eval)})
            print(f"# eval {evals[-1]}", file=sys.stderr, flush=True)
    out = {"workload": args.workload, "variant": args.variant, "K": K, "fields": args.fields, "steps": len(losses),
           "loss0": losses[0], "loss_final": losses[-1], "loss_best": best_loss, "best_step": best_step,
           "train_seconds": train_s, "eval": evals}
    if args.out:
        if darcy:
            desc = (f"Darcy cell-centred, {n_cells}x{n_cells} cells, 1e-6 inclusion on [0.4,0.6]^2, piecewise "
                    f"constant interpolation, {Bf} random starts, {args.cycles} unrolled V({nu},{nu}) steps, "
                    f"variant {args.variant}")
        else:
            desc = (f"block diffusion {side}x{side}, log10 a ~ U({lo:g},{hi:g}) on 16x16 blocks, "
                    f"{args.fields} field(s) from seed {args.field_seed}, {Bf} rhs ~ N(0,1) per field, "
                    f"{args.cycles} unrolled V(2,2) refinement steps, variant {args.variant}")
        PR.save(args.out, theta_np, {
            "trained_on": desc, "J": J, "KB": K, "KR": K, "KP": K, "nu": [nu, nu], "precision": args.precision,
            "variant": args.variant, "optimizer": f"Rprop lr={args.lr}", "steps": len(losses),
            "init": os.path.basename(args.init) if args.init else "identity",
            "loss0": losses[0], "loss_final": losses[-1], "loss_best": best_loss, "best_step": best_step,
            "kept": "last" if args.keep_last else "lowest loss", "eval": evals})
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

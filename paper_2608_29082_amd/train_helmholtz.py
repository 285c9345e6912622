"""Train the two-feature Helmholtz cycle (paper Sec. 4.2) through the HIP forward path.

    python -m paper_2608_29082_amd.train_helmholtz --steps 60 --out hz.npy

Loss (Alg. 3's): mean over right-hand sides of ||f - A u^(m)||^2 / ||f||^2
after m cycles u <- LMG(A, f, u) from u = 0 (FP64 cycles, the library's
FP64 residual), minimised with Rprop from the identity initialisation.  The
paper back-propagates through the cycle; a GMRES smoothing step has no
reverse sweep in this library, so the gradient of the same loss is formed by
central differences of the forward cycle, one pair of evaluations per
parameter (relative step 1e-6).  Every evaluation runs on the GPU; only the
Rprop update of the few dozen parameters runs on the host.

Training right-hand sides are smoothed disks at seeded random centres
(one or two disks each, seeds disjoint from the benchmark's); the evaluation
solves the benchmark's 16 sources (the paper's training and test sources and
14 random ones) by FGMRES(40) with the cycle and with FMG as preconditioner,
FP32 cycles, with the identity and with the trained parameters.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--side", type=int, default=257)
    ap.add_argument("--k", type=float, default=16.0 * np.pi)
    ap.add_argument("--levels", type=int, default=5)
    ap.add_argument("--K", type=int, default=1)
    ap.add_argument("--B", type=int, default=8, help="training right-hand sides")
    ap.add_argument("--cycles", type=int, default=10, help="cycles m of the loss")
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--lr", type=float, default=0.01)
    ap.add_argument("--fd-step", type=float, default=1e-6, help="relative central-difference step")
    ap.add_argument("--init", default=None, help="start from this parameter file (.npy)")
    ap.add_argument("--out", default=None)
    ap.add_argument("--eval-B", type=int, default=16)
    ap.add_argument("--eval-only", default=None,
                    help="evaluate this parameter file (trained on any hierarchy of the same problem family, moved "
                         "over by the partial transfer rule) on --side/--k/--levels and exit")
    ap.add_argument("--src-side", type=int, default=None, help="--eval-only: side of the source hierarchy")
    ap.add_argument("--src-k", type=float, default=None, help="--eval-only: wave number of the source problem")
    ap.add_argument("--src-levels", type=int, default=None, help="--eval-only: levels of the source hierarchy")
    return ap.parse_args(argv)


def transfer(theta, plan_src, plan_dst, K: int) -> np.ndarray:
    """Partial weight transfer to another hierarchy (Sec. 4.2, the transfer
    rule): a target level whose smoother kind matches the source level of the
    same index takes its weights; a target level beyond the source's takes the
    deepest source level of its kind; a level without a match keeps the
    classical (identity) weights of its kind; the shared Phi_R and Phi_P are
    always copied.  plan_*: per level (kind, nu_pre, nu_post)."""
    from mginputs import configs as C
    per = 2 + 4 * (K + 1)
    Js, Jd = len(plan_src) + 1, len(plan_dst) + 1
    src = np.asarray(theta, dtype=np.float64)
    assert src.size == C.hz_n_params(Js, K, K, K)
    out = C.hz_identity_params(Jd, K, K, K, plan_dst)
    lv_s = src[:(Js - 1) * per].reshape(Js - 1, per)
    lv_d = out[:(Jd - 1) * per].reshape(Jd - 1, per)
    for l in range(Jd - 1):
        kind = plan_dst[l][0]
        if l < Js - 1:
            if plan_src[l][0] == kind:
                lv_d[l] = lv_s[l]
        else:
            for m in range(Js - 2, -1, -1):
                if plan_src[m][0] == kind:
                    lv_d[l] = lv_s[m]
                    break
    out[(Jd - 1) * per:] = src[(Js - 1) * per:]
    return out


class Loss:
    """L(theta) on the GPU: m FP64 cycles from zero on the training sources."""

    def __init__(self, w, f, cycles):
        import torch
        from paper_2608_29082_amd import helmholtz as HB
        self.torch = torch
        self.ctx = HB.HelmholtzContext(w.hier.A, w.hier.P, w.params, w.KB, w.KR, w.KP, w.plan, v=w.v,
                                       precision="fp64", nrhs=f.shape[1])
        self.f = torch.tensor(f, dtype=torch.complex128, device="cuda")
        self.u = torch.zeros_like(self.f)
        self.fn2 = np.linalg.norm(f, axis=0) ** 2
        self.cycles = cycles
        self.evals = 0

    def __call__(self, theta) -> float:
        self.ctx.set_params(theta)
        self.u.zero_()
        for _ in range(self.cycles):
            self.ctx.vcycle(self.f, self.u)
        _, norms = self.ctx.residual(self.f, self.u, want_r=False)
        self.evals += 1
        return float(np.mean(norms.cpu().numpy() ** 2 / self.fn2))

    def grad(self, theta, rel):
        g = np.zeros_like(theta)
        for i in range(theta.size):
            h = rel * max(1.0, abs(theta[i]))
            tp, tm = theta.copy(), theta.copy()
            tp[i] += h
            tm[i] -= h
            g[i] = (self(tp) - self(tm)) / (2.0 * h)
        return g


def stationary(w, theta, B, max_cycles=400, rtol=1e-8):
    """Cycles of u <- LMG(A, f, u) (FP64 cycles) until every column's relative
    residual meets rtol (None: not within max_cycles), checked after every cycle."""
    import torch
    from paper_2608_29082_amd import helmholtz as HB
    ctx = HB.from_workload(w, precision="fp64", params=theta)
    f = torch.tensor(w.f[:, :B], dtype=torch.complex128, device="cuda")
    fn = np.linalg.norm(w.f[:, :B], axis=0)
    u = torch.zeros_like(f)
    done = None
    for c in range(1, max_cycles + 1):
        ctx.vcycle(f, u)
        _, norms = ctx.residual(f, u, want_r=False)
        rel = norms.cpu().numpy() / fn
        if not np.all(np.isfinite(rel)) or rel.max() > 1e12:
            break
        if rel.max() <= rtol:
            done = c
            break
    ctx.close()
    return done


def evaluate(w, theta, B):
    """FGMRES(40) iterations and seconds with FP32 cycles, V-cycle and FMG
    preconditioners; cycles of the stationary iteration with FP64 cycles."""
    import torch
    from paper_2608_29082_amd import helmholtz as HB
    ctx = HB.from_workload(w, precision="fp32", params=theta)
    f = torch.tensor(w.f[:, :B], dtype=torch.complex128, device="cuda")
    out = {"stationary_cycles": stationary(w, theta, B)}
    for pc in ("vcycle", "fmg"):
        x = torch.zeros_like(f)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = ctx.fgmres(f, x, restart=40, max_iter=200, rtol=1e-8, precond=pc)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[pc] = {"iters_max": int(info.iters.max()), "iters_mean": float(info.iters.mean()),
                   "converged": bool(info.code == 0), "seconds": dt}
    ctx.close()
    return out


def main(argv=None):
    args = parse(argv)
    import torch
    from mginputs import configs as C
    from mginputs import helmholtz as HZ

    w = C.helmholtz(args.side, args.k, args.levels, B=args.eval_B, K=args.K)
    J = w.hier.nlevels
    if args.eval_only:
        src_plan = HZ.smoother_plan(HZ.hierarchy(args.src_side or args.side, args.src_k or args.k,
                                                 args.src_levels or args.levels))
        theta = transfer(np.load(args.eval_only), src_plan, w.plan, args.K)
        ev = {"identity": evaluate(w, C.hz_identity_params(J, args.K, args.K, args.K, w.plan), args.eval_B),
              "transferred": evaluate(w, theta, args.eval_B)}
        print(json.dumps({"params": os.path.basename(args.eval_only), "target": f"helmholtz-{args.side}",
                          "k": args.k, "levels": J, "eval": ev}))
        return
    # training sources: random disks only (columns 0 and 1 of every source set are the paper's two
    # fixed sources), seeds disjoint from the benchmark's
    cents = HZ.source_centres(args.B + 2, C.rng(10, 2, 1))[2:]
    f_train = HZ.load_vectors(args.side, cents)
    theta0 = C.hz_identity_params(J, args.K, args.K, args.K, w.plan)
    start = theta0
    if args.init:
        start = np.load(args.init)
        if start.size != theta0.size:
            raise SystemExit(f"{args.init}: {start.size} parameters, expected {theta0.size}")
    loss = Loss(w, f_train, args.cycles)
    phi = torch.tensor(start, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Rprop([phi], lr=args.lr, etas=(0.5, 1.2), step_sizes=(1e-6, 50.0))
    L0 = loss(start)
    hist = [L0]
    best, best_L = start.copy(), L0
    t0 = time.time()
    print(f"# step 0 loss {L0:.4e}", file=sys.stderr, flush=True)
    for it in range(args.steps):
        th = phi.detach().numpy().copy()
        g = loss.grad(th, args.fd_step)
        opt.zero_grad()
        phi.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        L = loss(phi.detach().numpy().copy())
        hist.append(L)
        if L < best_L:
            best, best_L = phi.detach().numpy().copy(), L
        print(f"# step {it + 1} loss {L:.4e} ({time.time() - t0:.1f}s, {loss.evals} evaluations)",
              file=sys.stderr, flush=True)
    train_s = time.time() - t0
    ev = {"identity": evaluate(w, theta0, args.eval_B), "trained": evaluate(w, best, args.eval_B)}
    print(f"# eval {json.dumps(ev)}", file=sys.stderr, flush=True)
    meta = {"workload": f"helmholtz-{args.side}", "k": args.k, "levels": J, "K": args.K,
            "smoothers": [list(p) for p in w.plan], "gmres_steps": w.v,
            "trained_on": f"{args.B} random smoothed-disk sources (seed 1), loss after {args.cycles} FP64 cycles",
            "optimizer": f"Rprop lr={args.lr}, gradient by central differences (relative step {args.fd_step})",
            "steps": args.steps, "loss0": L0, "loss_best": best_L, "loss_history": hist,
            "train_seconds": train_s, "loss_evaluations": loss.evals, "eval": ev,
            "init": os.path.basename(args.init) if args.init else "identity"}
    if args.out:
        np.save(args.out, best)
        with open(os.path.splitext(args.out)[0] + ".json", "w") as fh:
            json.dump(meta, fh, indent=1)
    print(json.dumps(meta))


if __name__ == "__main__":
    main()

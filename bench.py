"""Benchmark: solves/s at 1e-8 relative residual on one MI355X.

Workload (default): variable-coefficient diffusion on a 513 x 513 grid
(261 121 unknowns, 8 levels), a piecewise constant on 16 x 16 blocks with
log10 a ~ U(-3, 3), 64 right-hand sides ~ N(0, 1), learnable V(2,2) cycles
with K = 3 convolutions in FP32 inside FP64 iterative refinement, to a
relative residual of 1e-8 per column.  One step = one batched solve of the
64 right-hand sides from u = 0, inputs resident in HBM.

Also reported: the plain FP64 GPU V-cycle (classical components, K = 0) on the
same hierarchy and right-hand sides, the roofline of the dominant kernel
family (HIP events around each of its launches in the timed region), the
per-family time of the finest level's kernels, the same solve with the
graph convolutions as chains of per-hop sweeps instead of the fused LDS-tile
kernel, flexible
GMRES with the learned and the classical cycle (or FMG) as preconditioner on
the same inputs, the request loop, and the CPU FP64 oracle timed on a bounded
sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="diffusion-513", choices=["diffusion-513", "poisson-33", "training-257"])
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16", "fp64"])
    ap.add_argument("--K", type=int, default=3)
    ap.add_argument("--params", default="default",
                    help="'default' (parameters trained on this workload's operator, shipped with the package), "
                         "'identity', or a .npy parameter file")
    ap.add_argument("--roofline-family", default="conv",
                    help="kernel family of the roofline entry (conv: the fused LDS-tile convolution)")
    ap.add_argument("--roofline-level", type=int, default=0)
    ap.add_argument("--max-outer", type=int, default=20000)
    ap.add_argument("--check-every", type=int, default=5,
                    help="mg_solve reads the active-column count on the host every this many cycles (every solve "
                         "in the run; a solve ends at the first check after its last column converged)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-krylov", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="skip the convolution-variant and Darcy sections")
    ap.add_argument("--no-tiles", action="store_true",
                    help="run the convolutions as chains of per-hop sweeps (no fused LDS-tile kernel)")
    ap.add_argument("--no-ablation", action="store_true",
                    help="skip the per-family finest-level timing and the per-hop-sweep comparison")
    ap.add_argument("--restart", type=int, default=30, help="FGMRES restart length of the Krylov comparison")
    ap.add_argument("--no-helmholtz", action="store_true", help="skip the complex Helmholtz section")
    ap.add_argument("--helmholtz-only", action="store_true",
                    help="run only the complex Helmholtz section (no CPU leg) and print its JSON")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--cpu-worker", type=int, default=-1, help=argparse.SUPPRESS)
    ap.add_argument("--serving-requests", type=int, default=60,
                    help="requests per run of the per-request serving loop (closed loop, 0.5x its rate, FGMRES); "
                         "0 skips")
    ap.add_argument("--batched-requests", type=int, default=10000,
                    help="requests of the continuous-batching loop's closed-loop run (its rate T sets the "
                         "open-loop arrival rates); 0 skips")
    ap.add_argument("--open-requests", type=int, default=1000,
                    help="requests of each open-loop run of the batched loop (0.5 T, 0.8 T, 1.2 T)")
    ap.add_argument("--batch-capacity", type=int, default=32, help="column slots per batch of the batched loop")
    ap.add_argument("--serving-compare", type=int, default=100,
                    help="requests of the learned-vs-plain-FP64 batched comparison (0: skip)")
    ap.add_argument("--cycles-per-round", type=int, default=8, help="refinement cycles per round of the batched loop")
    return ap.parse_args()


def workload(name, K):
    from mginputs import configs as C
    if name == "diffusion-513":
        return C.diffusion_513(K=K), "log10 a ~ U(-3,3) on 16x16 blocks"
    if name == "training-257":
        return C.training_257(K=K), "log10 a ~ U(-2,2) on 16x16 blocks"
    w = C.poisson_unit(K=K, B=64)
    return w, "a = 1"


def main():
    args = parse()
    if args.cpu_worker >= 0:
        cpu_worker(args.cpu_worker, args.cpu_seconds, args.K)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU; --gpus above 1 is not supported"}))
        sys.exit(2)
    import torch
    from mginputs import configs as C
    from paper_2608_29082_amd import binding as Bd

    if args.helmholtz_only:
        print(json.dumps({"helmholtz": helmholtz(args)}), flush=True)
        return
    t0 = time.time()
    w, coef = workload(args.workload, args.K)
    h = w.hier
    J = h.nlevels
    B = w.B
    from paper_2608_29082_amd import params as PR
    pfile = args.params
    if pfile == "default":
        pfile = PR.default_file(args.workload, args.K)
    if pfile and pfile != "identity":
        theta, meta = PR.load(pfile)
        params = PR.map_levels(theta, meta["J"], J, args.K, args.K, args.K)
        param_desc = f"{os.path.basename(pfile)}: {meta.get('trained_on', '')}"
    else:
        params = PR.identity(J, args.K, args.K, args.K)
        param_desc = "identity initialisation (classical components)"
    print(f"# hierarchy {h.sizes} built in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    ctx = Bd.Context(h.A, h.P, params, args.K, args.K, args.K, precision=args.precision, nrhs=B,
                     max_outer=args.max_outer, check_every=args.check_every, stream=stream, tiles=not args.no_tiles)
    f = torch.tensor(w.f, dtype=torch.float64, device=dev)
    u = torch.zeros_like(f)

    def step():
        u.zero_()
        return ctx.solve(f, u)

    for _ in range(args.warmup):
        info = step()
        print(f"# warmup: iters {int(info.iters.min())}..{int(info.iters.max())}, code {info.code}",
              file=sys.stderr, flush=True)
    ctx.timing_start(None if args.roofline_family == "none" else args.roofline_family, args.roofline_level)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    infos = []
    for _ in range(args.steps):
        infos.append(step())
        print(f"# step done: iters {int(infos[-1].iters.max())}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    launches, kms, kbytes = ctx.timing_read()
    ctx.timing_start(None)
    elapsed = t2 - t1
    info = infos[-1]
    u_host = u.cpu().numpy()
    relres_host = np.linalg.norm(w.f - h.A[0] @ u_host, axis=0) / np.linalg.norm(w.f, axis=0)
    solves = B * args.steps
    # the library stops each column on its own FP64 residual; the host
    # recomputation differs from it by cancellation (about eps ||A|| ||u|| / ||f||
    # relative to ||f||), so the cross-check allows a relative 1e-3 on 1e-8
    converged_all = all(i.code == 0 for i in infos) and float(relres_host.max()) <= 1e-8 * (1 + 1e-3)
    # a throughput only counts when every column reached the tolerance
    value = solves / elapsed if converged_all else 0.0
    avg_ms = kms / max(launches, 1)
    achieved = kbytes / (kms * 1e-3) / 1e9 if kms > 0 else 0.0
    copy_gbps = device_copy_gbps()

    out = {
        "metric": "solves/sec at 1e-8 rel. residual vs plain GMG; HBM GB/s; p50/p99 solve latency",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision != "fp64" else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {h.sizes[0]} unknowns, {J} levels, {coef}, {B} rhs ~ N(0,1)",
            "nrhs": B, "levels": J, "unknowns": h.sizes[0], "K": args.K, "nu": [2, 2],
            "cycle_precision": args.precision, "refinement": "fp64", "rtol": 1e-8,
            "params": param_desc,
        },
        "iters": {"min": int(info.iters.min()), "max": int(info.iters.max()), "mean": float(info.iters.mean())},
        "relres_max_fp64_host": float(relres_host.max()),
        "converged": bool(converged_all),
        "roofline": {
            "bound": "hbm", "kernel_family": args.roofline_family, "level": args.roofline_level,
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "copy_GBps": copy_gbps, "frac_of_copy": achieved / copy_gbps if copy_gbps else None,
            "traffic": counter_traffic(args.roofline_family, args.roofline_level),
            "launches": launches, "avg_launch_us": 1e3 * avg_ms,
            "alg_bytes_per_launch": kbytes / max(launches, 1),
        },
    }

    if not args.no_ablation:
        out["level0_kernels"] = level0_kernels(ctx, f)
    if not args.no_ablation and not args.no_tiles and args.precision != "fp64":
        # the same solve with every convolution as a chain of per-hop sweeps
        hctx = Bd.Context(h.A, h.P, params, args.K, args.K, args.K, precision=args.precision, nrhs=B,
                          max_outer=args.max_outer, check_every=args.check_every, stream=stream, tiles=False)
        uh = torch.zeros_like(f)
        hctx.solve(f, uh)
        uh.zero_()
        torch.cuda.synchronize()
        ta = time.perf_counter()
        hinfo = hctx.solve(f, uh)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        out["per_hop_sweeps"] = {"value": B / (tb - ta), "unit": "solves/s", "iters_max": int(hinfo.iters.max()),
                                 "converged": bool(hinfo.code == 0),
                                 "level0_kernels": level0_kernels(hctx, f)}
        hctx.close()
        print(f"# per-hop sweeps: {out['per_hop_sweeps']['value']:.1f} solves/s", file=sys.stderr, flush=True)

    if not args.no_plain:
        # plain FP64 GPU V-cycle: classical components (K = 0, identity), same inputs
        pctx = Bd.Context(h.A, h.P, C.identity_params(J, 0, 0, 0), 0, 0, 0, precision="fp64", nrhs=B,
                          max_outer=args.max_outer, check_every=args.check_every, stream=stream)
        up = torch.zeros_like(f)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        pinfo = pctx.solve(f, up)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        out["plain_fp64_gmg"] = {"value": B / (tb - ta), "unit": "solves/s", "ms_per_solve_batch": 1e3 * (tb - ta),
                                 "iters_max": int(pinfo.iters.max()), "converged": bool(pinfo.code == 0)}
        out["speedup_vs_plain_fp64_gmg"] = value / out["plain_fp64_gmg"]["value"]
        out["learned_fp64"] = learned_fp64(args, h, params, f, B, stream)
        out["learned_unbatched"] = unbatched(args, h, params, f, stream)
        if not args.no_krylov:
            out["krylov"] = krylov(args, {"learned_" + args.precision: ctx, "classical_fp64": pctx}, f, w, h, B)
        pctx.close()
    elif not args.no_krylov:
        out["krylov"] = krylov(args, {"learned_" + args.precision: ctx}, f, w, h, B)

    if not args.no_ablation and args.workload == "diffusion-513":
        out["cycle_cost"] = cycle_cost(args, h, params, f, B, stream)
        seeds = (tuple(s for s in meta.get("held_out_seeds", (10, 11, 12, 13, 14)) if s != 0)
                 if pfile and pfile != "identity" else ())
        if seeds:
            out["held_out_fields"] = held_out(args, params, stream, seeds)

    if not args.no_variants:
        out["conv_variants"] = conv_variants(args, h, f, B, stream)
        out["darcy"] = darcy(args)

    if args.serving_requests > 0 or args.batched_requests > 0:
        out["serving"] = serving(args)

    if not args.no_helmholtz:
        out["helmholtz"] = helmholtz(args)

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, params, args, float(info.iters.mean()))
        if "helmholtz" in out:
            out["helmholtz"]["cpu_baseline"] = cpu_baseline_helmholtz()
    ctx.close()
    print(json.dumps(out), flush=True)


def krylov(args, ctxs, f, w, h, B):
    """Flexible GMRES(restart) to 1e-8 with the cycle (or FMG) as right
    preconditioner (the paper's Sec. 4.2 usage), same inputs as the main
    solve: solves/s, iterations (preconditioner calls) and the host FP64
    residual.  One untimed call first (it allocates the Krylov basis)."""
    import torch
    from paper_2608_29082_amd import binding as Bd
    out = {"restart": args.restart, "rtol": 1e-8, "reorth": Bd.REORTH_DEFAULT}
    for name, c in ctxs.items():
        for pc in ("vcycle", "fmg"):
            x = torch.zeros_like(f)
            c.fgmres(f, x, restart=args.restart, max_iter=2, rtol=1e-8, precond=pc)
            x.zero_()
            c.timing_start("krylov", 0)
            torch.cuda.synchronize()
            ta = time.perf_counter()
            info = c.fgmres(f, x, restart=args.restart, max_iter=2000, rtol=1e-8, precond=pc)
            torch.cuda.synchronize()
            tb = time.perf_counter()
            kl, kms, kby = c.timing_read()
            c.timing_start(None)
            rr = np.linalg.norm(w.f - h.A[0] @ x.cpu().numpy(), axis=0) / np.linalg.norm(w.f, axis=0)
            # the library stops on its own FP64 residual; the host recomputation of a
            # residual 1e8 times smaller than f differs from it by cancellation (about
            # eps ||A|| ||u|| / ||f||), so the cross-check allows a relative 1e-3
            ok = info.code == 0 and float(rr.max()) <= 1e-8 * (1 + 1e-3)
            out[f"{name}_{pc}"] = {"value": B / (tb - ta) if ok else 0.0, "unit": "solves/s",
                                   "ms_per_solve_batch": 1e3 * (tb - ta), "iters_max": int(info.iters.max()),
                                   "iters_mean": float(info.iters.mean()), "relres_max_fp64_host": float(rr.max()),
                                   "converged": bool(ok),
                                   "gram_schmidt_ms": kms, "gram_schmidt_GBps": kby / (kms * 1e-3) / 1e9 if kms else 0.0}
            print(f"# fgmres {name} {pc}: {out[f'{name}_{pc}']}", file=sys.stderr, flush=True)
    return out


def conv_variants(args, h, f, B, stream):
    """Per-cycle cost of the convolution variants on the same hierarchy and
    right-hand sides (identity parameters, so every variant runs the same
    number of hops): ms per refinement step and the finest-level fused
    convolution's time and achieved bandwidth (algorithmic bytes over
    HIP-event time)."""
    import torch
    from paper_2608_29082_amd import binding as Bd
    from paper_2608_29082_amd import params as PR
    J = h.nlevels
    out = {}
    for agg, basis in (("mean", "monomial"), ("weighted", "monomial"), ("sym", "chebyshev")):
        ctx = Bd.Context(h.A, h.P, PR.identity(J, args.K, args.K, args.K), args.K, args.K, args.K,
                         precision=args.precision, nrhs=B, stream=stream, basis=basis, aggregation=agg)
        u = torch.zeros_like(f)
        ctx.refine_step(f, u, u)
        ctx.timing_start("conv", 0)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for _ in range(10):
            ctx.refine_step(f, u, u)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        n, ms, by = ctx.timing_read()
        ctx.timing_start(None)
        ctx.close()
        out[f"{agg}_{basis}"] = {"ms_per_cycle": 1e2 * (tb - ta),
                                 "conv_level0_GBps": by / (ms * 1e-3) / 1e9 if ms > 0 else None,
                                 "conv_level0_us": 1e3 * ms / n if n else None}
        print(f"# variant {agg}/{basis}: {out[f'{agg}_{basis}']}", file=sys.stderr, flush=True)
    return out


def darcy(args):
    """Darcy pressure equation of Sec. 4.1 (100 x 100 cells, 1e-6 inclusion,
    piecewise constant interpolation, 7 levels, V(4,4), 8 seeded random
    starts, FP32 cycles in FP64 refinement to 1e-8): the classical cycle and
    the shipped LMG-RP / LMG-RPS parameters."""
    import torch
    from mginputs import configs as C
    from paper_2608_29082_amd import binding as Bd
    from paper_2608_29082_amd import params as PR
    w, u0 = C.darcy_inclusion(B=8)
    h = w.hier
    J = h.nlevels
    f = torch.tensor(w.f, dtype=torch.float64, device="cuda")
    out = {"workload": "darcy-100: 10000 cells, 7 levels, 1e-6 inclusion, 8 random starts"}
    sets = {"classical": PR.identity(J, 3, 3, 3)}
    for v in ("rp", "rps"):
        pf = PR.default_file(f"darcy-100-{v}", 3)
        if pf:
            sets[f"lmg_{v}"] = PR.load(pf)[0]
    for name, theta in sets.items():
        ctx = Bd.Context(h.A, h.P, theta, 3, 3, 3, nu_pre=4, nu_post=4, precision="fp32", nrhs=8, max_outer=5000)
        u = torch.tensor(u0, dtype=torch.float64, device="cuda")
        ctx.solve(f, u)
        u.copy_(torch.tensor(u0, dtype=torch.float64, device="cuda"))
        torch.cuda.synchronize()
        ta = time.perf_counter()
        info = ctx.solve(f, u)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        rr = np.linalg.norm(w.f - h.A[0] @ u.cpu().numpy(), axis=0) / np.linalg.norm(w.f, axis=0)
        ok = info.code == 0 and float(rr.max()) <= 1e-8 * (1 + 1e-3)
        out[name] = {"solves_per_s": 8 / (tb - ta) if ok else 0.0, "cycles_max": int(info.iters.max()),
                     "ms": 1e3 * (tb - ta), "relres_max_fp64_host": float(rr.max()), "converged": bool(ok)}
        ctx.close()
        print(f"# darcy {name}: {out[name]}", file=sys.stderr, flush=True)
    return out


TRAFFIC_FILES = {("conv", 0): "k_conv_tile_level0_diffusion513_traffic.json",
                 ("hop", 0): "k_hop_level0_diffusion513_traffic.json"}


def kernel_sources_sha256():
    """SHA-256 over the kernel and tiling sources (kernels.hpp, tiles.hpp)."""
    import hashlib
    hsh = hashlib.sha256()
    for name in ("kernels.hpp", "tiles.hpp"):
        with open(os.path.join(ROOT, "paper_2608_29082_amd", "csrc", name), "rb") as fh:
            hsh.update(fh.read())
    return hsh.hexdigest()


def counter_traffic(kernel_family, level):
    """Calibrated HBM bytes per dispatch of the timed kernel from the committed
    PMC measurement, or None if the kernel sources changed since it was taken."""
    name = TRAFFIC_FILES.get((kernel_family, level))
    path = os.path.join(ROOT, "profiles", name) if name else None
    if not path or not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    return rec["bytes_per_dispatch"] if rec.get("kernel_sources_sha256") == kernel_sources_sha256() else None


def level0_kernels(ctx, f, steps=3):
    """Per kernel family on the finest level: launches per refinement step,
    microseconds per launch and achieved algorithmic GB/s (HIP events), over
    `steps` refinement steps from zero."""
    import torch
    out = {}
    u = torch.zeros_like(f)
    for fam in ("conv", "hop", "resid", "restrict", "prolong", "outer"):
        ctx.timing_start(fam, 0)
        u.zero_()
        for _ in range(steps):
            ctx.refine_step(f, u, u)
        n, ms, by = ctx.timing_read()
        if n:
            out[fam] = {"launches_per_step": n // steps, "us": 1e3 * ms / n, "GBps": by / (ms * 1e-3) / 1e9}
    ctx.timing_start(None)
    return out


def serving(args):
    """Request loops over the serving stream (sides uniform over 65..1025, log10 a
    ~ U(-2, 2) on 16 x 16 blocks per request, f ~ N(0, 1), per-size trained FP32
    parameters, FP64 refinement to 1e-8).  Latency = done - arrival, setup
    (the request's hierarchy) included.
      * batched: continuous batching (serve.BatchServer, per-column operators,
        capacity columns per grid, slots refilled between rounds): closed loop
        over --batched-requests requests for the saturated rate T, then Poisson
        arrivals at 0.5 T, 0.8 T and 1.2 T (overload) over --open-requests; then the first --serving-compare requests
        of the stream batched with the learned FP32 cycle and with the plain
        FP64 classical V-cycle (closed loops, same accuracy);
      * per_request: one context per request (serve.Server, B = 1) on
        --serving-requests requests, closed loop and 0.5 T, and flexible
        GMRES(30) around the learned cycle (closed loop)."""
    from paper_2608_29082_amd import params as PR
    from paper_2608_29082_amd import serve as S
    theta = {}
    for side in (65, 129, 257, 513, 1025):
        f = PR.default_file(f"serving-{side}", 3)
        if f:
            th, meta = PR.load(f)
            theta[side] = (th, meta["J"])
    out = {"sides": [65, 129, 257, 513, 1025]}
    budget = 96 << 30
    if args.batched_requests > 0:
        nb = args.batched_requests
        runs = {}

        def bsrv():
            return S.BatchServer(theta, None, capacity=args.batch_capacity, cycles_per_round=args.cycles_per_round,
                                 setup_threads=16, hbm_budget=budget, progress=True)
        srv = bsrv()
        res, errs, wall = srv.run(S.make_stream(nb, 0.0, seed=11), open_loop=False)
        runs["closed_loop"] = dict(S.summarize(res, wall), errors=len(errs), batches=srv.batches,
                                   fallbacks=srv.fallbacks)
        print(f"# batched closed loop: {runs['closed_loop']['solves_per_s']:.1f} solves/s over {nb} requests",
              file=sys.stderr, flush=True)
        T = runs["closed_loop"]["solves_per_s"]
        no = min(nb, args.open_requests)
        for frac in (0.5, 0.8, 1.2):
            srv = bsrv()
            res, errs, wall = srv.run(S.make_stream(no, frac * T, seed=12), open_loop=True)
            runs[f"open_loop_{frac}T"] = dict(S.summarize(res, wall), qps=frac * T, errors=len(errs),
                                              fallbacks=srv.fallbacks)
            print(f"# batched open loop {frac} T: p50 {runs[f'open_loop_{frac}T']['p50_ms']:.1f} ms, "
                  f"p99 {runs[f'open_loop_{frac}T']['p99_ms']:.1f} ms", file=sys.stderr, flush=True)
        if args.serving_compare > 0:
            # the same first requests, batched, with the plain FP64 GPU V-cycle (classical components)
            nc = args.serving_compare
            cmp = {}
            for name, th, prec in (("learned_fp32", theta, "fp32"), ("plain_fp64_classical", None, "fp64")):
                srv = S.BatchServer(th, None, precision=prec, capacity=args.batch_capacity,
                                    cycles_per_round=args.cycles_per_round, setup_threads=16, hbm_budget=budget,
                                    progress=True)
                res, errs, wall = srv.run(S.make_stream(nc, 0.0, seed=11), open_loop=False)
                sm = S.summarize(res, wall)
                by_side = sm.pop("by_side")
                cmp[name] = dict(sm, errors=len(errs), fallbacks=srv.fallbacks,
                                 mean_cycles_by_side={k: v["mean_iters"] for k, v in by_side.items()})
                print(f"# batched {name} on {nc} requests: {cmp[name]['solves_per_s']:.1f} solves/s",
                      file=sys.stderr, flush=True)
            a, b = cmp["learned_fp32"]["solves_per_s"], cmp["plain_fp64_classical"]["solves_per_s"]
            cmp["speedup"] = a / b if b > 0 else None
            runs[f"closed_loop_first_{nc}"] = cmp
        out["batched"] = dict(requests_closed_loop=nb, requests_open_loop=min(nb, args.open_requests),
                              capacity=args.batch_capacity,
                              cycles_per_round=args.cycles_per_round, **runs)
    if args.serving_requests > 0:
        n1 = args.serving_requests
        runs = {}
        res, errs, wall = S.Server(theta, None, slots=4, setup_threads=8, hbm_budget=budget).run(
            S.make_stream(n1, 0.0, seed=11), open_loop=False)
        runs["closed_loop"] = S.summarize(res, wall)
        T = runs["closed_loop"]["solves_per_s"]
        res, errs, wall = S.Server(theta, None, slots=4, setup_threads=8, hbm_budget=budget).run(
            S.make_stream(n1, 0.5 * T, seed=12), open_loop=True)
        runs["open_loop_0.5T"] = dict(S.summarize(res, wall), qps=0.5 * T)
        # flexible GMRES around the learned cycle (Sec. 4.2)
        res, errs, wall = S.Server(theta, None, slots=4, setup_threads=8, solver="fgmres", hbm_budget=budget).run(
            S.make_stream(n1, 0.0, seed=11), open_loop=False)
        runs["fgmres_closed_loop"] = S.summarize(res, wall)
        out["per_request"] = dict(requests_per_run=n1, **runs)
    for grp in ("batched", "per_request"):
        for r in out.get(grp, {}).values():
            if isinstance(r, dict):
                r.pop("by_side", None)
    print(f"# serving: {json.dumps(out)}", file=sys.stderr, flush=True)
    return out


def helmholtz(args):
    """Complex Helmholtz with an impedance boundary (Sec. 4.2): k = 16 pi on
    the 257 x 257 P1 mesh of the centred unit square (66 049 unknowns, k h =
    0.196), 5 levels, Jacobi V(1,1) where k h <= 1/2 and GMRES(4) V(1,2)
    elsewhere, two-feature K = 1 convolutions at identity initialisation,
    16 smoothed-disk sources.  FGMRES(40) to 1e-8 with the cycle or FMG as
    preconditioner, FP32 and FP64 cycles (one warm-up solve, one timed);
    the time of one cycle of the K = 1 form and of the form without
    convolution hops (K = 0); FGMRES with FP32 cycles on 6, 7 and 8 levels of
    the same problem.  The oracle's FGMRES-FMG solve of one column is the
    CPU-baseline leg's (cpu_baseline_helmholtz)."""
    import torch
    from mginputs import configs as C
    from paper_2608_29082_amd import helmholtz as HB
    w = C.helmholtz(B=16)
    h = w.hier
    J, B = h.nlevels, w.B
    dev = torch.device("cuda:0")
    f = torch.tensor(w.f, dtype=torch.complex128, device=dev)
    fn = np.linalg.norm(w.f, axis=0)
    out = {"workload": f"helmholtz-257: k = 16 pi, {h.sizes[0]} unknowns, {J} levels, impedance boundary, "
                       f"{B} smoothed-disk sources",
           "smoothers": [f"{p[0]} V({p[1]},{p[2]})" for p in w.plan], "kh": [round(h.kh(l), 3) for l in range(J)],
           "gmres_steps": w.v, "K": 1, "params": "identity initialisation (classical smoothers, two-feature form)",
           "restart": 40, "rtol": 1e-8}

    def cycle_ms(ctx, reps=20):
        fc = f.to(ctx.cycle_dtype)
        u = torch.zeros_like(fc)
        ctx.vcycle(fc, u)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for _ in range(reps):
            ctx.vcycle(fc, u)
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - ta) / reps

    for prec in ("fp32", "fp64"):
        ctx = HB.from_workload(w, precision=prec)
        for pc in ("vcycle", "fmg"):
            x = torch.zeros_like(f)
            ctx.fgmres(f, x, restart=40, max_iter=200, rtol=1e-8, precond=pc)
            x.zero_()
            torch.cuda.synchronize()
            ta = time.perf_counter()
            info = ctx.fgmres(f, x, restart=40, max_iter=200, rtol=1e-8, precond=pc)
            torch.cuda.synchronize()
            tb = time.perf_counter()
            rr = np.linalg.norm(w.f - h.A[0] @ x.cpu().numpy(), axis=0) / fn
            ok = info.code == 0 and float(rr.max()) <= 1e-8 * (1 + 1e-3)
            out[f"fgmres_{pc}_{prec}"] = {"value": B / (tb - ta) if ok else 0.0, "unit": "solves/s",
                                          "iters_max": int(info.iters.max()), "iters_mean": float(info.iters.mean()),
                                          "relres_max_fp64_host": float(rr.max()), "converged": bool(ok)}
            print(f"# helmholtz fgmres {pc} {prec}: {out[f'fgmres_{pc}_{prec}']}", file=sys.stderr, flush=True)
        out[f"cycle_ms_{prec}"] = cycle_ms(ctx)
        ctx.close()
    # the shipped trained parameters (train_helmholtz.py: Rprop on the loss after 10 cycles, training
    # sources disjoint from these), FP32 cycles, and the stationary iteration with FP64 cycles
    theta = np.load(os.path.join(ROOT, "paper_2608_29082_amd", "theta", "hz_k1_helmholtz257.npy"))
    ctx = HB.from_workload(w, precision="fp32", params=theta)
    for pc in ("vcycle", "fmg"):
        x = torch.zeros_like(f)
        ctx.fgmres(f, x, restart=40, max_iter=200, rtol=1e-8, precond=pc)
        x.zero_()
        torch.cuda.synchronize()
        ta = time.perf_counter()
        info = ctx.fgmres(f, x, restart=40, max_iter=200, rtol=1e-8, precond=pc)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        rr = np.linalg.norm(w.f - h.A[0] @ x.cpu().numpy(), axis=0) / fn
        ok = info.code == 0 and float(rr.max()) <= 1e-8 * (1 + 1e-3)
        out[f"fgmres_{pc}_fp32_learned"] = {"value": B / (tb - ta) if ok else 0.0, "unit": "solves/s",
                                            "iters_max": int(info.iters.max()),
                                            "iters_mean": float(info.iters.mean()),
                                            "relres_max_fp64_host": float(rr.max()), "converged": bool(ok)}
        print(f"# helmholtz learned fgmres {pc}: {out[f'fgmres_{pc}_fp32_learned']}", file=sys.stderr, flush=True)
    ctx.close()
    ctx = HB.from_workload(w, precision="fp64", params=theta)
    u = torch.zeros_like(f)
    ctx.solve(f, u, rtol=1e-8, max_cycles=400, check_every=5)
    u.zero_()
    torch.cuda.synchronize()
    ta = time.perf_counter()
    sinfo = ctx.solve(f, u, rtol=1e-8, max_cycles=400, check_every=5)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    rr = np.linalg.norm(w.f - h.A[0] @ u.cpu().numpy(), axis=0) / fn
    ok = sinfo.code == 0 and float(rr.max()) <= 1e-8 * (1 + 1e-3)
    out["stationary_fp64_learned"] = {"value": B / (tb - ta) if ok else 0.0, "unit": "solves/s",
                                      "cycles_max": int(sinfo.iters.max()), "cycles_mean": float(sinfo.iters.mean()),
                                      "relres_max_fp64_host": float(rr.max()), "converged": bool(ok),
                                      "note": "mgh_solve: u <- LMG(A, f, u), FP64 residual after every cycle"}
    ctx.close()
    out["params_learned"] = "hz_k1_helmholtz257 (trained on 16 random-disk sources, seeds disjoint from these)"
    # the K = 2 (polynomial) form with its own trained parameters
    w2 = C.helmholtz(B=B, K=2)
    theta2 = np.load(os.path.join(ROOT, "paper_2608_29082_amd", "theta", "hz_k2_helmholtz257.npy"))
    ctx = HB.from_workload(w2, precision="fp32", params=theta2)
    for pc in ("vcycle", "fmg"):
        x = torch.zeros_like(f)
        ctx.fgmres(f, x, restart=40, max_iter=200, rtol=1e-8, precond=pc)
        x.zero_()
        torch.cuda.synchronize()
        ta = time.perf_counter()
        info = ctx.fgmres(f, x, restart=40, max_iter=200, rtol=1e-8, precond=pc)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        rr = np.linalg.norm(w.f - h.A[0] @ x.cpu().numpy(), axis=0) / fn
        ok = info.code == 0 and float(rr.max()) <= 1e-8 * (1 + 1e-3)
        out[f"fgmres_{pc}_fp32_learned_k2"] = {"value": B / (tb - ta) if ok else 0.0, "unit": "solves/s",
                                               "iters_max": int(info.iters.max()),
                                               "iters_mean": float(info.iters.mean()),
                                               "relres_max_fp64_host": float(rr.max()), "converged": bool(ok)}
    out["cycle_ms_fp32_learned_k2"] = cycle_ms(ctx)
    ctx.close()
    ctx = HB.from_workload(w2, precision="fp64", params=theta2)
    u = torch.zeros_like(f)
    ctx.solve(f, u, rtol=1e-8, max_cycles=400, check_every=5)
    u.zero_()
    torch.cuda.synchronize()
    ta = time.perf_counter()
    sinfo = ctx.solve(f, u, rtol=1e-8, max_cycles=400, check_every=5)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    out["stationary_fp64_learned_k2"] = {"value": B / (tb - ta) if sinfo.code == 0 else 0.0, "unit": "solves/s",
                                         "cycles_max": int(sinfo.iters.max()), "converged": bool(sinfo.code == 0)}
    ctx.close()

    # deeper hierarchies of the same problem (the paper's level sweep, J = 5..8), FP32 cycles
    # (identity parameters, and the 5-level trained ones moved over by the partial transfer rule)
    from paper_2608_29082_amd import train_helmholtz as TH
    by_levels = {}
    for Jx in (6, 7, 8):
        wx = C.helmholtz(B=B, J=Jx)
        row = {"smoothers": "".join("J" if p[0] == "jacobi" else "G" for p in wx.plan),
               "coarsest_unknowns": wx.hier.sizes[-1]}
        for label, prm in (("", wx.params), ("_transferred", TH.transfer(theta, w.plan, wx.plan, 1))):
            cx_ = HB.from_workload(wx, precision="fp32", params=prm)
            for pc in ("vcycle", "fmg"):
                x = torch.zeros_like(f)
                cx_.fgmres(f, x, restart=40, max_iter=200, rtol=1e-8, precond=pc)
                x.zero_()
                torch.cuda.synchronize()
                ta = time.perf_counter()
                info = cx_.fgmres(f, x, restart=40, max_iter=200, rtol=1e-8, precond=pc)
                torch.cuda.synchronize()
                tb = time.perf_counter()
                rr = np.linalg.norm(w.f - h.A[0] @ x.cpu().numpy(), axis=0) / fn
                ok = info.code == 0 and float(rr.max()) <= 1e-8 * (1 + 1e-3)
                row[pc + label] = {"value": B / (tb - ta) if ok else 0.0, "iters_max": int(info.iters.max()),
                                   "iters_mean": float(info.iters.mean()), "converged": bool(ok)}
            cx_.close()
        by_levels[f"J{Jx}"] = row
    out["fgmres_fp32_by_levels"] = by_levels
    print(f"# helmholtz by levels: {json.dumps(by_levels)}", file=sys.stderr, flush=True)
    ctx0 = HB.HelmholtzContext(h.A, h.P, C.hz_identity_params(J, 0, 0, 0, w.plan), 0, 0, 0, w.plan, v=w.v,
                               precision="fp32", nrhs=B)
    out["cycle_ms_fp32_no_hops"] = cycle_ms(ctx0)
    ctx0.close()
    out["cycle_cost_K1_over_no_hops"] = out["cycle_ms_fp32"] / out["cycle_ms_fp32_no_hops"]
    print(f"# helmholtz: {json.dumps(out)}", file=sys.stderr, flush=True)
    return out


def device_copy_gbps(mib=256, reps=5):
    """Read + write bandwidth of a plain device-to-device copy of `mib` MiB
    (torch's copy kernel, HIP events), the practical streaming ceiling."""
    import torch
    a = torch.empty(mib * 2**20 // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    return 2 * a.numel() * 4 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9


def learned_fp64(args, h, params, f, B, stream):
    """The same learned parameters with FP64 cycles (no mixed precision), same
    right-hand sides: the mixed form's gain at equal parameters."""
    import torch
    from paper_2608_29082_amd import binding as Bd
    ctx = Bd.Context(h.A, h.P, params, args.K, args.K, args.K, precision="fp64", nrhs=B,
                     max_outer=args.max_outer, check_every=args.check_every, stream=stream)
    u = torch.zeros_like(f)
    torch.cuda.synchronize()
    ta = time.perf_counter()
    info = ctx.solve(f, u)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    ctx.close()
    out = {"value": B / (tb - ta), "unit": "solves/s", "iters_max": int(info.iters.max()),
           "converged": bool(info.code == 0)}
    print(f"# learned fp64: {out}", file=sys.stderr, flush=True)
    return out


def unbatched(args, h, params, f, stream, cols=4):
    """The learned mixed form solving one right-hand side at a time (B = 1
    contexts; no tiles, the whole coarse part in the LDS tail) on the first
    `cols` columns: solves/s = cols / total time."""
    import torch
    from paper_2608_29082_amd import binding as Bd
    ctx = Bd.Context(h.A, h.P, params, args.K, args.K, args.K, precision=args.precision, nrhs=1,
                     max_outer=args.max_outer, check_every=args.check_every, stream=stream)
    iters = []
    torch.cuda.synchronize()
    ta = time.perf_counter()
    for c in range(cols):
        fc = f[:, c:c + 1].contiguous()
        u = torch.zeros_like(fc)
        info = ctx.solve(fc, u)
        iters.append(int(info.iters.max()))
    torch.cuda.synchronize()
    tb = time.perf_counter()
    ctx.close()
    out = {"value": cols / (tb - ta), "unit": "solves/s", "columns": cols, "iters": iters}
    print(f"# learned {args.precision} unbatched: {out}", file=sys.stderr, flush=True)
    return out


def cycle_cost(args, h, params, f, B, stream):
    """Where the time goes (paper Sec. 4.2: a learnable cycle costs about 1.5 classical
    ones; Sec. 3: graph convolutions are expensive on large problems): ms per FP32
    refinement step (one V(2,2) cycle on all levels, FP64 residual and update) on
    the benchmark hierarchy and right-hand sides, learned K = 3 cycle against the
    classical K = 0 cycle (identity parameters), both FP32, the fused convolution
    and the coarse tail in both; beside the per-hop byte model's ratio of vector
    passes on a level, 2 nu 3 (K + 1) + (3 K + 1.25) + (3 K + 2.25) against 6 nu + 4.5."""
    import torch
    from mginputs import configs as C
    from paper_2608_29082_amd import binding as Bd
    J = h.nlevels
    out = {}
    for name, K, prm in (("learned_K3", args.K, params), ("classical_K0", 0, C.identity_params(J, 0, 0, 0))):
        ctx = Bd.Context(h.A, h.P, prm, K, K, K, precision="fp32", nrhs=B, stream=stream)
        u = torch.zeros_like(f)
        for _ in range(3):
            ctx.refine_step(f, u, u)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps = 30
        for _ in range(steps):
            ctx.refine_step(f, u, u)
        torch.cuda.synchronize()
        out[name] = {"ms_per_cycle": 1e3 * (time.perf_counter() - t0) / steps}
        ctx.close()
    nu, K = 2, args.K
    out["ratio_learned_over_classical"] = out["learned_K3"]["ms_per_cycle"] / out["classical_K0"]["ms_per_cycle"]
    out["per_hop_model_ratio"] = (2 * nu * 3 * (K + 1) + (3 * K + 1.25) + (3 * K + 2.25)) / (6 * nu + 4.5)
    out["paper_ratio"] = 1.5
    print(f"# cycle cost: {json.dumps(out)}", file=sys.stderr, flush=True)
    return out


def held_out(args, params, stream, seeds):
    """Solves/s and cycle counts on coefficient fields of the workload's law
    that the parameters never saw in training (the parameter file's
    `held_out_seeds`; same solver, right-hand sides of the same distribution),
    beside the benchmark's own field."""
    import torch
    from mginputs import configs as C
    from paper_2608_29082_amd import binding as Bd
    out = {}
    for sd in seeds:
        w2 = C.diffusion_513(seed=sd, B=64)
        h2 = w2.hier
        ctx = Bd.Context(h2.A, h2.P, params, args.K, args.K, args.K, precision=args.precision, nrhs=64,
                         max_outer=args.max_outer, check_every=args.check_every, stream=stream)
        f2 = torch.tensor(w2.f, dtype=torch.float64, device="cuda:0")
        u2 = torch.zeros_like(f2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = ctx.solve(f2, u2)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rr = np.linalg.norm(w2.f - h2.A[0] @ u2.cpu().numpy(), axis=0) / np.linalg.norm(w2.f, axis=0)
        out[f"field_{sd}"] = {"value": 64 / dt if info.code == 0 else 0.0, "unit": "solves/s",
                              "iters_max": int(info.iters.max()), "iters_mean": float(info.iters.mean()),
                              "relres_max_fp64_host": float(rr.max()), "converged": bool(info.code == 0)}
        ctx.close()
    print(f"# held-out fields: {json.dumps(out)}", file=sys.stderr, flush=True)
    return out


def cpu_baseline_helmholtz():
    """The CPU complex128 oracle's FGMRES(40)-FMG solve of one column (the
    training source) of the Helmholtz workload, identity parameters."""
    import resource
    from mginputs import configs as C
    from oracle import helmholtz as OH
    w = C.helmholtz(B=1)
    h = w.hier
    J = h.nlevels
    lev = OH.make_levels(h.A, h.P, h.R)
    prm = OH.unpack(w.params, J, 1, 1, 1, w.plan, w.v)
    ru0 = resource.getrusage(resource.RUSAGE_SELF)
    ta = time.perf_counter()
    _, it, rr, _ = OH.fgmres(lev, prm, w.f, restart=40, rtol=1e-8, max_iter=200, precond="fmg")
    wall = time.perf_counter() - ta
    ru1 = resource.getrusage(resource.RUSAGE_SELF)
    cpu_s = (ru1.ru_utime - ru0.ru_utime) + (ru1.ru_stime - ru0.ru_stime)
    return {"value": 1.0 / wall, "unit": "solves/s", "iters": int(it[0]), "cores": max(1, int(round(cpu_s / wall))),
            "kind": "oracle", "sample": f"one column (the training source), FGMRES(40)-FMG, {wall:.1f}s wall"}


def cpu_worker(col: int, seconds: float, K: int):
    """One oracle process (single-threaded BLAS): cycles of the learned V-cycle with the
    solver's per-cycle FP64 residual on column `col` of the benchmark workload for
    `seconds`; prints its count as one JSON line."""
    import resource
    from mginputs import configs as C
    from oracle import lmg as O
    from paper_2608_29082_amd import params as PR
    w = C.diffusion_513(B=64)
    h = w.hier
    J = h.nlevels
    theta, meta = PR.load(PR.default_file("diffusion-513", K))
    prm = O.unpack(PR.map_levels(theta, meta["J"], J, K, K, K), J, K, K, K)
    lv = O.make_levels(h.A, h.P, h.R)
    f = w.f[:, col:col + 1]
    A = h.A[0]
    u = np.zeros_like(f)
    ru0 = resource.getrusage(resource.RUSAGE_SELF)
    t0 = time.perf_counter()
    cycles = 0
    while time.perf_counter() - t0 < seconds:
        np.linalg.norm(f - A @ u, axis=0)
        u = O.lmg(lv, prm, 0, f, u)
        cycles += 1
    wall = time.perf_counter() - t0
    ru1 = resource.getrusage(resource.RUSAGE_SELF)
    cpu = (ru1.ru_utime - ru0.ru_utime) + (ru1.ru_stime - ru0.ru_stime)
    print(json.dumps({"cycles": cycles, "wall": wall, "cpu": cpu}), flush=True)


def host_cpu():
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_count": os.cpu_count(), "model": model}


def cpu_baseline(w, params, args, cycles_per_solve):
    """The CPU FP64 oracle on a bounded sample of the same workload, in the two modes
    of a CPU baseline: one process on one core (single-threaded BLAS), and N
    independent processes (one right-hand side each) over the host's cores (N =
    min(cpu_count, 16)).  Each process runs oracle cycles for --cpu-seconds after
    building its hierarchy (not timed); solves/s = columns x cycles / (seconds x
    the GPU run's mean cycle count per solve)."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    n_host = os.cpu_count() or 1
    modes = {}
    for name, nproc in (("single_process", 1), ("all_cores", max(1, min(n_host, 16)))):
        procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker", str(c),
                                   "--cpu-seconds", str(args.cpu_seconds), "--K", str(args.K)],
                                  stdout=subprocess.PIPE, stderr=subprocess.DEVNULL, env=env, text=True)
                 for c in range(nproc)]
        runs = []
        for p in procs:
            outp, _ = p.communicate(timeout=600)
            runs.append(json.loads(outp.strip().splitlines()[-1]))
        rate = sum(r["cycles"] / r["wall"] for r in runs)   # column-cycles per second over all processes
        modes[name] = {"value": rate / cycles_per_solve, "unit": "solves/s", "cores": nproc,
                       "cycles": [r["cycles"] for r in runs],
                       "cpu_over_wall": [round(r["cpu"] / r["wall"], 2) for r in runs]}
        print(f"# cpu baseline {name}: {modes[name]['value']:.4f} solves/s on {nproc} processes",
              file=sys.stderr, flush=True)
    allc = modes["all_cores"]
    return {"value": allc["value"], "unit": "solves/s", "cores": allc["cores"], "kind": "oracle",
            "sample": f"{allc['cores']} single-threaded oracle processes, one right-hand side each, "
                      f"{args.cpu_seconds:.0f} s of V-cycles with the per-cycle FP64 residual after the setup; "
                      f"solves/s = column-cycles per second / {cycles_per_solve:.0f} (the GPU run's mean cycles "
                      f"per solve)",
            "single_process": modes["single_process"], "host": host_cpu()}


if __name__ == "__main__":
    main()

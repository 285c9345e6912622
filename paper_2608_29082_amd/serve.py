"""Request loop: continuous admission of solve requests of different grid sizes.

A request is (side, coefficient blocks, right-hand side).  The loop:
  1. setup workers (threads) build the hierarchy natively (mg_square_hierarchy;
     the GIL is released inside the library), size its device footprint
     (mg_workspace_bytes plus the request's vectors) and wait for that much
     of the HBM budget to be free (admission by footprint), then set the
     context up (mg_setup) on their own stream;
  2. solve slots (threads, one HIP stream each) take admitted requests in
     arrival order and run mg_solve (FP32 or BF16 cycles, FP64 refinement) or,
     with solver="fgmres", mg_fgmres (flexible GMRES with the cycle as
     preconditioner, Sec. 4.2; its Krylov workspace is part of the request's
     footprint); the slots' kernels overlap on the GPU;
  3. a finished request releases its context and its budget; latency is
     done - arrival.
Requests that arrive while others run are admitted as budget and slots free
up; a request's result does not depend on what else is in flight (each has
its own context, stream and buffers, and every kernel is deterministic).
"""
from __future__ import annotations

import queue
import threading
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    side: int
    blocks: np.ndarray          # (16, 16) coefficient per block
    f: np.ndarray               # (n, 1) right-hand side
    arrival: float = 0.0        # seconds from the start of the stream


@dataclass
class Result:
    rid: int
    side: int
    n: int
    iters: int
    relres: float
    status: int
    t_arrival: float
    t_admitted: float
    t_started: float
    t_done: float
    footprint: int
    u: np.ndarray | None = None

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


class _Budget:
    def __init__(self, total: int):
        self.total, self.used = total, 0
        self.cv = threading.Condition()

    def acquire(self, nbytes: int):
        with self.cv:
            if nbytes > self.total:
                raise MemoryError(f"request footprint {nbytes} exceeds the HBM budget {self.total}")
            while self.used + nbytes > self.total:
                self.cv.wait()
            self.used += nbytes

    def release(self, nbytes: int):
        with self.cv:
            self.used -= nbytes
            self.cv.notify_all()


class Server:
    """theta: flat parameters trained on a J_src-level hierarchy (mapped to each
    request's level count by params.map_levels, levels matched by mesh size),
    a dict {side: (theta, J)} of parameters per grid size, or None for the
    identity (classical) parameters.  A request whose learned cycle diverges
    is solved again with the classical parameters (counted in `fallbacks`)."""

    def __init__(self, theta=None, J_src=None, K=3, precision="fp32", slots=4, setup_threads=4,
                 hbm_budget=16 << 30, rtol=1e-8, max_outer=20000, keep_solution=False, device="cuda:0",
                 solver="refine", restart=30, fail_setup=None):
        import torch
        from . import binding as Bd
        from . import params as PR
        self.torch, self.Bd, self.PR = torch, Bd, PR
        self.theta, self.J_src, self.K = theta, J_src, K
        self.precision, self.slots, self.setup_threads = precision, slots, setup_threads
        self.budget = _Budget(hbm_budget)
        self.rtol, self.max_outer, self.keep = rtol, max_outer, keep_solution
        self.device = torch.device(device)
        self.peak_used = 0
        self.fallbacks = 0
        if solver not in ("refine", "fgmres"):
            raise ValueError("solver must be 'refine' or 'fgmres'")
        self.solver, self.restart = solver, restart
        # fail_setup(request) -> bool: make that request's setup fail after admission (tests of the
        # error path: the budget it took must come back)
        self.fail_setup = fail_setup

    def _params(self, J, side):
        K = self.K
        if self.theta is None:
            return self.PR.identity(J, K, K, K)
        if isinstance(self.theta, dict):
            if side not in self.theta:
                return self.PR.identity(J, K, K, K)
            th, Js = self.theta[side]
            return self.PR.map_levels(th, Js, J, K, K, K)
        return self.PR.map_levels(self.theta, self.J_src, J, K, K, K, shift=self.J_src - J)

    def _footprint(self, hier, params, n) -> int:
        import ctypes as Cc
        Bd, K = self.Bd, self.K
        lib = Bd.load_library()
        p = np.ascontiguousarray(params)
        pr = Bd._Params(K, K, K, 2, 2, p.ctypes.data_as(Cc.POINTER(Cc.c_double)))
        o = Bd._Options(Bd.PRECISIONS[self.precision], 1, self.max_outer, 10, self.rtol, 1e6, 0)
        ws, ck = Cc.c_size_t(), Cc.c_size_t()
        Bd._check(lib.mg_workspace_bytes(Cc.byref(hier.view), Cc.byref(pr), Cc.byref(o), Cc.byref(ws),
                                         Cc.byref(ck)), "mg_workspace_bytes")
        return int(ws.value) + 2 * n * 8 + (krylov_bytes_bound(n, 1, self.restart) if self.solver == "fgmres" else 0)

    def run(self, requests, open_loop=True):
        """Serve `requests` (sorted by arrival).  open_loop: each request enters
        at its arrival time; otherwise all are queued at t = 0 (saturation)."""
        torch, Bd = self.torch, self.Bd
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0
        incoming: queue.Queue = queue.Queue()
        ready: queue.PriorityQueue = queue.PriorityQueue()
        results, errors = [], []
        lock = threading.Lock()
        n_total = len(requests)

        def setup_worker():
            stream = torch.cuda.Stream(device=self.device)
            while True:
                item = incoming.get()
                if item is None:
                    return
                req, t_arr = item
                hier = ctx = None
                fp = 0
                try:
                    hier = Bd.SquareHierarchy(req.side, req.blocks)
                    params = self._params(hier.nlevels, req.side)
                    need = self._footprint(hier, params, hier.sizes[0])
                    self.budget.acquire(need)
                    fp = need
                    with lock:
                        self.peak_used = max(self.peak_used, self.budget.used)
                    t_adm = now()
                    if self.fail_setup is not None and self.fail_setup(req):
                        raise RuntimeError(f"setup of request {req.rid} failed (injected)")
                    with torch.cuda.stream(stream):
                        ctx = Bd.Context(None, None, params, self.K, self.K, self.K, precision=self.precision,
                                         nrhs=1, max_outer=self.max_outer, check_every=10, rtol=self.rtol,
                                         stream=stream, device=self.device, native=hier)
                        f = torch.tensor(req.f, dtype=torch.float64, device=self.device)
                        work = None
                        if self.solver == "fgmres":
                            kb = ctx.fgmres_workspace_bytes(self.restart)
                            if kb > krylov_bytes_bound(hier.sizes[0], 1, self.restart):
                                raise RuntimeError("Krylov workspace exceeds its admission bound")
                            work = torch.empty(kb, dtype=torch.uint8, device=self.device)
                    stream.synchronize()
                    hier.close()
                    ready.put((t_arr, req.rid, (req, ctx, f, fp, t_arr, t_adm, work)))
                except Exception as e:  # report, give back what was taken and keep serving
                    if ctx is not None:
                        ctx.close()
                    if hier is not None:
                        hier.close()
                    if fp:
                        self.budget.release(fp)
                    with lock:
                        errors.append((req.rid, repr(e)))
                    ready.put((t_arr, req.rid, None))

        def solve_worker():
            stream = torch.cuda.Stream(device=self.device)
            while True:
                _, _, job = ready.get()
                if job == "stop":
                    return
                if job is None:
                    with lock:
                        results.append(None)
                    continue
                req, ctx, f, fp, t_arr, t_adm, work = job
                t_start = now()
                ctx.stream = stream
                with torch.cuda.stream(stream):
                    u = torch.zeros_like(f)
                    run = (lambda: ctx.fgmres(f, u, restart=self.restart, max_iter=self.max_outer, rtol=self.rtol,
                                              work=work)) if self.solver == "fgmres" else (lambda: ctx.solve(f, u))
                    info = run()
                    if info.status[0] != 0 and self.theta is not None:
                        # learned parameters failed on this request: classical cycle
                        ctx.set_params(self.PR.identity(ctx.J, self.K, self.K, self.K))
                        u.zero_()
                        info = run()
                        with lock:
                            self.fallbacks += 1
                    u_host = u.cpu().numpy() if self.keep else None
                stream.synchronize()
                t_done = now()
                ctx.close()
                del ctx, f, u, work
                self.budget.release(fp)
                with lock:
                    results.append(Result(req.rid, req.side, req.f.shape[0], int(info.iters[0]),
                                          float(info.relres[0]), int(info.status[0]), t_arr, t_adm, t_start,
                                          t_done, fp, u_host))

        setups = [threading.Thread(target=setup_worker, daemon=True) for _ in range(self.setup_threads)]
        solvers = [threading.Thread(target=solve_worker, daemon=True) for _ in range(self.slots)]
        for t in setups + solvers:
            t.start()
        for req in requests:
            if open_loop:
                delay = req.arrival - now()
                if delay > 0:
                    time.sleep(delay)
            incoming.put((req, req.arrival if open_loop else 0.0))
        for _ in setups:
            incoming.put(None)
        for t in setups:
            t.join()
        # every request is in `ready` now; stop the slots after them
        for k in range(self.slots):
            ready.put((float("inf"), k, "stop"))
        for t in solvers:
            t.join()
        wall = now()
        done = [r for r in results if r is not None]
        return done, errors, wall


def krylov_bytes_bound(n: int, B: int, m: int) -> int:
    """Upper bound of mg_fgmres_workspace_bytes for n unknowns, B columns and
    restart m: (m+1) FP64 basis vectors, m preconditioned vectors (counted at
    8 bytes), one FP64 vector, per-block partial sums for at most 1024 blocks
    and the per-column Hessenberg state, plus alignment padding."""
    nB = n * B
    return (nB * ((m + 1) * 8 + m * 8 + 8) + 128 * m * 8
            + B * 8 * (1024 * (m + 2) + (m + 1) * m + 10 * (m + 2)) + (1 << 16))


def summarize(results, wall):
    lat = np.array([r.latency for r in results])
    by_side = {}
    for r in results:
        by_side.setdefault(r.side, []).append(r)
    return {
        "requests": len(results),
        "solves_per_s": len(results) / wall if wall > 0 else 0.0,
        "p50_ms": float(np.percentile(lat, 50) * 1e3) if len(lat) else None,
        "p99_ms": float(np.percentile(lat, 99) * 1e3) if len(lat) else None,
        "max_relres": float(max(r.relres for r in results)) if results else None,
        "all_converged": all(r.status == 0 for r in results),
        "by_side": {int(s): {"n": len(v), "mean_iters": float(np.mean([r.iters for r in v])),
                             "p50_ms": float(np.percentile([r.latency for r in v], 50) * 1e3),
                             "mean_solve_ms": float(np.mean([r.t_done - r.t_started for r in v]) * 1e3)}
                    for s, v in sorted(by_side.items())},
    }


def make_stream(count, qps, seed=0, sides=None):
    """Seeded request stream: side uniform over the serving sizes, log10 a ~
    U(-2, 2) on 16 x 16 blocks, f ~ N(0, 1), Poisson arrivals at `qps`."""
    from mginputs import configs as C
    sides = sides or C.SERVING_SIDES
    arr = C.serving_arrivals(count, qps, seed) if qps else np.zeros(count)
    reqs = []
    for k in range(count):
        side, blocks = C.serving_request(k, seed, sides)
        n = (side - 2) ** 2
        reqs.append(Request(k, side, blocks, C.serving_rhs(k, n, seed), float(arr[k])))
    return reqs


def main(argv=None):
    import argparse
    import json
    import os
    from . import params as PR
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--requests", type=int, default=100)
    ap.add_argument("--qps", type=float, default=0.0, help="0: closed loop (all queued at t = 0)")
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--setup-threads", type=int, default=4)
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--params", default="default")
    ap.add_argument("--sides", default=None, help="comma-separated grid sides")
    ap.add_argument("--budget-gb", type=float, default=16.0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--solver", default="refine", choices=["refine", "fgmres"])
    ap.add_argument("--restart", type=int, default=30)
    args = ap.parse_args(argv)
    path = None
    if args.params == "identity":
        theta, J_src = None, None
    elif args.params == "default":
        theta, J_src = {}, None
        for side in (65, 129, 257, 513, 1025):
            f = PR.default_file(f"serving-{side}", 3)
            if f:
                th, meta = PR.load(f)
                theta[side] = (th, meta["J"])
        path = "per-size k3_serving*.npy"
    else:
        path = args.params
        theta, meta = PR.load(path)
        J_src = meta["J"]
    sides = [int(s) for s in args.sides.split(",")] if args.sides else None
    reqs = make_stream(args.requests, args.qps, args.seed, sides)
    srv = Server(theta, J_src, precision=args.precision, slots=args.slots, setup_threads=args.setup_threads,
                 hbm_budget=int(args.budget_gb * (1 << 30)), solver=args.solver, restart=args.restart)
    res, errs, wall = srv.run(reqs, open_loop=args.qps > 0)
    out = summarize(res, wall)
    out.update({"solver": args.solver, "qps": args.qps, "wall_s": wall, "errors": errs[:5], "peak_budget_bytes": srv.peak_used,
                "fallbacks": srv.fallbacks, "params": os.path.basename(path) if path else "identity"})
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

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

BatchServer is the continuous-batching form: requests of one grid size share
a context of column slots, each column with its own operator values
(per-column operators, mg_load_column), advanced in rounds of refinement
cycles with free slots refilled between rounds.  In both loops a request whose
learned stationary iteration fails the Progress test (divergence, no residual
below ||f|| after 64 cycles, no new best residual for 128 cycles) is solved by
flexible GMRES around the same learned cycle, and if that fails too, around
the classical cycle.
"""
from __future__ import annotations

import queue
import sys
import threading
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    side: int
    blocks: np.ndarray          # (16, 16) coefficient per block
    f_data: np.ndarray | None = None   # (n, 1) right-hand side, or None: drawn from the stream seed when used
    arrival: float = 0.0        # seconds from the start of the stream
    seed: int = 0               # stream seed of a drawn right-hand side

    @property
    def n(self) -> int:
        return (self.side - 2) ** 2

    @property
    def f(self) -> np.ndarray:
        """The right-hand side (drawn again at each use when not stored, so a long
        stream does not hold every request's vector in host memory)."""
        if self.f_data is not None:
            return self.f_data
        from mginputs import configs as C
        return C.serving_rhs(self.rid, self.n, self.seed)


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
    fallback: bool = False      # left the learned stationary iteration (diverged or stalled); solved by
                                # FGMRES around the learned cycle, or around the classical one

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


class Progress:
    """Stop test of the learned stationary iteration, applied by both request
    loops at the end of every round of cycles (a request's own cycle count
    `it`): the request leaves the learned iteration when the solver reports
    divergence or its residual exceeds `diverge_factor` ||f||, when after
    `stall_cycles` cycles its residual is still not below ||f||, or when its
    best residual has not improved for `window` cycles (a slowly diverging or
    stagnating iteration)."""

    def __init__(self, diverge_factor=1e6, stall_cycles=64, window=128):
        self.diverge_factor, self.stall_cycles, self.window = diverge_factor, stall_cycles, window
        self.best, self.best_it = float("inf"), 0

    def failed(self, it: int, relres: float, status: int) -> bool:
        if status == 6 or not relres <= self.diverge_factor:
            return True
        if relres < self.best:
            self.best, self.best_it = relres, it
        if self.stall_cycles and it >= self.stall_cycles and not relres < 1.0:
            return True
        return bool(self.window) and it - self.best_it >= self.window


class Server:
    """theta: flat parameters trained on a J_src-level hierarchy (mapped to each
    request's level count by params.map_levels, levels matched by mesh size),
    a dict {side: (theta, J)} of parameters per grid size, or None for the
    identity (classical) parameters.

    A request whose learned stationary iteration diverges (the library's
    divergence test), or has not brought its residual below ||f|| after
    `stall_cycles` cycles, is solved again from zero by flexible GMRES(restart)
    preconditioned with the same learned cycle (a Krylov method converges where
    the stationary iteration of a few bad modes does not), and if that fails
    too, around the classical cycle; counted in `fallbacks`, its iteration
    count is then the FGMRES one.  With solver="fgmres" a failed learned FGMRES
    solve is repeated around the classical cycle."""

    def __init__(self, theta=None, J_src=None, K=3, precision="fp32", slots=4, setup_threads=4,
                 hbm_budget=16 << 30, rtol=1e-8, max_outer=20000, keep_solution=False, device="cuda:0",
                 solver="refine", restart=30, fail_setup=None, stall_cycles=64, stall_window=128,
                 round_cycles=8, diverge_factor=1e6, fallback_iters=2000, budget=None):
        import torch
        from . import binding as Bd
        from . import params as PR
        self.torch, self.Bd, self.PR = torch, Bd, PR
        self.theta, self.J_src, self.K = theta, J_src, K
        self.precision, self.slots, self.setup_threads = precision, slots, setup_threads
        self.budget = budget if budget is not None else _Budget(hbm_budget)   # shareable between loops
        self.rtol, self.max_outer, self.keep = rtol, max_outer, keep_solution
        self.device = torch.device(device)
        self.peak_used = 0
        self.fallbacks = 0
        if solver not in ("refine", "fgmres"):
            raise ValueError("solver must be 'refine' or 'fgmres'")
        self.solver, self.restart = solver, restart
        self.stall_cycles, self.fallback_iters = stall_cycles, fallback_iters
        self.stall_window, self.round_cycles, self.diverge_factor = stall_window, round_cycles, diverge_factor
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

    def _stationary(self, ctx, f, u):
        """The refinement solver from u = 0.  With learned parameters it runs in
        rounds of `round_cycles` cycles with the Progress test after each (the
        batched loop's rounds and test, so both loops take the same decisions);
        the iteration depends only on the current iterate, so the rounds change
        no bit.  With the classical parameters it is one solve."""
        if self.theta is None:
            return ctx.solve(f, u)
        prog = Progress(self.diverge_factor, self.stall_cycles, self.stall_window)
        total, st, rr = 0, 5, float("nan")
        while total < self.max_outer:
            ctx.set_solver_options(max_outer=min(self.round_cycles, self.max_outer - total))
            info = ctx.solve(f, u)
            total += int(info.iters[0])
            st, rr = int(info.status[0]), float(info.relres[0])
            if st == 0:
                break
            if prog.failed(total, rr, st):
                st = 6
                break
        ctx.set_solver_options(max_outer=self.max_outer)
        return self.Bd.SolveInfo(np.array([total]), np.array([st]), np.array([rr]), st)

    def _krylov(self, ctx, f, u, work):
        """FGMRES(restart) from zero around the context's cycle, then (learned
        parameters failing) around the classical cycle.  Returns (info, fell)."""
        torch = self.torch
        owned = work is None
        if owned:   # a stationary solver's context: its fallback workspace was counted at admission
            kb = ctx.fgmres_workspace_bytes(self.restart)
            if kb > krylov_bytes_bound(ctx.n[0], 1, self.restart):
                raise RuntimeError("Krylov workspace exceeds its admission bound")
            work = torch.empty(kb, dtype=torch.uint8, device=self.device)
        try:
            iters = self.fallback_iters if owned else self.max_outer
            run = lambda: ctx.fgmres(f, u, restart=self.restart, max_iter=iters, rtol=self.rtol, work=work)
            u.zero_()
            info = run()
            fell = owned            # reached from a failed stationary solve
            if info.status[0] != 0 and self.theta is not None:
                ctx.set_params(self.PR.identity(ctx.J, self.K, self.K, self.K))
                u.zero_()
                info = run()
                fell = True
            return info, fell
        finally:
            if owned:
                torch.cuda.current_stream(self.device).synchronize()
                del work

    def _solve_one(self, ctx, f, u, work):
        """One request on its context: (SolveInfo, fell back)."""
        if self.solver == "fgmres":
            return self._krylov(ctx, f, u, work)
        info = self._stationary(ctx, f, u)
        if info.status[0] == 0 or self.theta is None:
            return info, False
        info, _ = self._krylov(ctx, f, u, None)
        return info, True

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
        # a Krylov workspace: the FGMRES solver's, or the fallback's of a learned stationary solver
        # (counted at admission, so that a fallback never waits for budget that admitted requests hold)
        krylov = self.solver == "fgmres" or self.theta is not None
        return int(ws.value) + 2 * n * 8 + (krylov_bytes_bound(n, 1, self.restart) if krylov else 0)

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
                try:
                    with torch.cuda.stream(stream):
                        u = torch.zeros_like(f)
                        info, fell = self._solve_one(ctx, f, u, work)
                        if fell:
                            with lock:
                                self.fallbacks += 1
                        u_host = u.cpu().numpy() if self.keep else None
                    stream.synchronize()
                except Exception as e:  # report the request, free what it holds and keep serving
                    ctx.close()
                    del ctx, f, work
                    self.budget.release(fp)
                    with lock:
                        errors.append((req.rid, repr(e)))
                        results.append(None)
                    continue
                t_done = now()
                ctx.close()
                del ctx, f, u, work
                self.budget.release(fp)
                with lock:
                    results.append(Result(req.rid, req.side, req.n, int(info.iters[0]),
                                          float(info.relres[0]), int(info.status[0]), t_arr, t_adm, t_start,
                                          t_done, fp, u_host, fell))

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


class Intake:
    """Requests waiting for setup in the batched loop: one FIFO per grid side,
    and per side the number of hierarchies set up (or being set up) that no
    batch slot has taken yet, at most `limit` (host memory).  A setup worker
    takes the oldest request among the sides below their limit, so a side
    whose batch is full does not hold up the requests of the other sides
    behind it."""

    def __init__(self, limit: int):
        import collections
        self._deque = collections.deque
        self.limit = limit
        self.cv = threading.Condition()
        self.q = {}          # side -> deque of (arrival order, request, arrival time)
        self.held = {}       # side -> hierarchies not yet in a slot
        self.seq = 0
        self.closed = False

    def put(self, req, t_arr: float):
        with self.cv:
            self.q.setdefault(req.side, self._deque()).append((self.seq, req, t_arr))
            self.seq += 1
            self.cv.notify()

    def close(self):
        """No more requests will be put."""
        with self.cv:
            self.closed = True
            self.cv.notify_all()

    def take(self):
        """(request, arrival time) to set up next, its side's count raised; None
        once closed and empty.  Waits while every waiting side is at its limit."""
        with self.cv:
            while True:
                best = None
                for side, dq in self.q.items():
                    if dq and self.held.get(side, 0) < self.limit and (best is None or dq[0][0] < self.q[best][0][0]):
                        best = side
                if best is not None:
                    _, req, t_arr = self.q[best].popleft()
                    self.held[best] = self.held.get(best, 0) + 1
                    return req, t_arr
                if self.closed and not any(self.q.values()):
                    return None
                self.cv.wait()

    def release(self, side: int):
        """A hierarchy of `side` went into a slot (or its setup failed)."""
        with self.cv:
            self.held[side] -= 1
            self.cv.notify_all()


def pattern_key(hier) -> str:
    """Key of a native hierarchy's level patterns (row pointers and columns of
    every A_l): requests with equal keys can share a batch context.  The arrays
    are hashed in place (xxh3-128, or SHA-1 where xxhash is not installed)."""
    try:
        import xxhash
        hs = xxhash.xxh3_128()
    except ImportError:
        import hashlib
        hs = hashlib.sha1()
    for l in range(hier.nlevels):
        m = hier.view.A[l]
        hs.update(np.ctypeslib.as_array(m.rowptr, shape=(m.nrows + 1,)))
        if m.nnz > 0:
            hs.update(np.ctypeslib.as_array(m.col, shape=(int(m.nnz),)))
    return f"{hier.sizes[0]}:{hs.hexdigest()[:16]}"


class BatchServer:
    """Continuous batching of solve requests (stationary refinement solver).

    Requests whose hierarchies have the same level patterns (in practice: the
    same grid side) share one batch context of `capacity` column slots with
    per-column operators (mg_hierarchy.ncolumn_values): each request brings its
    own coefficient field's operators into its slot (mg_load_column), its right-
    hand side into column b of f and a zero start into column b of u.  A group
    worker (one thread and HIP stream per batch, so batches of different sides
    overlap on the GPU) runs rounds of at most `cycles_per_round` refinement
    cycles (mg_solve); between rounds it takes finished requests out and puts
    waiting ones into the free slots, so a request that arrives while others
    run starts at the next round boundary.  The iteration u <- u + LMG(A, f - A u, 0)
    depends only on the current iterate, so a request's iterates, cycle count
    and result are the same whatever the rounds and whatever the other columns
    hold (columns are independent; empty slots carry f = 0 and are skipped by
    the solver's column compaction).  Setup workers build the hierarchies and
    draw the right-hand sides; they take requests from an Intake, one queue
    per grid side with at most 2 x capacity set-up hierarchies per side
    waiting for slots, so a side whose batch is full never holds up the other
    sides.  Each batch's device footprint (workspace,
    tile lists excluded, plus f and u) is acquired from the HBM budget before its
    context is set up and released when the batch retires.  A request whose
    learned cycle diverges, or stalls (Server's test), leaves the batch and is
    solved on its own by FGMRES around the learned cycle, then around the
    classical one (counted in `fallbacks`)."""

    def __init__(self, theta=None, J_src=None, K=3, precision="fp32", capacity=32, cycles_per_round=8,
                 setup_threads=4, hbm_budget=16 << 30, rtol=1e-8, max_outer=20000, keep_solution=False,
                 device="cuda:0", fail_setup=None, diverge_factor=1e6, progress=False, stall_cycles=64,
                 stall_window=128, fallback_iters=2000):
        import torch
        from . import binding as Bd
        from . import params as PR
        self.torch, self.Bd, self.PR = torch, Bd, PR
        self.theta, self.J_src, self.K = theta, J_src, K
        self.precision, self.capacity = precision, capacity
        self.diverge_factor = diverge_factor
        self.stall_cycles, self.fallback_iters = stall_cycles, fallback_iters
        self.stall_window = stall_window
        self.fallback_workers = 8   # each rebuilds its request's hierarchy on the host, then runs FGMRES
        self.idle_s = 0.25          # an idle batch retires after this long without requests
        self.progress = progress    # a line on stderr every ~10 s while batches run
        self.cycles_per_round, self.setup_threads = cycles_per_round, setup_threads
        self.budget = _Budget(hbm_budget)
        self.rtol, self.max_outer, self.keep = rtol, max_outer, keep_solution
        self.device = torch.device(device)
        self.peak_used = 0
        self.fallbacks = 0
        self.batches = 0
        self.fail_setup = fail_setup
        self._learned = Server(theta, J_src, K, precision, slots=1, setup_threads=1, hbm_budget=hbm_budget,
                               rtol=rtol, max_outer=max_outer, keep_solution=keep_solution, device=device)
        # the fallback of a request that left the batch: FGMRES around the learned cycle, then around
        # the classical one (the same chain as Server's after its stationary solve failed)
        self._fallback_args = dict(K=K, precision=precision, slots=1, setup_threads=1, hbm_budget=hbm_budget,
                                   rtol=rtol, max_outer=fallback_iters, keep_solution=keep_solution,
                                   device=device, solver="fgmres")

    def _params(self, J, side):
        return self._learned._params(J, side)

    def _footprint(self, hier, params) -> int:
        import ctypes as Cc
        Bd, K, cap = self.Bd, self.K, self.capacity
        lib = Bd.load_library()
        p = np.ascontiguousarray(params)
        pr = Bd._Params(K, K, K, 2, 2, p.ctypes.data_as(Cc.POINTER(Cc.c_double)))
        o = Bd._Options(Bd.PRECISIONS[self.precision], cap, self.max_outer, 2, self.rtol, 1e6, 0)
        hh = Bd._Hier()
        Cc.memmove(Cc.byref(hh), Cc.byref(hier.view), Cc.sizeof(Bd._Hier))
        vals = (Cc.POINTER(Cc.c_double) * (hier.nlevels * cap))()
        for l in range(hier.nlevels):
            for b in range(cap):
                vals[l * cap + b] = hier.view.A[l].val
        hh.ncolumn_values = cap
        hh.column_values = vals
        ws, ck = Cc.c_size_t(), Cc.c_size_t()
        Bd._check(lib.mg_workspace_bytes(Cc.byref(hh), Cc.byref(pr), Cc.byref(o), Cc.byref(ws), Cc.byref(ck)),
                  "mg_workspace_bytes")
        return int(ws.value) + 2 * hier.sizes[0] * cap * 8

    def run(self, requests, open_loop=True):
        """Serve `requests` (sorted by arrival).  open_loop: each request enters
        at its arrival time; otherwise all are queued at t = 0 (saturation)."""
        torch, Bd = self.torch, self.Bd
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0
        # built hierarchies wait on the host until a slot takes them: at most 2 * capacity per side
        intake = Intake(2 * self.capacity)
        results, errors = [], []
        lock = threading.Lock()
        groups = {}          # pattern key -> group record
        workers = []
        setups_done = threading.Event()

        class Group:
            def __init__(self, key):
                self.key = key
                self.q: queue.Queue = queue.Queue()
                self.alive = True

        def admit(item):
            """Put a set-up request into its batch group, creating the group (and its worker) when the
            grid has none or its batch has retired."""
            key = item[3]
            with lock:
                g = groups.get(key)
                if g is None or not g.alive:
                    g = groups[key] = Group(key)
                    th = threading.Thread(target=group_worker, args=(g,), daemon=True)
                    workers.append(th)
                    th.start()
                g.q.put(item)

        def retire(g) -> bool:
            """An idle batch retires (freeing its context and budget) unless work arrived meanwhile."""
            with lock:
                if not g.q.empty():
                    return False
                g.alive = False
                if groups.get(g.key) is g:
                    del groups[g.key]
                return True

        def setup_worker():
            while True:
                it = intake.take()
                if it is None:
                    return
                req, t_arr = it
                hier = None
                try:
                    hier = Bd.SquareHierarchy(req.side, req.blocks)
                    if self.fail_setup is not None and self.fail_setup(req):
                        raise RuntimeError(f"setup of request {req.rid} failed (injected)")
                    # the right-hand side is drawn here, in parallel, not in the batch's thread
                    fv = torch.from_numpy(np.ascontiguousarray(req.f[:, 0], dtype=np.float64)).pin_memory()
                    admit((req, t_arr, hier, pattern_key(hier), fv))
                except Exception as e:  # report and keep serving
                    if hier is not None:
                        hier.close()
                    intake.release(req.side)
                    with lock:
                        errors.append((req.rid, repr(e)))

        def finish(req, t_arr, t_adm, t_start, iters, relres, status, fp, u_host, fell=False):
            with lock:
                results.append(Result(req.rid, req.side, req.n, iters, relres, status, t_arr, t_adm, t_start,
                                      now(), fp, u_host, fell))

        # the learned cycle diverged on a request: the classical cycle solves it on its own, in a
        # fallback worker, so that the batch it left keeps running
        fallback_q: queue.Queue = queue.Queue()
        fallback_threads = []

        def fallback_worker():
            krylov = Server(self.theta, self.J_src, budget=self.budget, **self._fallback_args)
            while True:
                job = fallback_q.get()
                if job is None:
                    return
                req, t_arr, t_adm, t_start, fp = job
                res, errs, _ = krylov.run([Request(req.rid, req.side, req.blocks, req.f_data, 0.0, req.seed)],
                                          open_loop=False)
                if res:
                    r = res[0]
                    finish(req, t_arr, t_adm, t_start, r.iters, r.relres, r.status, fp, r.u, True)
                else:
                    with lock:
                        errors.append((req.rid, "fallback failed: " + repr(errs[:1])))

        def fallback(req, t_arr, t_adm, t_start, iters, fp):
            with lock:
                self.fallbacks += 1
                if not fallback_threads:
                    for _ in range(self.fallback_workers):
                        th = threading.Thread(target=fallback_worker, daemon=True)
                        fallback_threads.append(th)
                        th.start()
            fallback_q.put((req, t_arr, t_adm, t_start, fp))

        def group_worker(g):
            stream = torch.cuda.Stream(device=self.device)
            cap = self.capacity
            ctx = None
            fp = 0
            slots = [None] * cap      # (req, t_arr, t_adm, t_start, iters so far)
            pending = []
            try:
                with torch.cuda.stream(stream):
                    first = g.q.get()
                    pending.append(first)
                    req0, _, hier0 = first[:3]
                    params = self._params(hier0.nlevels, req0.side)
                    fp = self._footprint(hier0, params)
                    self.budget.acquire(fp)
                    with lock:
                        self.peak_used = max(self.peak_used, self.budget.used)
                        self.batches += 1
                    ctx = Bd.Context(None, None, params, self.K, self.K, self.K, precision=self.precision, nrhs=cap,
                                     max_outer=self.cycles_per_round, check_every=2, rtol=self.rtol, stream=stream,
                                     device=self.device, native=hier0, columns=[hier0] * cap)
                    n = hier0.sizes[0]
                    f = torch.zeros((n, cap), dtype=torch.float64, device=self.device)
                    u = torch.zeros_like(f)
                    while True:
                        # fill free slots with waiting requests of this group
                        while True:
                            free = [b for b in range(cap) if slots[b] is None]
                            if not free:
                                break
                            if not pending:
                                try:
                                    pending.append(g.q.get_nowait())
                                except queue.Empty:
                                    break
                            req, t_arr, hier, _, fv = pending.pop(0)
                            b = free[0]
                            try:
                                ctx.load_column(b, hier)
                            finally:
                                hier.close()
                                intake.release(req.side)
                            f[:, b].copy_(fv, non_blocking=True)
                            u[:, b] = 0.0
                            slots[b] = [req, t_arr, now(), None, 0,
                                        Progress(self.diverge_factor, self.stall_cycles, self.stall_window)]
                        busy = [b for b in range(cap) if slots[b] is not None]
                        if not busy:
                            # idle: wait a little for more requests of this grid, else retire (so
                            # that a batch never holds budget another grid's batch waits for)
                            try:
                                pending.append(g.q.get(timeout=0.02 if setups_done.is_set() else self.idle_s))
                            except queue.Empty:
                                if retire(g):
                                    break
                            continue
                        t_round = now()
                        for b in busy:
                            if slots[b][3] is None:
                                slots[b][3] = t_round
                        info = ctx.solve(f, u)
                        for b in busy:
                            req, t_arr, t_adm, t_start, it, prog = slots[b]
                            it += int(info.iters[b])
                            st = int(info.status[b])
                            rr = float(info.relres[b])
                            # relres is against the request's start (u = 0, so ||f||), not this round's;
                            # learned parameters: the Progress test (Server's, at the same cycle counts
                            # when the rounds have the same length); classical: divergence only
                            if st != 0 and (prog.failed(it, rr, st) if self.theta is not None
                                            else not rr <= self.diverge_factor):
                                st = 6
                            done = st == 0 or st == 6 or it >= self.max_outer
                            if not done:
                                slots[b][4] = it
                                continue
                            slots[b] = None
                            if st == 6 and self.theta is not None:
                                f[:, b] = 0.0
                                u[:, b] = 0.0
                                fallback(req, t_arr, t_adm, t_start, it, fp)
                                continue
                            u_host = u[:, b].cpu().numpy()[:, None] if self.keep else None
                            stream.synchronize()
                            finish(req, t_arr, t_adm, t_start, it, float(info.relres[b]), 0 if st == 0 else
                                   (6 if st == 6 else 5), fp, u_host)
                            f[:, b] = 0.0
                            u[:, b] = 0.0
                    stream.synchronize()
            except Exception as e:
                # the batch failed: report every request it held or would have taken
                left = [sl[0] for sl in slots if sl is not None]
                waiting = list(pending)
                while True:
                    try:
                        waiting.append(g.q.get_nowait())
                    except queue.Empty:
                        break
                for rq, _, hh, *_ in waiting:   # built hierarchies never loaded: free them
                    hh.close()
                    intake.release(rq.side)
                left += [it[0] for it in waiting]
                with lock:
                    errors.append(("group " + g.key, repr(e)))
                    for rq in left:
                        errors.append((rq.rid, "batch failed"))
            finally:
                if ctx is not None:
                    ctx.close()
                if fp:
                    self.budget.release(fp)

        setups = [threading.Thread(target=setup_worker, daemon=True) for _ in range(self.setup_threads)]
        for t in setups:
            t.start()
        for req in requests:
            if open_loop:
                delay = req.arrival - now()
                if delay > 0:
                    time.sleep(delay)
            intake.put(req, req.arrival if open_loop else 0.0)
        intake.close()
        last = now()
        for t in setups:
            while t.is_alive():
                t.join(timeout=0.5)
                if self.progress and now() - last > 10.0:
                    last = now()
                    with lock:
                        print(f"# batched serving: {len(results)} done, {len(errors)} errors, {now():.0f} s",
                              file=sys.stderr, flush=True)
        setups_done.set()
        while True:
            with lock:
                ws = list(workers)
            if all(not w.is_alive() for w in ws):
                break
            for w in ws:
                w.join(timeout=0.1)
            if self.progress and now() - last > 10.0:
                last = now()
                with lock:
                    print(f"# batched serving: {len(results)} done, {len(errors)} errors, {now():.0f} s",
                          file=sys.stderr, flush=True)
        # every batch has retired, so no fallback can be added any more
        with lock:
            fts = list(fallback_threads)
        for _ in fts:
            fallback_q.put(None)
        for th in fts:
            while th.is_alive():
                th.join(timeout=0.5)
                if self.progress and now() - last > 10.0:
                    last = now()
                    print(f"# batched serving: {len(results)} done, fallbacks running, {now():.0f} s",
                          file=sys.stderr, flush=True)
        wall = now()
        return results, errors, wall


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
        reqs.append(Request(k, side, blocks, None, float(arr[k]), seed))
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

"""Request loop: every request reaches 1e-8 (checked in FP64 on the host), a
request's result is identical alone and in a mix of concurrent requests of
other sizes, and admission respects the HBM budget."""
import numpy as np
import pytest

from mginputs import hierarchy as H

pytestmark = pytest.mark.gpu


def _server(**kw):
    from paper_2608_29082_amd import params as PR
    from paper_2608_29082_amd import serve as S
    theta = {}
    for side in (65, 129):
        f = PR.default_file(f"serving-{side}", 3)
        if f:
            th, meta = PR.load(f)
            theta[side] = (th, meta["J"])
    return S.Server(theta, None, keep_solution=True, **kw)


def _relres(req, u):
    A = H.square_hierarchy(req.side, req.blocks).A[0]
    return np.linalg.norm(req.f - A @ u) / np.linalg.norm(req.f)


def test_mixed_stream_converges_and_is_invariant():
    from paper_2608_29082_amd import serve as S
    reqs = S.make_stream(10, 0.0, seed=3, sides=(33, 65, 129))
    srv = _server(slots=3, setup_threads=3)
    res, errs, wall = srv.run(reqs, open_loop=False)
    assert not errs and len(res) == len(reqs)
    byid = {r.rid: r for r in res}
    for q in reqs:
        r = byid[q.rid]
        assert r.status == 0 and _relres(q, r.u) <= 1e-8, (q.side, r.relres)
    # the same requests alone, one at a time
    for q in reqs[:4]:
        alone, e2, _ = _server(slots=1, setup_threads=1).run([q], open_loop=False)
        assert not e2 and alone[0].iters == byid[q.rid].iters
        assert np.array_equal(alone[0].u, byid[q.rid].u)


def test_admission_respects_budget():
    from paper_2608_29082_amd import serve as S
    reqs = S.make_stream(6, 0.0, seed=4, sides=(65, 129))
    probe = _server(slots=2, setup_threads=2)
    res, errs, _ = probe.run(reqs, open_loop=False)
    assert not errs
    biggest = max(r.footprint for r in res)
    srv = _server(slots=2, setup_threads=2, hbm_budget=biggest)
    res2, errs2, _ = srv.run(reqs, open_loop=False)
    assert not errs2 and len(res2) == len(reqs)
    assert srv.peak_used <= biggest
    # at every admission, the footprints of the requests holding memory fit the budget
    for r in res2:
        held = sum(x.footprint for x in res2 if x.t_admitted <= r.t_admitted < x.t_done)
        assert held <= biggest


def test_fgmres_serving_converges_and_is_invariant():
    """solver="fgmres": every request reaches 1e-8 in far fewer
    preconditioner calls than stationary cycles, the Krylov workspace stays
    within its admission bound, and results are the same alone and mixed."""
    from paper_2608_29082_amd import serve as S
    reqs = S.make_stream(8, 0.0, seed=5, sides=(33, 65, 129))
    srv = _server(slots=3, setup_threads=3, solver="fgmres")
    res, errs, wall = srv.run(reqs, open_loop=False)
    assert not errs and len(res) == len(reqs)
    ref, _, _ = _server(slots=3, setup_threads=3).run(reqs, open_loop=False)
    iters_ref = {r.rid: r.iters for r in ref}
    byid = {r.rid: r for r in res}
    for q in reqs:
        r = byid[q.rid]
        assert r.status == 0 and _relres(q, r.u) <= 1e-8 * (1 + 1e-3), (q.side, r.relres)
        assert r.iters < iters_ref[q.rid]
    for q in reqs[:3]:
        alone, e2, _ = _server(slots=1, setup_threads=1, solver="fgmres").run([q], open_loop=False)
        assert not e2 and alone[0].iters == byid[q.rid].iters
        assert np.array_equal(alone[0].u, byid[q.rid].u)


def test_failed_setup_returns_its_budget():
    """A request whose setup fails after admission is reported as an error and
    gives its HBM budget back: with a budget of one request, later requests are
    still admitted and served, and nothing is held at the end."""
    from paper_2608_29082_amd import serve as S
    reqs = S.make_stream(5, 0.0, seed=6, sides=(65,))
    probe = _server(slots=1, setup_threads=1)
    res, errs, _ = probe.run(reqs, open_loop=False)
    assert not errs
    srv = _server(slots=2, setup_threads=2, hbm_budget=max(r.footprint for r in res),
                  fail_setup=lambda q: q.rid in (0, 2))
    res2, errs2, _ = srv.run(reqs, open_loop=False)
    assert sorted(r for r, _ in errs2) == [0, 2]
    assert sorted(r.rid for r in res2) == [1, 3, 4]
    assert all(r.status == 0 for r in res2)
    assert srv.budget.used == 0


def _batch_server(**kw):
    from paper_2608_29082_amd import params as PR
    from paper_2608_29082_amd import serve as S
    theta = {}
    for side in (65, 129, 257):
        f = PR.default_file(f"serving-{side}", 3)
        if f:
            th, meta = PR.load(f)
            theta[side] = (th, meta["J"])
    return S.BatchServer(theta, None, keep_solution=True, **kw)


def test_batched_stream_converges_and_is_invariant():
    """Continuous batching: 40 requests of three sides (more than the 16 column
    slots per side, so slots are refilled between rounds) all reach 1e-8 in
    FP64 on the host; a request served alone (alone in its batch) and in the
    stream gives the same cycle count and the same bits; the batches overlap."""
    from paper_2608_29082_amd import serve as S
    reqs = S.make_stream(40, 0.0, seed=8, sides=(65, 129, 257))
    srv = _batch_server(capacity=16, cycles_per_round=6)
    res, errs, wall = srv.run(reqs, open_loop=False)
    assert not errs and len(res) == len(reqs), errs[:3]
    byid = {r.rid: r for r in res}
    for q in reqs:
        r = byid[q.rid]
        assert r.status == 0 and _relres(q, r.u) <= 1e-8, (q.side, r.relres)
    print(f"batched: {len(res)} requests in {wall:.2f} s, {srv.batches} batches, fallbacks {srv.fallbacks}",
          flush=True)
    for q in reqs[:5]:
        alone, e2, _ = _batch_server(capacity=16, cycles_per_round=5).run([q], open_loop=False)
        assert not e2 and alone[0].iters == byid[q.rid].iters
        assert np.array_equal(alone[0].u, byid[q.rid].u)


def test_batched_matches_per_request_solver():
    """The batched loop and the per-request loop solve the same requests to
    1e-8 with the same cycle counts up to one cycle at the threshold (different
    launch configurations round differently) and nearly the same iterates."""
    from paper_2608_29082_amd import serve as S
    reqs = S.make_stream(12, 0.0, seed=9, sides=(65, 129))
    rb, eb, _ = _batch_server(capacity=16).run(reqs, open_loop=False)
    rs, es, _ = _server(slots=3, setup_threads=3).run(reqs, open_loop=False)
    assert not eb and not es
    b, s = {r.rid: r for r in rb}, {r.rid: r for r in rs}
    for q in reqs:
        # both loops leave the learned stationary iteration for the same requests
        assert b[q.rid].fallback == s[q.rid].fallback
        assert abs(b[q.rid].iters - s[q.rid].iters) <= 1
        d = np.abs(b[q.rid].u - s[q.rid].u).max() / np.abs(s[q.rid].u).max()
        assert d <= 1e-6, d


def test_batched_budget_and_failed_setup():
    """A failed setup is reported and the rest served; with a budget of one
    batch, batches of different sides run one after the other and the budget
    comes back to zero."""
    from paper_2608_29082_amd import serve as S
    reqs = S.make_stream(10, 0.0, seed=10, sides=(65, 129))
    probe = _batch_server(capacity=16)
    hier = __import__("paper_2608_29082_amd.binding", fromlist=["x"]).SquareHierarchy(129, reqs[0].blocks)
    params = probe._params(hier.nlevels, 129)
    big = probe._footprint(hier, params)
    hier.close()
    srv = _batch_server(capacity=16, hbm_budget=big, fail_setup=lambda q: q.rid == 4)
    res, errs, _ = srv.run(reqs, open_loop=False)
    assert [r for r, _ in errs] == [4]
    assert sorted(r.rid for r in res) == [k for k in range(10) if k != 4]
    assert all(r.status == 0 for r in res)
    assert srv.peak_used <= big and srv.budget.used == 0


def _overshooting(sides):
    """Identity parameters with eta = 4 on every level: the damped Jacobi
    smoother overshoots and the stationary iteration diverges."""
    from paper_2608_29082_amd import params as PR
    from paper_2608_29082_amd import binding as Bd
    theta = {}
    for side in sides:
        h = Bd.SquareHierarchy(side, np.ones((16, 16)))
        J = h.nlevels
        h.close()
        p = PR.identity(J, 3, 3, 3).reshape(J - 1, -1)
        p[:, 1] = 4.0
        theta[side] = (p.ravel(), J)
    return theta


def test_fallback_chain_same_in_both_loops():
    """Requests whose learned stationary iteration diverges leave it (the
    divergence test or the stall test after 64 cycles) and are solved by FGMRES
    around the same cycle, else around the classical one: every request
    reaches 1e-8, is marked as a fallback, and the per-request and batched
    loops give the same FGMRES iteration counts and the same bits."""
    from paper_2608_29082_amd import serve as S
    reqs = S.make_stream(6, 0.0, seed=11, sides=(65, 129))
    theta = _overshooting((65, 129))
    rs, es, _ = S.Server(theta, None, keep_solution=True, slots=2, setup_threads=2).run(reqs, open_loop=False)
    bsrv = S.BatchServer(theta, None, keep_solution=True, capacity=16)
    rb, eb, _ = bsrv.run(reqs, open_loop=False)
    assert not es and not eb, (es[:2], eb[:2])
    s, b = {r.rid: r for r in rs}, {r.rid: r for r in rb}
    assert bsrv.fallbacks == len(reqs)
    for q in reqs:
        assert s[q.rid].fallback and b[q.rid].fallback
        assert s[q.rid].status == 0 and b[q.rid].status == 0
        assert _relres(q, s[q.rid].u) <= 1e-8 and _relres(q, b[q.rid].u) <= 1e-8
        assert s[q.rid].iters == b[q.rid].iters
        assert np.array_equal(s[q.rid].u, b[q.rid].u)
    print("fallback FGMRES iterations:", sorted((q.side, s[q.rid].iters) for q in reqs), flush=True)

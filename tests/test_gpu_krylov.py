"""GPU parity of full multigrid and of flexible GMRES with the learnable cycle
as preconditioner (mg_fmg, mg_fgmres) against the oracle (oracle/krylov.py)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from mginputs import configs as C
from oracle import krylov as KR
from oracle import mixed as MX
from oracle import lmg as O
from tests.gpu_util import ctx_for, oracle_levels, oracle_params, elem_rel, small_cases, to_dev, to_np

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 2e-5, "bf16": 3e-2}
CASES = small_cases()


@pytest.mark.parametrize("tail", [True, False], ids=["tail", "levels"])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("name,hier", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("B", [1, 3, 64])
def test_fmg_matches_oracle(prec, name, hier, B, tail):
    """FMG with the LDS tail (the coarse levels' nested iteration in one
    launch) and with per-level sweeps only."""
    import torch
    J = hier.nlevels
    flat = C.random_params(J, 2, 2, 2, seed=60 + B, spread=0.2)
    f = C.rng(6, 1, B).standard_normal((hier.sizes[0], B))
    want = KR.fmg(oracle_levels(hier), oracle_params(flat, J, 2), f)
    ctx = ctx_for(hier, flat, 2, B, prec, tail=tail)
    u = ctx.empty()
    u.fill_(float("nan"))             # the input value of u must not be used
    ctx.fmg(to_dev(f, ctx.cycle_dtype), u)
    err = elem_rel(to_np(u), want)
    print(f"fmg {name} {prec} B={B} tail={tail}: rel {err:.2e}", flush=True)
    assert err <= TOL[prec]


@pytest.mark.parametrize("precond", ["vcycle", "fmg", "none"])
@pytest.mark.parametrize("name,hier", CASES, ids=[c[0] for c in CASES])
def test_fgmres_fixed_iterations_match_oracle(precond, name, hier):
    """rtol = 0: exactly max_iter iterations with restarts every 4; the FP64
    iterate after 3 and after 7 iterations against the oracle's."""
    import torch
    J = hier.nlevels
    B = 3
    flat = C.random_params(J, 2, 2, 2, seed=70, spread=0.2)
    f = C.rng(6, 2, 0).standard_normal((hier.sizes[0], B))
    lv, prm = oracle_levels(hier), oracle_params(flat, J, 2)
    ctx = ctx_for(hier, flat, 2, B, "fp64")
    for k in (3, 7):
        want, it, _, _ = KR.fgmres(lv, prm, f, restart=4, rtol=0.0, max_iter=k, precond=precond)
        x = torch.zeros((hier.sizes[0], B), dtype=torch.float64, device="cuda")
        info = ctx.fgmres(to_dev(f, torch.float64), x, restart=4, max_iter=k, rtol=0.0, precond=precond)
        err = elem_rel(to_np(x), want)
        print(f"fgmres {precond} {name} k={k}: rel {err:.2e} iters {info.iters}", flush=True)
        assert list(info.iters) == list(it) == [k] * B
        assert info.code == 5 and np.all(info.status == 5)
        assert err <= 1e-9


@pytest.mark.parametrize("B", [100, 256])
def test_fgmres_wide_batches_match_oracle(B):
    """More than 64 columns (two and four lanes per work-item in the cycle
    sweeps, 128 / 256 lanes per row in the Krylov sweeps): the FP64 iterate
    after 6 iterations (restarts every 4) against the oracle's, on sampled
    columns, and every column's iteration count."""
    import torch
    name, hier = CASES[0]
    J = hier.nlevels
    flat = C.random_params(J, 2, 2, 2, seed=74, spread=0.2)
    f = C.rng(6, 6, B).standard_normal((hier.sizes[0], B))
    cols = [0, 1, B // 2, B - 1]
    want, it, _, _ = KR.fgmres(oracle_levels(hier), oracle_params(flat, J, 2), np.ascontiguousarray(f[:, cols]),
                               restart=4, rtol=0.0, max_iter=6, precond="vcycle")
    ctx = ctx_for(hier, flat, 2, B, "fp64")
    x = torch.zeros((hier.sizes[0], B), dtype=torch.float64, device="cuda")
    info = ctx.fgmres(to_dev(f, torch.float64), x, restart=4, max_iter=6, rtol=0.0, precond="vcycle")
    err = elem_rel(to_np(x)[:, cols], want)
    print(f"fgmres B={B}: rel {err:.2e}", flush=True)
    assert np.all(info.iters == 6) and err <= 1e-9


@pytest.mark.parametrize("reorth", [0.0, 1.0])
def test_fgmres_reorthogonalisation_policies_match_oracle(reorth):
    """Classical Gram-Schmidt without (0) and always with (1) the second pass
    give the oracle's (modified Gram-Schmidt) iterate after 7 iterations."""
    import torch
    name, hier = CASES[1]
    J = hier.nlevels
    B = 3
    flat = C.random_params(J, 2, 2, 2, seed=70, spread=0.2)
    f = C.rng(6, 2, 0).standard_normal((hier.sizes[0], B))
    want, it, _, _ = KR.fgmres(oracle_levels(hier), oracle_params(flat, J, 2), f, restart=4, rtol=0.0, max_iter=7,
                               precond="vcycle")
    ctx = ctx_for(hier, flat, 2, B, "fp64")
    x = torch.zeros((hier.sizes[0], B), dtype=torch.float64, device="cuda")
    info = ctx.fgmres(to_dev(f, torch.float64), x, restart=4, max_iter=7, rtol=0.0, precond="vcycle", reorth=reorth)
    err = elem_rel(to_np(x), want)
    print(f"fgmres reorth={reorth}: rel {err:.2e}", flush=True)
    assert list(info.iters) == [7] * B
    assert err <= 1e-9


@pytest.mark.parametrize("restart,k", [(40, 45), (63, 63)])
def test_fgmres_long_restart_matches_oracle(restart, k):
    """More than 32 basis vectors (separate second-pass dot sweep) and the
    largest restart: the FP64 iterate after k iterations against the oracle."""
    import torch
    name, hier = CASES[1]
    J = hier.nlevels
    B = 2
    flat = C.random_params(J, 2, 2, 2, seed=73, spread=0.2)
    f = C.rng(6, 5, 0).standard_normal((hier.sizes[0], B))
    want, it, _, _ = KR.fgmres(oracle_levels(hier), oracle_params(flat, J, 2), f, restart=restart, rtol=0.0,
                               max_iter=k, precond="none")
    ctx = ctx_for(hier, flat, 2, B, "fp64")
    x = torch.zeros((hier.sizes[0], B), dtype=torch.float64, device="cuda")
    info = ctx.fgmres(to_dev(f, torch.float64), x, restart=restart, max_iter=k, rtol=0.0, precond="none")
    err = elem_rel(to_np(x), want)
    print(f"fgmres none m={restart} k={k}: rel {err:.2e}", flush=True)
    assert list(info.iters) == list(it) == [k] * B
    assert err <= 1e-9


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("precond", ["vcycle", "fmg"])
def test_fgmres_converges_like_oracle(prec, precond):
    """Converged solves to 1e-10: true FP64 residual on the host, iteration
    counts against the FP64 oracle (equal in FP64; FP32 preconditioning may
    cost an iteration or two)."""
    import torch
    name, hier = CASES[1]
    J = hier.nlevels
    B = 4
    flat = C.random_params(J, 2, 2, 2, seed=71, spread=0.2)
    f = C.rng(6, 3, 0).standard_normal((hier.sizes[0], B))
    f[:, 2] = 0.0                          # a zero column stays zero, with no iterations
    _, it, _, _ = KR.fgmres(oracle_levels(hier), oracle_params(flat, J, 2), f, restart=10, rtol=1e-10,
                            max_iter=200, precond=precond)
    ctx = ctx_for(hier, flat, 2, B, prec)
    x = torch.zeros((hier.sizes[0], B), dtype=torch.float64, device="cuda")
    info = ctx.fgmres(to_dev(f, torch.float64), x, restart=10, max_iter=200, rtol=1e-10, precond=precond)
    xs = to_np(x)
    rr = np.linalg.norm(f - hier.A[0] @ xs, axis=0) / np.maximum(np.linalg.norm(f, axis=0), 1e-300)
    print(f"fgmres {prec} {precond}: gpu iters {info.iters} oracle {it} relres {rr}", flush=True)
    assert info.code == 0 and np.all(info.status == 0)
    assert np.all(rr <= 1e-10 * (1 + 1e-6))
    assert np.all(xs[:, 2] == 0.0) and info.iters[2] == 0 and it[2] == 0
    slack = 0 if prec == "fp64" else 2
    assert np.all(np.abs(info.iters - it) <= slack)
    # the FP64 residual of a converged iterate carries cancellation error of
    # about eps * ||A|| ||x|| / ||f||, so the two norms agree to a few digits
    assert np.allclose(info.relres, rr, rtol=1e-3, atol=1e-15)


def test_fgmres_caller_workspace_and_restart_growth():
    """Caller-supplied workspace gives the same result as the library's own;
    a larger restart after a smaller one regrows the library's buffer."""
    import torch
    name, hier = CASES[0]
    J = hier.nlevels
    flat = C.random_params(J, 2, 2, 2, seed=72, spread=0.2)
    f = C.rng(6, 4, 0).standard_normal((hier.sizes[0], 2))
    ctx = ctx_for(hier, flat, 2, 2, "fp32")
    fd = to_dev(f, torch.float64)
    xs = []
    for restart, own in ((3, False), (12, False), (12, True)):
        work = None
        if own:
            work = torch.empty(ctx.fgmres_workspace_bytes(restart), dtype=torch.uint8, device="cuda")
        x = torch.zeros_like(fd)
        info = ctx.fgmres(fd, x, restart=restart, max_iter=100, rtol=1e-9, work=work)
        assert info.code == 0
        xs.append(to_np(x))
    assert np.array_equal(xs[1], xs[2])
    assert elem_rel(xs[0], xs[1]) <= 1e-7
    with pytest.raises(Exception):
        ctx.fgmres(fd, torch.zeros_like(fd), restart=12,
                   work=torch.empty(16, dtype=torch.uint8, device="cuda"))


def test_fgmres_benchmark_configuration():
    """513 x 513, 64 rhs, log10 a ~ U(-3, 3), FP32 cycles with the shipped
    trained parameters: FGMRES(30) with the learnable V-cycle reaches 1e-8
    (host FP64 residual) in far fewer preconditioner calls than the
    stationary iteration needs cycles; FMG against the oracle on two columns."""
    import torch
    from paper_2608_29082_amd import params as PR
    w = C.diffusion_513(B=64)
    h = w.hier
    J = h.nlevels
    theta, meta = PR.load(PR.default_file("diffusion-513", 3))
    flat = PR.map_levels(theta, meta["J"], J, 3, 3, 3)
    ctx = ctx_for(h, flat, 3, 64, "fp32")
    f = to_dev(w.f, torch.float64)
    x = torch.zeros_like(f)
    info = ctx.fgmres(f, x, restart=30, max_iter=400, rtol=1e-8, precond="vcycle")
    xs = to_np(x)
    rr = np.linalg.norm(w.f - h.A[0] @ xs, axis=0) / np.linalg.norm(w.f, axis=0)
    print(f"513 fgmres: iters {info.iters.min()}..{info.iters.max()} relres max {rr.max():.2e}", flush=True)
    assert info.code == 0 and rr.max() <= 1e-8 * (1 + 1e-6)
    assert info.iters.max() < 200
    # FMG on the benchmark hierarchy, two columns, against the oracle: exact
    # in FP64; in FP32 the bound comes from the oracle's float32 emulation of
    # the same FMG (oracle/mixed.py): an FP32 execution whose operation order
    # differs from the emulation's lands within a few times the emulation's
    # own distance from the FP64 result
    f2 = np.ascontiguousarray(w.f[:, :2])
    lv = oracle_levels(h)
    prm = oracle_params(flat, J, 3)
    want = KR.fmg(lv, prm, f2)
    emu = MX.fmg32(MX.make_levels32(lv), prm, f2.astype(np.float32))
    err_emu = elem_rel(emu.astype(np.float64), want)
    ctx64 = ctx_for(h, flat, 3, 2, "fp64")
    u64 = ctx64.empty()
    ctx64.fmg(to_dev(f2, torch.float64), u64)
    err64 = elem_rel(to_np(u64), want)
    ctx2 = ctx_for(h, flat, 3, 2, "fp32")
    u = ctx2.empty()
    ctx2.fmg(to_dev(f2, torch.float32), u)
    err = elem_rel(to_np(u), want)
    print(f"513 fmg fp64 rel {err64:.2e}, fp32 rel {err:.2e} (float32 emulation {err_emu:.2e})", flush=True)
    assert err64 <= 1e-12
    assert 0.0 < err_emu and err <= 4.0 * err_emu

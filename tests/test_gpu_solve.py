"""GPU solver (refinement loop) against the oracle: iteration counts on the FP64
path, final relative residual <= 1e-8 recomputed by the oracle in FP64 on the
mixed paths, divergence and non-convergence reporting, column invariance."""
import numpy as np
import pytest

from mginputs import configs as C, hierarchy as H
from oracle import lmg as O
from tests.gpu_util import ctx_for, oracle_levels, oracle_params, elem_rel, to_dev, to_np

pytestmark = pytest.mark.gpu


def _solve(w, precision, B=None, params=None, **kw):
    import torch
    B = B or w.B
    flat = w.params if params is None else params
    ctx = ctx_for(w.hier, flat, (w.KB, w.KR, w.KP), B, precision, **kw)
    f = to_dev(w.f[:, :B], torch.float64)
    u = torch.zeros_like(f)
    info = ctx.solve(f, u)
    return info, to_np(u)


def test_poisson33_fp64_iterations_match_oracle():
    w = C.poisson_unit()
    info, u = _solve(w, "fp64")
    ref = O.solve(oracle_levels(w.hier), oracle_params(w.params, w.hier.nlevels, 2), w.f, rtol=1e-8)
    assert info.code == 0
    assert info.iters[0] == ref.iters[0]
    assert elem_rel(u, ref.u) <= 1e-10
    relres = np.linalg.norm(w.f - w.hier.A[0] @ u) / np.linalg.norm(w.f)
    assert relres <= 1e-8 and abs(relres - info.relres[0]) <= 1e-12


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_mixed_precision_reaches_1e8(precision):
    w = C.block_diffusion(2, 129, -2, 2, B=8, K=3)
    info, u = _solve(w, precision, max_outer=4000)
    relres = np.linalg.norm(w.f - w.hier.A[0] @ u, axis=0) / np.linalg.norm(w.f, axis=0)
    print(precision, info.iters, relres, flush=True)
    assert info.code == 0 and np.all(info.status == 0)
    assert np.all(relres <= 1e-8)
    ref = O.solve(oracle_levels(w.hier), oracle_params(w.params, w.hier.nlevels, 3), w.f[:, :2], rtol=1e-12)
    err = np.linalg.norm(u[:, :2] - ref.u, axis=0) / np.linalg.norm(ref.u, axis=0)
    # a posteriori bound for the SPD operator: ||u - u*|| <= ||A^{-1}||_2 ||f - A u|| = ||r|| / lambda_min,
    # plus the reference's own residual (rtol 1e-12) the same way
    from scipy.sparse.linalg import eigsh
    A = w.hier.A[0].tocsc()
    lam_min = float(eigsh(A, k=1, sigma=0.0, which="LM", return_eigenvectors=False)[0])
    r_gpu = np.linalg.norm(w.f[:, :2] - A @ u[:, :2], axis=0)
    r_ref = np.linalg.norm(w.f[:, :2] - A @ ref.u, axis=0)
    bound = (r_gpu + r_ref) / lam_min / np.linalg.norm(ref.u, axis=0)
    print("forward error vs FP64 oracle solution", err, "bound", bound, flush=True)
    assert np.all(err <= bound * (1 + 1e-6)) and np.all(bound < 1e-3)


def test_mixed_lshape_reaches_1e8():
    w = C.lshape_aniso(refinements=2, target_nodes=300)
    info, u = _solve(w, "fp32", max_outer=4000)
    relres = np.linalg.norm(w.f - w.hier.A[0] @ u) / np.linalg.norm(w.f)
    print("lshape", info.iters, relres, flush=True)
    assert info.code == 0 and relres <= 1e-8


def test_solve_columns_invariant_alone_and_in_batch():
    w = C.block_diffusion(2, 65, -2, 2, B=6, K=2)
    info_all, u_all = _solve(w, "fp32", B=6)
    import torch
    for b in (0, 3, 5):
        ctx = ctx_for(w.hier, w.params, 2, 1, "fp32")
        f = to_dev(w.f[:, b:b + 1], torch.float64)
        u = torch.zeros_like(f)
        info = ctx.solve(f, u)
        assert info.iters[0] == info_all.iters[b]
        assert np.array_equal(to_np(u)[:, 0], u_all[:, b])


def test_divergence_and_cap_are_reported():
    w = C.block_diffusion(2, 65, -1, 1, B=2, K=1)
    J = w.hier.nlevels
    bad = C.identity_params(J, 1, 1, 1).reshape(J - 1, -1)
    bad[:, 1] = 10.0           # eta = 10 makes the smoother unstable
    info, _ = _solve(w, "fp64", params=bad.ravel(), max_outer=500)
    assert info.code == 6 and np.all(info.status == 6)
    info, _ = _solve(w, "fp64", max_outer=1)
    assert info.code == 5 and np.all(info.iters == 1)


def test_zero_rhs_converges_immediately():
    import torch
    w = C.poisson_unit()
    ctx = ctx_for(w.hier, w.params, 2, 2)
    f = torch.zeros((w.hier.sizes[0], 2), dtype=torch.float64, device="cuda")
    u = torch.zeros_like(f)
    info = ctx.solve(f, u)
    assert info.code == 0 and np.all(info.iters == 0)


@pytest.mark.parametrize("precision,B,max_outer", [("fp32", 64, 4000), ("fp32", 64, 7), ("bf16", 48, 4000),
                                                   ("fp64", 32, 4000)])
def test_column_compaction_changes_nothing(precision, B, max_outer):
    """mg_solve narrows the cycle to the columns still iterating at its periodic
    checks (rounded up to 16) and fuses the update into the next FP64 residual
    sweep, alternating the iterate between the caller's u and a scratch vector.
    Against the same solve without compaction: the same iteration counts,
    statuses and residuals, and every element of u the same bits.  A third of
    the columns have f = 0 (stopped at the first check: compaction at once);
    the others are spread by scaling; max_outer = 7 ends at the cap with
    columns still iterating (odd update count: the iterate is copied back)."""
    import torch
    w = C.block_diffusion(2, 129, -2, 2, B=B, K=3)
    f = w.f.copy()
    f[:, : B // 3] = 0.0
    f[:, B // 3:] *= np.linspace(1e-3, 1e3, B - B // 3)[None, :]
    out = []
    for compact in (True, False):
        ctx = ctx_for(w.hier, w.params, 3, B, precision, max_outer=max_outer, check_every=3, compact=compact)
        fd = to_dev(f, torch.float64)
        u = torch.zeros_like(fd)
        info = ctx.solve(fd, u)
        out.append((info, to_np(u)))
        ctx.close()
    (i1, u1), (i2, u2) = out
    print(f"{precision} B={B} cap={max_outer}: code {i1.code}/{i2.code}, iters {sorted(set(i1.iters.tolist()))}",
          flush=True)
    assert i1.code == i2.code
    assert np.array_equal(i1.iters, i2.iters) and np.array_equal(i1.status, i2.status)
    assert np.array_equal(i1.relres, i2.relres)
    assert np.array_equal(u1, u2)
    assert np.all(u1[:, : B // 3] == 0.0)
    if max_outer > 100:
        assert i1.code == 0
        relres = np.linalg.norm(f[:, B // 3:] - w.hier.A[0] @ u1[:, B // 3:], axis=0) / np.linalg.norm(
            f[:, B // 3:], axis=0)
        assert np.all(relres <= 1e-8)
    else:
        assert i1.code == 5 and np.all(i1.iters[B // 3:] == max_outer)

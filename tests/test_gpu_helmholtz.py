"""Parity of the complex Helmholtz path (two features per node, Jacobi and
GMRES smoothing, FMG, complex FGMRES) through the C ABI against the
complex128 oracle."""
import numpy as np
import pytest

from mginputs import configs as C
from mginputs import helmholtz as HZ
from oracle import helmholtz as OH
from tests.gpu_util import elem_rel, to_np

pytestmark = pytest.mark.gpu


def dev(x, dtype):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def cdt(prec):
    import torch
    return torch.complex128 if prec == "fp64" else torch.complex64


def case(side, k, J, B, seed=0, plan=None, v=4):
    h = HZ.hierarchy(side, k, J)
    plan = plan or HZ.smoother_plan(h)
    f = HZ.load_vectors(side, HZ.source_centres(B, C.rng(10, 2, seed)))
    return h, plan, f


def ctx(h, plan, flat, K, B, prec, v=4):
    from paper_2608_29082_amd import helmholtz as HB
    KB, KR, KP = K
    return HB.HelmholtzContext(h.A, h.P, flat, KB, KR, KP, plan, v=v, precision=prec, nrhs=B)


CYCLE_CASES = [
    # (side, k, J, B, K orders, plan override, v)
    (33, 12.0, 4, 3, (1, 1, 1), None, 4),                   # Jacobi, GMRES, GMRES; ragged B
    (33, 12.0, 4, 16, (2, 1, 0), None, 4),                  # mixed orders, K = 0 transfers
    (65, 20.0, 5, 5, (1, 2, 1), None, 3),                   # four GMRES levels, v = 3
    (17, 40.0, 3, 2, (1, 1, 1), None, 4),                   # GMRES on the finest level
    (17, 5.0, 2, 1, (0, 0, 0), [("jacobi", 2, 1)], 4),      # two-grid, plain Jacobi, B = 1
    (33, 12.0, 3, 4, (3, 1, 1), [("gmres", 1, 0), ("jacobi", 0, 2)], 1),   # v = 1, nu = 0 sides
    (65, 40.0, 4, 3, (1, 1, 1), None, 4),                   # GMRES on a 65 x 65 finest level: scratch in HBM
]


@pytest.mark.parametrize("ci", range(len(CYCLE_CASES)))
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_cycle_matches_oracle(ci, prec):
    side, k, J, B, K, plan, v = CYCLE_CASES[ci]
    h, plan, f = case(side, k, J, B, seed=ci, plan=plan)
    flat = C.hz_random_params(J, *K, plan, seed=ci + 1)
    g = C.rng(10, 9, ci)
    u0 = 0.01 * (g.standard_normal(f.shape) + 1j * g.standard_normal(f.shape))
    prm = OH.unpack(flat, J, *K, plan, v)
    want = OH.lmg(OH.make_levels(h.A, h.P, h.R), prm, 0, f, u0)
    c = ctx(h, plan, flat, K, B, prec, v)
    u = dev(u0, cdt(prec))
    c.vcycle(dev(f, cdt(prec)), u)
    got = u.cpu().numpy().astype(np.complex128)
    err = elem_rel(got, want)
    print(f"case {ci} {prec}: rel {err:.2e}", flush=True)
    assert err <= (1e-11 if prec == "fp64" else 5e-5)
    # a second cycle from the first one's output (buffers reused, state cleared)
    want2 = OH.lmg(OH.make_levels(h.A, h.P, h.R), prm, 0, f, want)
    c.vcycle(dev(f, cdt(prec)), u)
    err2 = elem_rel(u.cpu().numpy().astype(np.complex128), want2)
    assert err2 <= (1e-11 if prec == "fp64" else 1e-4)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fmg_matches_oracle(prec):
    h, plan, f = case(65, 20.0, 5, 6, seed=3)
    K = (1, 1, 1)
    flat = C.hz_random_params(5, *K, plan, seed=7)
    want = OH.fmg(OH.make_levels(h.A, h.P, h.R), OH.unpack(flat, 5, *K, plan), f)
    c = ctx(h, plan, flat, K, 6, prec)
    u = c.empty()
    c.fmg(dev(f, cdt(prec)), u)
    err = elem_rel(u.cpu().numpy().astype(np.complex128), want)
    print(f"fmg {prec}: rel {err:.2e}", flush=True)
    assert err <= (1e-11 if prec == "fp64" else 5e-5)


def test_residual_and_norms():
    import torch
    h, plan, f = case(33, 12.0, 4, 5, seed=4)
    c = ctx(h, plan, C.hz_identity_params(4, 1, 1, 1, plan), (1, 1, 1), 5, "fp32")
    g = C.rng(10, 9, 77)
    u = g.standard_normal(f.shape) + 1j * g.standard_normal(f.shape)
    r, nr = c.residual(dev(f, torch.complex128), dev(u, torch.complex128))
    want = f - h.A[0] @ u
    assert elem_rel(r.cpu().numpy(), want) <= 1e-14
    assert np.allclose(nr.cpu().numpy(), np.linalg.norm(want, axis=0), rtol=1e-13, atol=0)


@pytest.mark.parametrize("precond", ["vcycle", "fmg", "none"])
def test_fgmres_fp64_matches_oracle(precond):
    """FP64 cycles: the same iteration count per column (+-1 at the stopping
    threshold) and a solution within the FGMRES tolerance of the oracle's."""
    import torch
    if precond == "none":        # unpreconditioned: a small system, restart >= n
        h, plan, f = case(9, 8.0, 2, 3, seed=5)
        J, m, mi = 2, 63, 81
    else:
        h, plan, f = case(33, 12.0, 4, 3, seed=5)
        J, m, mi = 4, 30, 60
    K = (1, 1, 1)
    flat = C.hz_random_params(J, *K, plan, seed=8, spread=0.05)
    lev = OH.make_levels(h.A, h.P, h.R)
    x_o, it_o, rr_o, _ = OH.fgmres(lev, OH.unpack(flat, J, *K, plan), f, restart=m, rtol=1e-8, max_iter=mi,
                                   precond=precond)
    c = ctx(h, plan, flat, K, 3, "fp64")
    x = torch.zeros(f.shape, dtype=torch.complex128, device="cuda")
    info = c.fgmres(dev(f, torch.complex128), x, restart=m, max_iter=mi, rtol=1e-8, precond=precond,
                    reorth=1.0)
    print(f"{precond}: gpu iters {info.iters} oracle {it_o}; relres {info.relres}", flush=True)
    assert info.code == 0 and (info.relres <= 1e-8).all()
    assert (np.abs(info.iters - it_o) <= 1).all()
    xs = x.cpu().numpy()
    assert np.linalg.norm(f - h.A[0] @ xs) / np.linalg.norm(f) <= 1.01e-8 * np.sqrt(3)
    assert elem_rel(xs, x_o) <= 1e-5


def test_fgmres_fp32_cycles_converge_and_report():
    import torch
    h, plan, f = case(65, 20.0, 5, 16, seed=6)
    K = (1, 1, 1)
    flat = C.hz_identity_params(5, *K, plan)
    c = ctx(h, plan, flat, K, 16, "fp32")
    for pc in ("vcycle", "fmg"):
        x = torch.zeros(f.shape, dtype=torch.complex128, device="cuda")
        info = c.fgmres(dev(f, torch.complex128), x, restart=40, max_iter=200, rtol=1e-8, precond=pc)
        rr = np.linalg.norm(f - h.A[0] @ x.cpu().numpy(), axis=0) / np.linalg.norm(f, axis=0)
        print(f"fp32 {pc}: iters {info.iters.min()}..{info.iters.max()}, relres max {rr.max():.2e}", flush=True)
        assert info.code == 0 and rr.max() <= 1.01e-8
        assert np.allclose(info.relres, rr, rtol=1e-6, atol=1e-15)


def test_fgmres_zero_rhs_and_iteration_cap():
    """A zero column is solved at once; a cap below the needed count returns
    MG_ERR_NOT_CONVERGED with the cap as the column's iteration count."""
    import torch
    h, plan, f = case(33, 12.0, 4, 3, seed=7)
    f[:, 1] = 0.0
    c = ctx(h, plan, C.hz_identity_params(4, 1, 1, 1, plan), (1, 1, 1), 3, "fp64")
    x = torch.zeros(f.shape, dtype=torch.complex128, device="cuda")
    info = c.fgmres(dev(f, torch.complex128), x, restart=4, max_iter=3, rtol=1e-8, precond="vcycle")
    assert info.code == 5
    assert info.iters[1] == 0 and info.status[1] == 0 and info.relres[1] == 0.0
    assert info.iters[0] == 3 and info.status[0] == 5
    assert np.abs(x.cpu().numpy()[:, 1]).max() == 0.0


def test_bench_configuration_cycle_and_fmg_solve():
    """The benchmark's configuration (k = 16 pi, 257 x 257, 5 levels, Jacobi on
    k h <= 1/2 and GMRES(4) above, 16 sources, FP32 cycles): one cycle from
    zero against the oracle on whole vectors (2 columns), and the FGMRES-FMG
    solve reaching 1e-8 on all 16."""
    import torch
    w = C.helmholtz(B=16)
    h = w.hier
    want = OH.lmg(OH.make_levels(h.A, h.P, h.R), OH.unpack(w.params, 5, 1, 1, 1, w.plan), 0, w.f[:, :2],
                  np.zeros((h.sizes[0], 2), complex))
    c = ctx(h, w.plan, w.params, (1, 1, 1), 16, "fp32")
    u = torch.zeros(w.f.shape, dtype=torch.complex64, device="cuda")
    c.vcycle(dev(w.f, torch.complex64), u)
    err = elem_rel(u.cpu().numpy()[:, :2].astype(np.complex128), want)
    print(f"bench-config fp32 cycle rel {err:.2e}", flush=True)
    assert err <= 5e-5
    x = torch.zeros(w.f.shape, dtype=torch.complex128, device="cuda")
    info = c.fgmres(dev(w.f, torch.complex128), x, restart=40, max_iter=200, rtol=1e-8, precond="fmg")
    rr = np.linalg.norm(w.f - h.A[0] @ x.cpu().numpy(), axis=0) / np.linalg.norm(w.f, axis=0)
    print(f"bench-config fgmres-fmg iters {info.iters.min()}..{info.iters.max()} relres {rr.max():.2e}", flush=True)
    assert info.code == 0 and rr.max() <= 1.01e-8


@pytest.mark.parametrize("B", [64, 256])
def test_cycle_wide_batches(B):
    """64 and the maximum 256 right-hand sides (lane groups of a whole
    wavefront and of a whole work-group per row)."""
    h, plan, f = case(17, 20.0, 3, B, seed=11)
    K = (1, 1, 1)
    flat = C.hz_random_params(3, *K, plan, seed=12)
    want = OH.lmg(OH.make_levels(h.A, h.P, h.R), OH.unpack(flat, 3, *K, plan), 0, f, np.zeros_like(f))
    c = ctx(h, plan, flat, K, B, "fp64")
    u = c.empty()
    u.zero_()
    c.vcycle(dev(f, cdt("fp64")), u)
    assert elem_rel(u.cpu().numpy(), want) <= 1e-11


def test_set_params_and_explicit_restriction():
    """mgh_set_params replaces the weights (same plan); an explicit R = 0.5 P^T
    is used as given."""
    from paper_2608_29082_amd import helmholtz as HB
    h, plan, f = case(33, 12.0, 4, 3, seed=13)
    K = (2, 1, 1)
    p1 = C.hz_random_params(4, *K, plan, seed=14)
    p2 = C.hz_random_params(4, *K, plan, seed=15)
    R = [0.5 * r for r in h.R]
    c = HB.HelmholtzContext(h.A, h.P, p1, *K, plan, precision="fp64", nrhs=3, R=R)
    lev = OH.make_levels(h.A, h.P, R)
    for p in (p1, p2):
        c.set_params(p)
        u = c.empty()
        u.zero_()
        c.vcycle(dev(f, cdt("fp64")), u)
        want = OH.lmg(lev, OH.unpack(p, 4, *K, plan), 0, f, np.zeros_like(f))
        assert elem_rel(u.cpu().numpy(), want) <= 1e-11


def test_fgmres_is_deterministic():
    """Block partial sums are reduced in a fixed order: two solves of the same
    system give bitwise equal iterates and iteration counts."""
    import torch
    h, plan, f = case(65, 20.0, 5, 8, seed=16)
    c = ctx(h, plan, C.hz_identity_params(5, 1, 1, 1, plan), (1, 1, 1), 8, "fp32")
    xs, its = [], []
    for _ in range(2):
        x = torch.zeros(f.shape, dtype=torch.complex128, device="cuda")
        info = c.fgmres(dev(f, torch.complex128), x, restart=20, max_iter=120, rtol=1e-8, precond="fmg")
        xs.append(x.cpu().numpy())
        its.append(info.iters.copy())
    assert np.array_equal(xs[0], xs[1]) and np.array_equal(its[0], its[1])


def test_training_loss_matches_oracle_and_descends():
    """The Helmholtz training loss evaluated through the library (m FP64
    cycles from zero) equals the oracle's, and steps against the sign of its
    central-difference gradient reduce it."""
    from paper_2608_29082_amd import train_helmholtz as TH
    w = C.helmholtz(33, 12.0, 4, B=2)
    f = HZ.load_vectors(33, HZ.source_centres(5, C.rng(10, 2, 1))[2:])
    loss = TH.Loss(w, f, 4)
    p = C.hz_random_params(4, 1, 1, 1, w.plan, seed=20, spread=0.05)
    L = loss(p)
    lev = OH.make_levels(w.hier.A, w.hier.P, w.hier.R)
    prm = OH.unpack(p, 4, 1, 1, 1, w.plan)
    u = np.zeros_like(f)
    for _ in range(4):
        u = OH.lmg(lev, prm, 0, f, u)
    Lo = float(np.mean(np.linalg.norm(f - w.hier.A[0] @ u, axis=0) ** 2 / np.linalg.norm(f, axis=0) ** 2))
    print(f"training loss gpu {L:.6e} oracle {Lo:.6e}", flush=True)
    assert abs(L - Lo) <= 1e-9 * Lo
    q = p.copy()
    for _ in range(3):
        g = loss.grad(q, 1e-6)
        q = q - 0.005 * np.sign(g)
    assert loss(q) < L


def test_overlapping_f_and_u_are_rejected():
    """mgh_vcycle and mgh_fmg reject f and u that share memory (the cycle
    reads f after it started writing u) with MG_ERR_INVALID_ARG."""
    from paper_2608_29082_amd import binding as Bd
    h, plan, f = case(17, 5.0, 2, 2, seed=21, plan=[("jacobi", 1, 1)])
    c = ctx(h, plan, C.hz_identity_params(2, 1, 1, 1, plan), (1, 1, 1), 2, "fp64")
    x = dev(f, cdt("fp64"))
    for call in (c.vcycle, c.fmg):
        with pytest.raises(Bd.MGError) as e:
            call(x, x)
        assert e.value.status == 1


@pytest.mark.parametrize("side,k,J", [(33, 12.0, 4), (65, 20.0, 5)])
def test_stationary_solve_matches_oracle(side, k, J):
    """mgh_solve: per column the oracle's cycle count to 1e-8 (+-1 at the
    threshold) and the oracle's iterate at that count; a column keeps its
    first converged iterate."""
    import torch
    h, plan, f = case(side, k, J, 3, seed=5)
    flat = C.hz_random_params(J, 1, 1, 1, plan, seed=30, spread=0.03)
    lev = OH.make_levels(h.A, h.P, h.R)
    prm = OH.unpack(flat, J, 1, 1, 1, plan)
    fn = np.linalg.norm(f, axis=0)
    u = np.zeros_like(f)
    its, iterates = [None] * 3, [None] * 3
    for cyc in range(1, 300):
        u = OH.lmg(lev, prm, 0, f, u)
        rr = np.linalg.norm(f - h.A[0] @ u, axis=0) / fn
        for b in range(3):
            if its[b] is None and rr[b] <= 1e-8:
                its[b], iterates[b] = cyc, u[:, b].copy()
        if all(i is not None for i in its):
            break
    c = ctx(h, plan, flat, (1, 1, 1), 3, "fp64")
    x = torch.zeros(f.shape, dtype=torch.complex128, device="cuda")
    info = c.solve(dev(f, torch.complex128), x, rtol=1e-8, max_cycles=300, check_every=3)
    print(f"stationary: gpu {info.iters} oracle {its}", flush=True)
    assert info.code == 0 and (info.relres <= 1e-8).all()
    assert (np.abs(info.iters - np.array(its)) <= 1).all()
    xs = x.cpu().numpy()
    for b in range(3):
        if info.iters[b] == its[b]:
            assert elem_rel(xs[:, b], iterates[b]) <= 1e-9


def test_stationary_solve_cap_and_precision():
    """The cycle cap gives MG_ERR_NOT_CONVERGED with the cap as every column's
    count; an FP32 context refuses the stationary solve (MG_ERR_UNSUPPORTED)."""
    import torch
    from paper_2608_29082_amd import binding as Bd
    h, plan, f = case(33, 12.0, 4, 2, seed=6)
    c = ctx(h, plan, C.hz_identity_params(4, 1, 1, 1, plan), (1, 1, 1), 2, "fp64")
    x = torch.zeros(f.shape, dtype=torch.complex128, device="cuda")
    info = c.solve(dev(f, torch.complex128), x, rtol=1e-8, max_cycles=4, check_every=2)
    assert info.code == 5 and list(info.iters) == [4, 4] and list(info.status) == [5, 5]
    c32 = ctx(h, plan, C.hz_identity_params(4, 1, 1, 1, plan), (1, 1, 1), 2, "fp32")
    with pytest.raises(Bd.MGError) as e:
        c32.solve(dev(f, torch.complex128), x)
    assert e.value.status == 8


@pytest.mark.parametrize("K", [1, 2])
def test_bench_configuration_trained_parameters_fp64_cycle(K):
    """The shipped trained parameters (K = 1 and K = 2) on the benchmark
    hierarchy: one FP64 cycle from zero against the oracle (2 columns, whole
    vectors)."""
    import torch
    import os
    w = C.helmholtz(B=2, K=K)
    h = w.hier
    theta = np.load(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                                 "paper_2608_29082_amd", "theta", f"hz_k{K}_helmholtz257.npy"))
    want = OH.lmg(OH.make_levels(h.A, h.P, h.R), OH.unpack(theta, 5, K, K, K, w.plan), 0, w.f,
                  np.zeros_like(w.f))
    c = ctx(h, w.plan, theta, (K, K, K), 2, "fp64")
    u = torch.zeros(w.f.shape, dtype=torch.complex128, device="cuda")
    c.vcycle(dev(w.f, torch.complex128), u)
    err = elem_rel(u.cpu().numpy(), want)
    print(f"trained fp64 cycle rel {err:.2e}", flush=True)
    assert err <= 1e-11

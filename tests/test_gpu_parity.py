"""GPU parity of the HIP V-cycle with the CPU FP64 oracle (through the C ABI).

Per-cycle tolerance on the FP64 path: relative 1e-12 in the 2-norm (the
accuracy target of the method's FP64 path).  FP32 cycles: 2e-5 (derived from
unit round-off 6e-8 times the ~100 dependent roundings of one V(2,2) cycle
with K <= 3 on <= 8 levels, with margin).  BF16 intermediates: 3e-2 (unit
round-off 3.9e-3 of the stored smoother/transfer intermediates, a few of them
in sequence per level).
"""
import numpy as np
import pytest

from mginputs import configs as C, hierarchy as H
from oracle import lmg as O
from tests.gpu_util import ctx_for, oracle_levels, oracle_params, elem_rel, small_cases, to_dev, to_np

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 2e-5, "bf16": 3e-2}


def _cycle_case(hier, K, B, seed, precision="fp64", nu=(2, 2), identity=False, R=None, G=None):
    import torch
    J = hier.nlevels
    KB, KR, KP = K if isinstance(K, tuple) else (K, K, K)
    flat = C.identity_params(J, KB, KR, KP) if identity else C.random_params(J, KB, KR, KP, seed=seed)
    g = C.rng(6, 2, seed)
    f = g.standard_normal((hier.sizes[0], B))
    u = g.standard_normal((hier.sizes[0], B))
    want = O.lmg(oracle_levels(hier, R, G), oracle_params(flat, J, K, nu), 0, f, u)
    ctx = ctx_for(hier, flat, K, B, precision, nu, R=R, G=G)
    dt = ctx.cycle_dtype
    fd, ud = to_dev(f, dt), to_dev(u, dt)
    ctx.vcycle(fd, ud)
    torch.cuda.synchronize()
    got = to_np(ud)
    return elem_rel(got, want), got, want


@pytest.mark.parametrize("case", ["poisson33", "blocks65", "lshape"])
@pytest.mark.parametrize("K", [0, 1, 2, 3])
def test_fp64_cycle_matches_oracle(case, K):
    hier = dict(small_cases())[case]
    for B in (1, 3):
        err, _, _ = _cycle_case(hier, K, B, seed=K + 10 * B)
        print(f"{case} K={K} B={B} rel={err:.2e}", flush=True)
        assert err <= TOL["fp64"]


@pytest.mark.parametrize("B", [2, 32, 64, 100, 256])
def test_fp64_cycle_batch_widths(B):
    hier = dict(small_cases())["blocks65"]
    err, got, _ = _cycle_case(hier, 3, B, seed=B)
    assert err <= TOL["fp64"]


def test_identity_theta_is_classical_vcycle_on_gpu():
    hier = dict(small_cases())["blocks65"]
    err, got, _ = _cycle_case(hier, 2, 2, seed=1, identity=True)
    assert err <= TOL["fp64"]
    g = C.rng(6, 2, 1)
    f = g.standard_normal((hier.sizes[0], 2))
    u = g.standard_normal((hier.sizes[0], 2))
    classical = O.classical_mg(oracle_levels(hier), 2 / 3, 2, 0, f, u)
    assert elem_rel(got, classical) <= TOL["fp64"]


@pytest.mark.parametrize("nu", [(0, 1), (1, 0), (3, 2), (0, 0)])
def test_fp64_smoothing_counts(nu):
    hier = dict(small_cases())["poisson33"]
    err, _, _ = _cycle_case(hier, (2, 1, 3), 3, seed=5, nu=nu)
    assert err <= TOL["fp64"]


def test_fp64_explicit_R_and_mesh_graph():
    """R given explicitly (scaled transpose, R = c P^T) and a separate graph
    (the mesh graph: "/" diagonals included although A_ij = 0 there)."""
    import scipy.sparse as sp
    hier = dict(small_cases())["blocks65"]
    R = [0.5 * r for r in hier.R]
    G = []
    for a in hier.A:
        n = a.shape[0]
        m = int(round(np.sqrt(n)))
        pat = (a != 0).astype(float).tolil()
        if m * m == n:
            for i in range(n):
                x, y = i % m, i // m
                if x + 1 < m and y + 1 < m:
                    pat[i, i + m + 1] = 1.0
                    pat[i + m + 1, i] = 1.0
        G.append(sp.csr_matrix(pat))
    err, _, _ = _cycle_case(hier, 2, 3, seed=9, R=R, G=G)
    assert err <= TOL["fp64"]


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("case", ["poisson33", "blocks65", "lshape"])
def test_reduced_precision_cycle_close_to_oracle(precision, case):
    hier = dict(small_cases())[case]
    err, _, _ = _cycle_case(hier, 3, 4, seed=3, precision=precision)
    print(f"{case} {precision} rel={err:.2e}", flush=True)
    assert err <= TOL[precision]


def test_full_size_513_sampled_cycle_fp64():
    """513 x 513 block-diffusion hierarchy (8 levels), B = 64, random Theta,
    FP64: the whole-vector relative difference of one cycle."""
    w = C.diffusion_513(B=64)
    err, got, want = _cycle_case(w.hier, 3, 64, seed=21)
    print(f"513 fp64 rel={err:.2e}", flush=True)
    # coarsest 9 x 9 operator of contrast 1e6 blocks: kappa(A_J) * eps bound
    kappa = np.linalg.cond(w.hier.A[-1].toarray())
    assert err <= max(TOL["fp64"], 50 * kappa * np.finfo(float).eps)


def test_residual_fp64_bitwise_close():
    import torch
    hier = dict(small_cases())["lshape"]
    g = C.rng(6, 3, 0)
    f = g.standard_normal((hier.sizes[0], 5))
    u = g.standard_normal((hier.sizes[0], 5))
    ctx = ctx_for(hier, C.identity_params(hier.nlevels, 1, 1, 1), 1, 5)
    r, norms = ctx.residual(to_dev(f, torch.float64), to_dev(u, torch.float64))
    want = f - hier.A[0] @ u
    assert np.abs(to_np(r) - want).max() <= 1e-13 * np.abs(want).max()
    assert np.allclose(to_np(norms), np.linalg.norm(want, axis=0), rtol=1e-13, atol=0)


def test_refine_step_equals_cycle_fp64():
    """u + LMG(A, f - A u, 0) equals LMG(A, f, u) (the cycle is affine, Sec. 1)."""
    import torch
    hier = dict(small_cases())["blocks65"]
    J = hier.nlevels
    flat = C.random_params(J, 2, 2, 2, seed=4)
    g = C.rng(6, 4, 0)
    f = g.standard_normal((hier.sizes[0], 3))
    u = g.standard_normal((hier.sizes[0], 3))
    want = O.lmg(oracle_levels(hier), oracle_params(flat, J, 2), 0, f, u)
    ctx = ctx_for(hier, flat, 2, 3)
    out = ctx.refine_step(to_dev(f, torch.float64), to_dev(u, torch.float64))
    assert elem_rel(to_np(out), want) <= 1e-11


def test_set_params_changes_cycle():
    import torch
    hier = dict(small_cases())["poisson33"]
    J = hier.nlevels
    p1 = C.random_params(J, 2, 2, 2, seed=1)
    p2 = C.random_params(J, 2, 2, 2, seed=2)
    ctx = ctx_for(hier, p1, 2, 1)
    ctx.set_params(p2)
    g = C.rng(6, 5, 0)
    f = g.standard_normal((hier.sizes[0], 1))
    u = g.standard_normal((hier.sizes[0], 1))
    ud = to_dev(u, torch.float64)
    ctx.vcycle(to_dev(f, torch.float64), ud)
    want = O.lmg(oracle_levels(hier), oracle_params(p2, J, 2), 0, f, u)
    assert elem_rel(to_np(ud), want) <= TOL["fp64"]


def test_deterministic_and_column_independent():
    """Two runs are bitwise equal; a column gives the same result alone and in a batch."""
    import torch
    hier = dict(small_cases())["blocks65"]
    J = hier.nlevels
    flat = C.random_params(J, 3, 3, 3, seed=8)
    g = C.rng(6, 6, 0)
    f = g.standard_normal((hier.sizes[0], 5))
    u = g.standard_normal((hier.sizes[0], 5))
    outs = []
    for _ in range(2):
        ctx = ctx_for(hier, flat, 3, 5, "fp32")
        ud = to_dev(u, torch.float32)
        ctx.vcycle(to_dev(f, torch.float32), ud)
        outs.append(to_np(ud))
    assert np.array_equal(outs[0], outs[1])
    ctx1 = ctx_for(hier, flat, 3, 1, "fp32")
    ud = to_dev(u[:, 2:3], torch.float32)
    ctx1.vcycle(to_dev(f[:, 2:3], torch.float32), ud)
    assert np.array_equal(to_np(ud)[:, 0], outs[0][:, 2])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_lds_coarse_tail_matches_per_level_sweeps(precision):
    """The coarse levels run as one LDS-resident kernel per column; the result
    must match the per-level sweeps (and the oracle) to the cycle tolerance."""
    import torch
    for case in ("poisson33", "blocks65"):
        hier = dict(small_cases())[case]
        J = hier.nlevels
        flat = C.random_params(J, 3, 3, 3, seed=31)
        g = C.rng(6, 8, 0)
        f = g.standard_normal((hier.sizes[0], 3))
        outs = []
        for tail in (True, False):
            ctx = ctx_for(hier, flat, 3, 3, precision, tail=tail)
            fd = to_dev(f, torch.float64)
            u = torch.zeros_like(fd)
            ctx.refine_step(fd, torch.zeros_like(fd), u)     # u = LMG(A, f, 0): tail from the finest level
            v = to_dev(np.zeros_like(f), ctx.cycle_dtype)
            ctx.vcycle(to_dev(f, ctx.cycle_dtype), v)           # tail below the finest level
            outs.append((to_np(u), to_np(v)))
        want = O.lmg(oracle_levels(hier), oracle_params(flat, J, 3), 0, f, np.zeros_like(f))
        for a, b in zip(outs[0], outs[1]):
            assert elem_rel(a, b) <= TOL[precision]
            assert elem_rel(a, want) <= TOL[precision]

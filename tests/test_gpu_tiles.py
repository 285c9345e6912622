"""GPU parity of the fused K-hop convolution over LDS tiles.

The fused kernel computes the same Horner hops as the chain of per-hop
sweeps, in the same order of operations per node and column, so with FP32
cycles its results are compared with the chain's bit for bit (contexts set
up with and without tiles, same inputs, per-level sweeps on every level);
the default configuration (coarse LDS tail below the tiled levels) and the
BF16 cycles, whose fused kernel keeps the hops in FP32, are compared with the
oracle.  Cases span
up to a thousand tiles, ragged column groups (B = 16, 48, 64), the three
aggregations in both bases, K from 2 to 4 and an unstructured mesh."""
import numpy as np
import pytest

from mginputs import configs as C, hierarchy as H
from oracle import lmg as O
from tests.gpu_util import ctx_for, elem_rel, to_dev, to_np

pytestmark = pytest.mark.gpu

TOL = {"fp32": 2e-5, "bf16": 3e-2}


def _cases():
    return [("blocks129", H.square_hierarchy(129, H.block_field(C.rng(7, 1, 1), 16, -3, 3))),
            ("blocks257", H.square_hierarchy(257, H.block_field(C.rng(7, 1, 0), 16, -2, 2))),
            ("lshape", H.lshape_hierarchy(C.rng(7, 4, 0), target_nodes=120, refinements=4))]


CASES = _cases()
IDS = [c[0] for c in CASES]


def _pair(hier, flat, K, B, prec, **kw):
    # the coarse LDS tail starts below the tiled levels, so it would start at
    # different levels in the two contexts; compare with per-level sweeps only
    on = ctx_for(hier, flat, K, B, prec, tail=False, **kw)
    off = ctx_for(hier, flat, K, B, prec, tiles=False, tail=False, **kw)
    return on, off


def _conv_launches(ctx, f, u):
    import torch
    ctx.timing_start("conv", -1)
    ctx.vcycle(f, u)
    torch.cuda.synchronize()
    n, ms, by = ctx.timing_read()
    ctx.timing_start(None)
    return n


@pytest.mark.parametrize("agg,basis", [("mean", "monomial"), ("mean", "chebyshev"), ("weighted", "monomial"),
                                       ("sym", "chebyshev")])
@pytest.mark.parametrize("K", [(3, 3, 3), (2, 2, 2), (4, 2, 3)])
@pytest.mark.parametrize("name,hier", CASES, ids=IDS)
def test_fused_conv_equals_hop_chain_fp32(agg, basis, K, name, hier):
    import torch
    J = hier.nlevels
    B = 16
    flat = C.random_params(J, *K, seed=101, spread=0.2)
    g = C.rng(6, 21, 0)
    f = g.standard_normal((hier.sizes[0], B))
    u = g.standard_normal((hier.sizes[0], B))
    on, off = _pair(hier, flat, K, B, "fp32", basis=basis, aggregation=agg)
    outs = []
    for ctx in (on, off):
        ud = to_dev(u, torch.float32)
        ctx.vcycle(to_dev(f, torch.float32), ud)
        e = ctx.refine_step(to_dev(f, torch.float64), torch.zeros((hier.sizes[0], B), dtype=torch.float64,
                                                                   device="cuda"))
        outs.append((to_np(ud), to_np(e)))
    n_on = _conv_launches(on, to_dev(f, torch.float32), to_dev(u, torch.float32))
    n_off = _conv_launches(off, to_dev(f, torch.float32), to_dev(u, torch.float32))
    d1 = float(np.abs(outs[0][0] - outs[1][0]).max())
    d2 = float(np.abs(outs[0][1] - outs[1][1]).max())
    print(f"{name} {agg}/{basis} K={K}: fused launches {n_on} (untiled {n_off}), max diff {d1:.1e} {d2:.1e}",
          flush=True)
    assert n_on > 0 and n_off == 0
    assert d1 == 0.0 and d2 == 0.0
    on.close(); off.close()


@pytest.mark.parametrize("B", [16, 48, 64])
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_fused_conv_cycle_matches_oracle(prec, B):
    import torch
    name, hier = CASES[0]
    J = hier.nlevels
    flat = C.random_params(J, 3, 3, 3, seed=102, spread=0.2)
    g = C.rng(6, 22, B)
    f = g.standard_normal((hier.sizes[0], B))
    u = g.standard_normal((hier.sizes[0], B))
    want = O.lmg(O.make_levels(hier.A, hier.P, hier.R), O.unpack(flat, J, 3, 3, 3), 0, f, u)
    ctx = ctx_for(hier, flat, 3, B, prec)
    ud = to_dev(u, torch.float32)
    ctx.vcycle(to_dev(f, torch.float32), ud)
    err = elem_rel(to_np(ud), want)
    # a refinement step from zero: the cycle from a zero iterate, with the coarse tail
    e = ctx.refine_step(to_dev(f, torch.float64), torch.zeros((hier.sizes[0], B), dtype=torch.float64, device="cuda"))
    err2 = elem_rel(to_np(e), O.lmg(O.make_levels(hier.A, hier.P, hier.R), O.unpack(flat, J, 3, 3, 3), 0, f,
                               np.zeros_like(f)))
    assert _conv_launches(ctx, to_dev(f, torch.float32), to_dev(u, torch.float32)) > 0
    print(f"{name} {prec} B={B}: cycle rel {err:.2e}, refinement step rel {err2:.2e}", flush=True)
    assert err <= TOL[prec] and err2 <= TOL[prec]
    ctx.close()


def test_fused_conv_solve_and_gradient_equal_hop_chain():
    """Stationary solve to 1e-8 (same cycle counts and iterates) and the
    reverse sweep (its forward recomputation uses the fused kernel)."""
    import torch
    from paper_2608_29082_amd import autograd as AG
    name, hier = CASES[0]
    J = hier.nlevels
    B = 16
    flat = C.random_params(J, 3, 3, 3, seed=103, spread=0.1)
    f = C.rng(6, 23, 0).standard_normal((hier.sizes[0], B))
    res = []
    for tiles in (True, False):
        ctx = ctx_for(hier, C.identity_params(J, 3, 3, 3), 3, B, "fp32", tiles=tiles, tail=False, max_outer=400)
        u = torch.zeros((hier.sizes[0], B), dtype=torch.float64, device="cuda")
        info = ctx.solve(to_dev(f, torch.float64), u)
        ctx.close()
        ctxb = ctx_for(hier, flat, 3, B, "fp32", tiles=tiles, tail=False, backward=True)
        th = torch.tensor(flat, dtype=torch.float64, requires_grad=True)
        L = AG.unrolled_loss(ctxb, th, to_dev(f, torch.float64), cycles=2)
        L.backward()
        ctxb.close()
        res.append((info.iters.copy(), to_np(u), L.item(), th.grad.numpy().copy()))
    print(f"iters {res[0][0].max()} / {res[1][0].max()}, loss {res[0][2]:.6e} / {res[1][2]:.6e}", flush=True)
    assert np.array_equal(res[0][0], res[1][0])
    assert np.array_equal(res[0][1], res[1][1])
    assert res[0][2] == res[1][2]
    assert np.array_equal(res[0][3], res[1][3])


def test_fused_conv_unaligned_vectors_use_hop_chain():
    """Vectors that are not 16-byte aligned take the per-hop sweeps (same result)."""
    import torch
    name, hier = CASES[0]
    J = hier.nlevels
    B = 16
    flat = C.random_params(J, 3, 3, 3, seed=104, spread=0.2)
    g = C.rng(6, 24, 0)
    n = hier.sizes[0]
    f = g.standard_normal((n, B))
    u = g.standard_normal((n, B))
    ctx = ctx_for(hier, flat, 3, B, "fp32")
    ref = to_dev(u, torch.float32)
    ctx.vcycle(to_dev(f, torch.float32), ref)
    buf = torch.zeros(n * B + 1, dtype=torch.float32, device="cuda")
    ud = buf[1:].view(n, B)
    ud.copy_(to_dev(u, torch.float32))
    ctx.vcycle(to_dev(f, torch.float32), ud)
    assert float((ud - ref).abs().max()) == 0.0
    ctx.close()


def _mesh_graph(A):
    """A's pattern plus the other diagonal of every grid cell (a graph that is
    not A's pattern, with more neighbours than A has)."""
    import scipy.sparse as sp
    n = A.shape[0]
    m = int(round(np.sqrt(n)))
    pat = (A != 0).astype(float).tolil()
    for i in range(n):
        x, y = i % m, i // m
        if x + 1 < m and y + 1 < m:
            pat[i, i + m + 1] = 1.0
            pat[i + m + 1, i] = 1.0
    return sp.csr_matrix(pat)


@pytest.mark.parametrize("K,graph", [((6, 2, 5), False), ((3, 3, 3), True)], ids=["K652", "mesh-graph"])
def test_fused_conv_high_order_and_given_graph(K, graph):
    """High convolution orders (deeper halos, smaller tiles) and a separately
    given graph: bit for bit the per-hop sweeps, and the oracle's cycle."""
    import torch
    name, hier = CASES[0]
    J = hier.nlevels
    B = 32
    flat = C.random_params(J, *K, seed=105, spread=0.1)
    G = [_mesh_graph(a) for a in hier.A] if graph else None
    g = C.rng(6, 25, 0)
    f = g.standard_normal((hier.sizes[0], B))
    u = g.standard_normal((hier.sizes[0], B))
    on, off = _pair(hier, flat, K, B, "fp32", G=G)
    outs = []
    for ctx in (on, off):
        ud = to_dev(u, torch.float32)
        ctx.vcycle(to_dev(f, torch.float32), ud)
        outs.append(to_np(ud))
    assert _conv_launches(on, to_dev(f, torch.float32), to_dev(u, torch.float32)) > 0
    want = O.lmg(O.make_levels(hier.A, hier.P, hier.R, G), O.unpack(flat, J, *K), 0, f, u)
    d = float(np.abs(outs[0] - outs[1]).max())
    err = elem_rel(outs[0], want)
    print(f"{name} K={K} graph={graph}: max diff {d:.1e}, rel to oracle {err:.2e}", flush=True)
    assert d == 0.0
    assert err <= TOL["fp32"]
    on.close(); off.close()


@pytest.mark.parametrize("B", [64, 48])
def test_fused_conv_equals_hop_chain_bench_hierarchy(B):
    """The benchmark's hierarchy (513 x 513, log10 a ~ U(-3, 3), 8 levels, four
    tiled levels) with the shipped trained parameters at B = 64 (four column
    groups per tile, the benchmark's launch) and B = 48 (three).  A cycle from a
    random iterate runs the smoothing update (out += scale Phi(s)), Phi_R
    (out = Phi(r)) and Phi_P (u += Phi(P e)); a refinement step from zero runs
    the zero-iterate smoothing launch on D^{-1} f (row scales applied as the
    input enters LDS).  Every element must equal the per-hop chain's bit for
    bit, and the fused context must have launched the tile kernel on every
    tiled level."""
    import torch
    from paper_2608_29082_amd import params as PR
    w = C.diffusion_513(B=B)
    h = w.hier
    J = h.nlevels
    theta, meta = PR.load(PR.default_file("diffusion-513", 3))
    flat = PR.map_levels(theta, meta["J"], J, 3, 3, 3)
    g = C.rng(6, 26, B)
    u = g.standard_normal((h.sizes[0], B))
    on, off = _pair(h, flat, 3, B, "fp32")
    outs = []
    for ctx in (on, off):
        ud = to_dev(u, torch.float32)
        ctx.vcycle(to_dev(w.f, torch.float32), ud)
        e = ctx.refine_step(to_dev(w.f, torch.float64), torch.zeros((h.sizes[0], B), dtype=torch.float64,
                                                                     device="cuda"))
        outs.append((to_np(ud), to_np(e)))
    per_level = []
    for l in range(4):
        on.timing_start("conv", l)
        on.vcycle(to_dev(w.f, torch.float32), to_dev(u, torch.float32))
        torch.cuda.synchronize()
        per_level.append(on.timing_read()[0])
    on.timing_start(None)
    n_off = _conv_launches(off, to_dev(w.f, torch.float32), to_dev(u, torch.float32))
    d1 = np.abs(outs[0][0] - outs[1][0])
    d2 = np.abs(outs[0][1] - outs[1][1])
    print(f"513 B={B}: fused launches per level {per_level}, untiled {n_off}; "
          f"differing elements {int((d1 > 0).sum())} / {int((d2 > 0).sum())}", flush=True)
    assert all(c == 6 for c in per_level) and n_off == 0
    assert d1.max() == 0.0 and d2.max() == 0.0
    on.close(); off.close()


@pytest.mark.parametrize("agg", ["mean", "weighted"])
def test_fused_conv_equals_hop_chain_widest_batch(agg):
    """The widest batch the library takes (B = 256: sixteen column groups per
    tile, 64 lanes per row in the sweeps) on the 129 x 129 hierarchy: the fused
    convolution equals the per-hop sweeps bit for bit, and the cycle is within
    the FP32 tolerance of the FP64 oracle on sampled columns."""
    import torch
    name, hier = CASES[0]
    J = hier.nlevels
    B, K = 256, (3, 3, 3)
    flat = C.random_params(J, *K, seed=103, spread=0.2)
    g = C.rng(6, 23, 0)
    f = g.standard_normal((hier.sizes[0], B))
    u = g.standard_normal((hier.sizes[0], B))
    on, off = _pair(hier, flat, K, B, "fp32", aggregation=agg)
    outs = []
    for ctx in (on, off):
        ud = to_dev(u, torch.float32)
        ctx.vcycle(to_dev(f, torch.float32), ud)
        outs.append(to_np(ud))
    n_on = _conv_launches(on, to_dev(f, torch.float32), to_dev(u, torch.float32))
    d = float(np.abs(outs[0] - outs[1]).max())
    cols = [0, 17, 100, 255]
    lv = O.make_levels(hier.A, hier.P, hier.R, aggregation=agg)
    want = O.lmg(lv, O.unpack(flat, J, *K, 2, 2), 0, f[:, cols], u[:, cols])
    err = elem_rel(outs[0][:, cols], want)
    print(f"{name} {agg} B=256: fused launches {n_on}, max diff to hop chain {d:.1e}, rel to oracle {err:.2e}",
          flush=True)
    assert n_on > 0 and d == 0.0
    assert err <= TOL["fp32"]
    on.close(); off.close()

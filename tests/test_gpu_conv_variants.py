"""GPU parity of the convolution variants (Chebyshev basis, weighted and
symmetric aggregation) against the oracle: cycles in every precision, the LDS
tail, the reverse sweep, and a given weighted graph."""
import numpy as np
import pytest
import scipy.sparse as sp

from mginputs import configs as C
from oracle import adjoint as AD
from oracle import lmg as O
from tests.gpu_util import ctx_for, elem_rel, small_cases, to_dev, to_np

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 2e-5, "bf16": 3e-2}
CASES = small_cases()
VARIANTS = [("mean", "chebyshev"), ("weighted", "monomial"), ("weighted", "chebyshev"), ("sym", "monomial"),
            ("sym", "chebyshev")]


def _oracle(hier, agg, G=None):
    return O.make_levels(hier.A, hier.P, hier.R, G, aggregation=agg)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("agg,basis", VARIANTS)
@pytest.mark.parametrize("name,hier", CASES, ids=[c[0] for c in CASES])
def test_variant_cycle_matches_oracle(prec, agg, basis, name, hier):
    """One cycle from a nonzero iterate (per-level sweeps) and one refinement
    step from zero (LDS tail where it applies)."""
    import torch
    J = hier.nlevels
    B = 3
    flat = C.random_params(J, 3, 3, 3, seed=91, spread=0.2)
    g = C.rng(6, 9, 0)
    f = g.standard_normal((hier.sizes[0], B))
    u = g.standard_normal((hier.sizes[0], B))
    lv = _oracle(hier, agg)
    prm = O.unpack(flat, J, 3, 3, 3, basis=basis)
    want = O.lmg(lv, prm, 0, f, u)
    ctx = ctx_for(hier, flat, 3, B, prec, basis=basis, aggregation=agg)
    ud = to_dev(u, ctx.cycle_dtype)
    ctx.vcycle(to_dev(f, ctx.cycle_dtype), ud)
    err = elem_rel(to_np(ud), want)
    e = ctx.refine_step(to_dev(f, torch.float64), torch.zeros((hier.sizes[0], B), dtype=torch.float64, device="cuda"))
    err2 = elem_rel(to_np(e), O.lmg(lv, prm, 0, f, np.zeros_like(f)))
    print(f"{name} {agg}/{basis} {prec}: cycle {err:.2e} refine {err2:.2e}", flush=True)
    assert err <= TOL[prec] and err2 <= TOL[prec]


@pytest.mark.parametrize("agg,basis", VARIANTS)
def test_variant_gradient_matches_oracle(agg, basis):
    import torch
    from paper_2608_29082_amd import autograd as AG
    name, hier = CASES[1]
    J = hier.nlevels
    B = 2
    flat = C.random_params(J, 3, 3, 3, seed=92, spread=0.2)
    f = C.rng(6, 10, 0).standard_normal((hier.sizes[0], B))
    ctx = ctx_for(hier, flat, 3, B, "fp64", basis=basis, aggregation=agg, backward=True)
    th = torch.tensor(flat, dtype=torch.float64, requires_grad=True)
    L = AG.unrolled_loss(ctx, th, to_dev(f, torch.float64), cycles=3)
    L.backward()
    Lo, go = AD.unrolled_loss_and_grad(_oracle(hier, agg), O.unpack(flat, J, 3, 3, 3, basis=basis), f, cycles=3)
    err = elem_rel(th.grad.numpy(), O.pack(go))
    print(f"grad {agg}/{basis}: loss {L.item():.6e} vs {Lo:.6e} rel {err:.2e}", flush=True)
    assert abs(L.item() - Lo) <= 1e-10 * Lo
    assert err <= 1e-9


def test_given_weighted_graph_matches_oracle():
    """A separately given graph with its own symmetric weights (the mesh
    pattern of A with seeded positive weights) under weighted aggregation."""
    import torch
    name, hier = CASES[1]
    J = hier.nlevels
    G = []
    for l, A in enumerate(hier.A):
        Ac = sp.coo_matrix(A)
        off = Ac.row != Ac.col
        w = C.rng(6, 11, l).uniform(0.5, 2.0, int(off.sum()))
        M = sp.csr_matrix((w, (Ac.row[off], Ac.col[off])), shape=A.shape)
        G.append(sp.csr_matrix(0.5 * (M + M.T)))
    flat = C.random_params(J, 2, 2, 2, seed=93, spread=0.2)
    f = C.rng(6, 12, 0).standard_normal((hier.sizes[0], 2))
    want = O.lmg(_oracle(hier, "weighted", G), O.unpack(flat, J, 2, 2, 2), 0, f, np.zeros_like(f))
    ctx = ctx_for(hier, flat, 2, 2, "fp64", G=G, aggregation="weighted")
    e = ctx.refine_step(to_dev(f, torch.float64), torch.zeros((hier.sizes[0], 2), dtype=torch.float64, device="cuda"))
    err = elem_rel(to_np(e), want)
    print(f"given weighted graph: rel {err:.2e}", flush=True)
    assert err <= 1e-12

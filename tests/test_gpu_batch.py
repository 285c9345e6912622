"""Per-column operators (a batch of requests on one grid, mg_hierarchy
.ncolumn_values = nrhs): every column solves with its own coefficient
field's hierarchy on the shared pattern.

  * one FP64 cycle per column against the oracle's cycle on that column's own
    hierarchy (1e-12, element by element), B = 5 (no tiles, ragged lanes);
  * FP32 solves at B = 16 (fused tiles, coarse tail, compaction): each
    column's cycle count equals the oracle's float32 emulation of its own
    solve, and its FP64 residual meets 1e-8;
  * mg_load_column puts another request into a column: that column then
    equals the same request in a freshly set-up batch, bit for bit, and a
    column's result does not depend on the other columns;
  * compaction on or off: the same bits; a pattern of another size is refused."""
import hashlib

import numpy as np
import pytest

from mginputs import configs as C
from oracle import lmg as O
from oracle import mixed as MX
from tests.gpu_util import elem_rel, to_dev, to_np

pytestmark = pytest.mark.gpu


def _pattern_key(h):
    hs = hashlib.sha1()
    for l in range(h.nlevels):
        m = h.view.A[l]
        hs.update(np.ctypeslib.as_array(m.rowptr, shape=(m.nrows + 1,)).tobytes())
        hs.update(np.ctypeslib.as_array(m.col, shape=(m.nnz,)).tobytes())
    return hs.hexdigest()


def _requests(side, count, seed=7):
    """`count` serving-distribution requests of one side sharing one pattern: (hierarchy, f) pairs."""
    from paper_2608_29082_amd import binding as Bd
    out, key, k = [], None, 0
    while len(out) < count:
        _, blocks = C.serving_request(k, seed, sides=(side,))
        h = Bd.SquareHierarchy(side, blocks)
        kk = _pattern_key(h)
        if key is None:
            key = kk
        if kk == key:
            out.append((h, C.serving_rhs(k, h.sizes[0], seed)[:, 0]))
        else:
            h.close()
        k += 1
    return out


def _params(side, J):
    from paper_2608_29082_amd import params as PR
    th, meta = PR.load(PR.default_file(f"serving-{side}", 3))
    return PR.map_levels(th, meta["J"], J, 3, 3, 3)


def _ctx(reqs, precision, flat, **kw):
    from paper_2608_29082_amd import binding as Bd
    h0 = reqs[0][0]
    return Bd.Context(None, None, flat, 3, 3, 3, precision=precision, nrhs=len(reqs), native=h0,
                      columns=[h for h, _ in reqs], **kw)


def test_fp64_cycle_per_column_matches_oracle():
    import torch
    reqs = _requests(65, 5)
    J = reqs[0][0].nlevels
    flat = C.random_params(J, 3, 3, 3, seed=31, spread=0.2)
    ctx = _ctx(reqs, "fp64", flat)
    g = C.rng(6, 70, 0)
    n = reqs[0][0].sizes[0]
    f = np.stack([r[1] for r in reqs], axis=1)
    u = g.standard_normal((n, len(reqs)))
    ud = to_dev(u, torch.float64)
    ctx.vcycle(to_dev(f, torch.float64), ud)
    got = to_np(ud)
    errs = []
    for b, (h, _) in enumerate(reqs):
        A, P = h.to_scipy()
        want = O.lmg(O.make_levels(A, P), O.unpack(flat, J, 3, 3, 3), 0, f[:, b:b + 1], u[:, b:b + 1])
        errs.append(elem_rel(got[:, b:b + 1], want))
    print("per-column fp64 cycle errors", ["%.1e" % e for e in errs], flush=True)
    assert max(errs) <= 1e-12
    ctx.close()


@pytest.mark.parametrize("side", [65, 129])
def test_fp32_batch_counts_match_emulation(side):
    import torch
    reqs = _requests(side, 16)
    J = reqs[0][0].nlevels
    flat = _params(side, J)
    ctx = _ctx(reqs, "fp32", flat, max_outer=2000, check_every=2)
    f = np.stack([r[1] for r in reqs], axis=1)
    u = torch.zeros((f.shape[0], 16), dtype=torch.float64, device="cuda")
    ctx.timing_start("conv", -1)
    info = ctx.solve(to_dev(f, torch.float64), u)
    nconv = ctx.timing_read()[0]
    ctx.timing_start(None)
    us = to_np(u)
    emu, rel = [], []
    for b, (h, _) in enumerate(reqs):
        A, P = h.to_scipy()
        lv = O.make_levels(A, P)
        r = MX.solve_mixed(lv, O.unpack(flat, J, 3, 3, 3), f[:, b:b + 1], rtol=1e-8, max_cycles=2000)
        emu.append(int(r.iters[0]))
        rel.append(np.linalg.norm(f[:, b] - A[0] @ us[:, b]) / np.linalg.norm(f[:, b]))
    print(f"{side}: gpu iters {info.iters.tolist()}, emulation {emu}, fused launches {nconv}", flush=True)
    assert info.code == 0 and max(rel) <= 1e-8
    assert info.iters.tolist() == emu
    assert nconv > 0
    ctx.close()


def test_load_column_and_column_independence():
    import torch
    reqs = _requests(65, 20)
    J = reqs[0][0].nlevels
    flat = _params(65, J)
    n = reqs[0][0].sizes[0]

    def run(cols, fcols, compact=True):
        ctx = _ctx(cols, "fp32", flat, max_outer=2000, check_every=3, compact=compact)
        fd = to_dev(np.stack(fcols, axis=1), torch.float64)
        u = torch.zeros_like(fd)
        info = ctx.solve(fd, u)
        return ctx, info, to_np(u)

    base = reqs[:16]
    fz = np.zeros(n)
    ctx, info0, u0 = run(base, [r[1] for r in base])
    # column 3 takes request 18
    ctx.load_column(3, reqs[18][0])
    fcols = [r[1] for r in base]
    fcols[3] = reqs[18][1]
    fd = to_dev(np.stack(fcols, axis=1), torch.float64)
    u1 = torch.zeros_like(fd)
    info1 = ctx.solve(fd, u1)
    u1 = to_np(u1)
    # the same request alone in a fresh batch (the other columns empty) and in column 3 of another mix
    alone_cols = [reqs[18]] + base[1:16]
    _, info2, u2 = run(alone_cols, [reqs[18][1]] + [fz] * 15)
    mix = base[:3] + [reqs[18]] + reqs[4:16]
    _, info3, u3 = run(mix, [r[1] for r in mix], compact=False)
    print(f"request 18: iters {info1.iters[3]} / {info2.iters[0]} / {info3.iters[3]}", flush=True)
    assert info1.iters[3] == info2.iters[0] == info3.iters[3]
    assert np.array_equal(u1[:, 3], u2[:, 0]) and np.array_equal(u1[:, 3], u3[:, 3])
    # the other columns did not change
    keep = [b for b in range(16) if b != 3]
    assert np.array_equal(u1[:, keep], u0[:, keep]) and np.array_equal(info1.iters[keep], info0.iters[keep])
    # a hierarchy of another grid is refused before the library reads it
    other = _requests(129, 1)[0][0]
    with pytest.raises(ValueError):
        ctx.load_column(0, other)
    ctx.close()

"""Iteration counts of the mixed-precision solver against the oracle's
float32 / bfloat16 emulation (oracle/mixed.py).

mg_solve runs the refinement form u += LMG_p(A, fl_p(f - A u), 0) with FP64
residuals and FP32 cycles (BF16 storage of the smoother input, of Phi_R's
output and of P e_c on the levels whose convolutions run over LDS tiles,
FP32 on the LDS-resident coarse levels).  The emulation computes the same
iteration with NumPy float32 arithmetic and bfloat16 rounding of the same
stored intermediates, so the GPU's per-column cycle counts must agree with
it up to the effect of operation order near the stopping threshold (a
column whose residual crosses rtol in the same cycle in both, give or take
the slack written below)."""
import numpy as np
import pytest

from mginputs import configs as C
from oracle import lmg as O
from oracle import mixed as MX
from tests.gpu_util import ctx_for, to_dev, to_np

pytestmark = pytest.mark.gpu

TILE_MIN_ROWS = 2048   # levels with at least this many rows run the fused tile kernel (B % 16 == 0)


def _case(side, B, params):
    from paper_2608_29082_amd import params as PR
    w = C.block_diffusion(2, side, -2, 2, B=B, K=3, seed=5)
    J = w.hier.nlevels
    if params == "trained":
        th, meta = PR.load(PR.default_file(f"serving-{side}", 3))
        flat = PR.map_levels(th, meta["J"], J, 3, 3, 3)
    else:
        flat = C.identity_params(J, 3, 3, 3)
    return w, flat


@pytest.mark.parametrize("side,B,params", [(129, 16, "trained"), (129, 16, "identity"), (257, 16, "trained")])
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_cycle_counts_match_emulation(precision, side, B, params):
    import torch
    w, flat = _case(side, B, params)
    h = w.hier
    J = h.nlevels
    ctx = ctx_for(h, flat, 3, B, precision, max_outer=3000, check_every=1)
    f = to_dev(w.f, torch.float64)
    u = torch.zeros_like(f)
    info = ctx.solve(f, u)
    ctx.close()
    bf16_levels = {l for l in range(J - 1) if h.sizes[l] >= TILE_MIN_ROWS} if precision == "bf16" else ()
    emu = MX.solve_mixed(O.make_levels(h.A, h.P, h.R), O.unpack(flat, J, 3, 3, 3), w.f, rtol=1e-8,
                         max_cycles=3000, bf16_levels=bf16_levels)
    d = info.iters - emu.iters
    rel = np.linalg.norm(w.f - h.A[0] @ to_np(u), axis=0) / np.linalg.norm(w.f, axis=0)
    print(f"{side} {params} {precision}: gpu {info.iters.min()}..{info.iters.max()} (mean {info.iters.mean():.1f}), "
          f"emulation {emu.iters.min()}..{emu.iters.max()} (mean {emu.iters.mean():.1f}), "
          f"differences {sorted(set(d.tolist()))}", flush=True)
    assert info.code == 0 and np.all(rel <= 1e-8) and np.all(emu.converged)
    # slack: one cycle per column, and the mean within 1 %
    assert np.all(np.abs(d) <= 1)
    assert abs(info.iters.mean() - emu.iters.mean()) <= 0.01 * emu.iters.mean()

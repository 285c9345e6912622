"""mg_fgmres_static, the allocation-free FGMRES entry point, through the C ABI:
its results equal mg_fgmres's (same kernels, the workspace in the library's
static per-GPU buffer instead of a caller buffer) on two calls in a row, the
second on a smaller problem, and a workspace beyond the static size is refused
before any device work."""
import numpy as np
import pytest

from mginputs import configs as C, hierarchy as H
from tests.gpu_util import ctx_for, elem_rel, to_dev, to_np

pytestmark = pytest.mark.gpu


def _pair(hier, B, seed, precond, restart):
    """(reference mg_fgmres result, mg_fgmres_static result) from the same start."""
    import torch
    J = hier.nlevels
    ctx = ctx_for(hier, C.random_params(J, 3, 3, 3, seed=seed, spread=0.1), 3, B, "fp32")
    f = to_dev(C.rng(6, 60, seed).standard_normal((hier.sizes[0], B)), torch.float64)
    x_ref = torch.zeros_like(f)
    need = ctx.fgmres_workspace_bytes(restart, precond)
    assert need <= 64 << 20
    work = torch.empty(need, dtype=torch.uint8, device="cuda")
    i_ref = ctx.fgmres(f, x_ref, restart=restart, max_iter=400, precond=precond, work=work)
    x = torch.zeros_like(f)
    i_st = ctx.fgmres_static(f, x, restart=restart, max_iter=400, precond=precond)
    torch.cuda.synchronize()
    return ctx, (i_ref, to_np(x_ref)), (i_st, to_np(x))


def test_static_fgmres_equals_fgmres_two_calls():
    big = H.square_hierarchy(129, H.block_field(C.rng(7, 1, 3), 16, -2, 2))
    small = H.square_hierarchy(65, H.block_field(C.rng(7, 1, 4), 16, -2, 2))
    for hier, B, seed, pc, m in ((big, 16, 1, "vcycle", 10), (small, 3, 2, "fmg", 20)):
        ctx, (i_ref, x_ref), (i_st, x) = _pair(hier, B, seed, pc, m)
        print(f"n = {hier.sizes[0]}, B = {B}, {pc}: iterations {i_ref.iters.tolist()} / {i_st.iters.tolist()}, "
              f"max difference {float(np.abs(x - x_ref).max()):.1e}", flush=True)
        assert i_ref.code == 0 and i_st.code == 0
        assert np.array_equal(i_ref.iters, i_st.iters)
        assert np.array_equal(i_ref.relres, i_st.relres)
        assert np.array_equal(x, x_ref) and elem_rel(x, x_ref) == 0.0
        ctx.close()


def test_static_fgmres_refuses_oversize_workspace():
    import torch
    from paper_2608_29082_amd.binding import MGError
    hier = H.square_hierarchy(129)
    J = hier.nlevels
    ctx = ctx_for(hier, C.identity_params(J, 1, 1, 1), 1, 16, "fp32")
    assert ctx.fgmres_workspace_bytes(40) > 64 << 20
    f = to_dev(C.rng(6, 61, 0).standard_normal((hier.sizes[0], 16)), torch.float64)
    x = torch.zeros_like(f)
    with pytest.raises(MGError) as e:
        ctx.fgmres_static(f, x, restart=40, raise_on_failure=True)
    assert e.value.status == 3           # MG_ERR_OOM
    assert float(x.abs().max()) == 0.0   # nothing ran
    ctx.close()

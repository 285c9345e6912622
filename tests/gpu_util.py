"""Shared helpers of the GPU tests (imports the binding lazily)."""
import numpy as np

from mginputs import configs as C, hierarchy as H
from oracle import lmg as O


def ctx_for(hier, params, K, nrhs, precision="fp64", nu=(2, 2), backward=False, R=None, G=None, **kw):
    from paper_2608_29082_amd import binding as Bd
    KB, KR, KP = K if isinstance(K, tuple) else (K, K, K)
    return Bd.Context(hier.A, hier.P, params, KB, KR, KP, nu_pre=nu[0], nu_post=nu[1], precision=precision,
                      nrhs=nrhs, R=R, G=G, backward=backward, **kw)


def oracle_levels(hier, R=None, G=None):
    return O.make_levels(hier.A, hier.P, R if R is not None else hier.R, G)


def oracle_params(flat, J, K, nu=(2, 2)):
    KB, KR, KP = K if isinstance(K, tuple) else (K, K, K)
    return O.unpack(flat, J, KB, KR, KP, nu[0], nu[1])


def to_dev(x, dtype):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def to_np(t):
    return t.detach().double().cpu().numpy()


def elem_rel(a, b):
    """Element-wise error of `a` against the reference `b`, normalised per
    column: max over columns c of max_i |a_ic - b_ic| / max_i |b_ic| (a 1-D
    array is one column).  Every element is held to the bound, so one wrong
    row, halo or column group cannot hide behind the rest of the array as it
    can in a whole-array 2-norm.  A zero reference column is measured by the
    largest magnitude of the reference array instead."""
    a = np.asarray(a)
    b = np.asarray(b)
    if b.ndim == 1:
        a, b = a[:, None], b[:, None]
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    d = np.abs(a - b).max(axis=0)
    s = np.abs(b).max(axis=0)
    floor = max(float(np.abs(b).max()), 1e-300)
    s = np.where(s > 0, s, floor)
    r = d / s
    return float(np.nan_to_num(r, nan=np.inf).max())


def small_cases():
    """(name, hierarchy) pairs spanning several tiles and ragged tails."""
    out = [("poisson33", H.square_hierarchy(33)),
           ("blocks65", H.square_hierarchy(65, H.block_field(C.rng(7, 1, 0), 16, -2, 2))),
           ("lshape", H.lshape_hierarchy(C.rng(7, 4, 0), target_nodes=120, refinements=2))]
    return out

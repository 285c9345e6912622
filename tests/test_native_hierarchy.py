"""The library's native structured-hierarchy builder (host code, no GPU)
reproduces the seeded Python generator: same sparsity patterns, values equal
to round-off, R = P^T, exactly symmetric operators."""
import os

import numpy as np
import pytest

from mginputs import configs as C, hierarchy as H


def _lib():
    from paper_2608_29082_amd import binding as Bd
    if not os.path.exists(Bd.LIB_PATH):
        pytest.skip("libmgl.so not built")
    return Bd


@pytest.mark.parametrize("side,lo,hi", [(33, 0.0, 0.0), (65, -2.0, 2.0), (129, -3.0, 3.0)])
def test_native_square_hierarchy_matches_generator(side, lo, hi):
    Bd = _lib()
    blocks = H.block_field(C.rng(5, 1, side), 16, lo, hi) if hi > lo else np.ones((16, 16))
    ref = H.square_hierarchy(side, blocks)
    nat = Bd.SquareHierarchy(side, blocks)
    A, P = nat.to_scipy()
    assert nat.sizes == ref.sizes
    for a, b in zip(A, ref.A):
        assert (a != 0).sum() == (b != 0).sum()
        assert abs((a != 0).astype(int) - (b != 0).astype(int)).sum() == 0
        d = abs(a - b)
        assert d.max() <= 1e-14 * abs(b).max()
        assert (a != a.T).nnz == 0
    for p, q in zip(P, ref.P):
        assert (p != q).nnz == 0


def test_native_builder_rejects_bad_sizes():
    Bd = _lib()
    with pytest.raises(Bd.MGError):
        Bd.SquareHierarchy(34, np.ones((4, 4)))
    with pytest.raises(Bd.MGError):
        Bd.SquareHierarchy(33, -np.ones((4, 4)))


@pytest.mark.parametrize("side,count", [(65, 6), (257, 4), (513, 3)])
def test_same_side_requests_share_one_pattern(side, count):
    """Every level's pattern depends on the grid and the block geometry, not on
    the coefficient values: the rounding residue of exactly cancelling Galerkin
    couplings is removed on every level, so requests of one side can share a
    batch (per-column operators on one pattern)."""
    Bd = _lib()
    pats = []
    for k in range(count):
        _, blocks = C.serving_request(k, 21, sides=(side,))
        h = Bd.SquareHierarchy(side, blocks)
        A, _ = h.to_scipy()
        h.close()
        pats.append([(a.indptr.copy(), a.indices.copy()) for a in A])
    for p in pats[1:]:
        for (r0, c0), (r1, c1) in zip(pats[0], p):
            assert np.array_equal(r0, r1) and np.array_equal(c0, c1)

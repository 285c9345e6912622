"""Host logic of the Helmholtz training module (CPU): the partial weight
transfer between hierarchies (Sec. 4.2, transfer rule)."""
import numpy as np

from mginputs import configs as C
from paper_2608_29082_amd import train_helmholtz as TH

K = 1
PER = 2 + 4 * (K + 1)


def _levels(theta, J):
    return theta[:(J - 1) * PER].reshape(J - 1, PER), theta[(J - 1) * PER:]


def test_transfer_same_hierarchy_is_identity_map():
    plan = [("jacobi", 1, 1), ("jacobi", 1, 1), ("gmres", 1, 2), ("gmres", 1, 2)]
    th = C.hz_random_params(5, K, K, K, plan, seed=1)
    assert np.array_equal(TH.transfer(th, plan, plan, K), th)


def test_transfer_to_deeper_hierarchy_copies_the_deepest_matching_level():
    src_plan = [("jacobi", 1, 1), ("jacobi", 1, 1), ("gmres", 1, 2), ("gmres", 1, 2)]
    dst_plan = src_plan + [("gmres", 1, 2), ("gmres", 1, 2)]
    th = C.hz_random_params(5, K, K, K, src_plan, seed=2)
    out = TH.transfer(th, src_plan, dst_plan, K)
    ls, ss = _levels(th, 5)
    ld, sd = _levels(out, 7)
    assert np.array_equal(ld[:4], ls)
    assert np.array_equal(ld[4], ls[3]) and np.array_equal(ld[5], ls[3])
    assert np.array_equal(sd, ss)


def test_transfer_mismatched_level_falls_back_to_the_classical_smoother():
    src_plan = [("jacobi", 1, 1), ("gmres", 1, 2)]
    dst_plan = [("gmres", 1, 2), ("gmres", 1, 2), ("gmres", 1, 2)]
    th = C.hz_random_params(3, K, K, K, src_plan, seed=3)
    out = TH.transfer(th, src_plan, dst_plan, K)
    ls, _ = _levels(th, 3)
    ld, _ = _levels(out, 4)
    ident, _ = _levels(C.hz_identity_params(4, K, K, K, dst_plan), 4)
    assert np.array_equal(ld[0], ident[0])          # theta = 0, eta = 1, W_0 = I: classical GMRES
    assert np.array_equal(ld[1], ls[1]) and np.array_equal(ld[2], ls[1])

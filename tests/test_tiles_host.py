"""Host-side tiling of the fused K-hop convolution (csrc/tiles.hpp), no GPU.

A small C++ driver (tests/native/tiles_check.cpp) compiled with the host
compiler builds the tiles of seeded graphs, runs the library's invariant
check, and recomputes every hop of the convolution per tile from the tile's
own lists; the result must equal the hops applied to the whole graph
(double precision, identical summation order, so exactly), and every node
must be the own node of exactly one tile."""
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

from mginputs import configs as C, hierarchy as H

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = tmp_path_factory.mktemp("tiles") / "tiles_check"
    subprocess.run([cxx, "-O2", "-std=c++17", "-pthread", "-I", os.path.join(ROOT, "paper_2608_29082_amd", "csrc"),
                    os.path.join(HERE, "native", "tiles_check.cpp"), "-o", str(exe)], check=True)
    return str(exe)


def _ell(A, tmp):
    """Slot-major ELL pattern of A's off-diagonal entries (padding col == row), written for the driver."""
    A = sp.csr_matrix(A)
    n = A.shape[0]
    rows = []
    for i in range(n):
        c = A.indices[A.indptr[i]:A.indptr[i + 1]]
        rows.append(c[c != i])
    w = max(4, -(-max(len(r) for r in rows) // 4) * 4)
    col = np.tile(np.arange(n, dtype=np.int32), (w, 1))
    for i, r in enumerate(rows):
        col[:len(r), i] = r
    path = os.path.join(tmp, f"g{n}_{w}.bin")
    with open(path, "wb") as fh:
        np.array([n, w], dtype=np.int32).tofile(fh)
        col.astype(np.int32).tofile(fh)
    return path


def _run(driver, path, KM, side):
    out = subprocess.run([driver, path, str(KM), str(side)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    tok = out.stdout.split()
    assert tok[0] == "ok"
    return int(tok[1]), float(tok[2]), float(tok[3]), int(tok[4])


def _random_graph(n, deg, seed):
    g = C.rng(8, 1, seed)
    i = np.repeat(np.arange(n), deg)
    j = g.integers(0, n, size=n * deg)
    M = sp.coo_matrix((np.ones(n * deg), (i, j)), shape=(n, n)).tocsr()
    return M + M.T


@pytest.mark.parametrize("KM,side", [(2, 16), (3, 15), (4, 12), (3, 8)])
def test_tiles_on_grid_levels(driver, tmp_path, KM, side):
    hier = H.square_hierarchy(129, H.block_field(C.rng(8, 2, 0), 16, -2, 2))
    for A in hier.A[:3]:
        ntiles, listed, err, cover = _run(driver, _ell(A, str(tmp_path)), KM, side)
        assert err == 0.0 and cover == 1
        assert 1.0 <= listed < 4.0


def test_tiles_on_unstructured_mesh(driver, tmp_path):
    hier = H.lshape_hierarchy(C.rng(7, 4, 0), target_nodes=120, refinements=3)
    ntiles, listed, err, cover = _run(driver, _ell(hier.A[0], str(tmp_path)), 3, 12)
    assert err == 0.0 and cover == 1 and ntiles > 10


def test_tiles_on_disconnected_and_random_graphs(driver, tmp_path):
    # two disconnected grids (several breadth-first searches) and an expander-like random graph
    A = H.square_hierarchy(33).A[0]
    B = sp.block_diag([A, A]).tocsr()
    ntiles, listed, err, cover = _run(driver, _ell(B, str(tmp_path)), 3, 8)
    assert err == 0.0 and cover == 1
    R = _random_graph(3000, 2, 0)
    ntiles, listed, err, cover = _run(driver, _ell(R, str(tmp_path)), 2, 8)
    assert err == 0.0 and cover == 1

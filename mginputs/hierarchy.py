"""Multigrid hierarchies (A_l, P_l, R_l) built as input data.

The learnable V-cycle (paper Alg. 2) takes, for every level l, the system
matrix A_l, the prolongation P_l and the restriction R_l as given.  This module
builds them the way the paper describes for geometric multigrid (Sec. 2.2):
P_l is the natural inclusion of nested P1 spaces, R_l = P_l^T, and the coarse
operators are either rediscretised on the coarse mesh or Galerkin products
A_{l+1} = R_l A_l P_l.  Level 0 is the finest (the paper's level 1).

Galerkin products are symmetrised and off-diagonal entries that are round-off
residue of cancellation (|a_ij| <= 1e-11 sqrt(|a_ii a_jj|)) are removed, so the
stored pattern of A_l is its graph {(i, j): A_ij != 0} (Sec. 2.1).  Couplings
that are exactly zero (the diagonal direction inside a block of constant
coefficient) leave a residue that grows with every product, to ~1e-13 of the
diagonal on the coarsest levels; couplings that are not zero stay above ~1e-4
of it, so the threshold separates the two and the pattern depends on the grid
and the block geometry only, not on the coefficient values.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from . import fem

DROP_TOL = 1e-11


@dataclass
class Hierarchy:
    A: list                      # [J] scipy CSR, float64, sorted indices
    P: list                      # [J-1] CSR n_l x n_{l+1}
    R: list                      # [J-1] CSR n_{l+1} x n_l (= P^T)
    meta: dict = field(default_factory=dict)

    @property
    def nlevels(self) -> int:
        return len(self.A)

    @property
    def sizes(self):
        return [a.shape[0] for a in self.A]


def clean_csr(A: sp.spmatrix) -> sp.csr_matrix:
    A = sp.csr_matrix(A)
    A.sum_duplicates()
    A.eliminate_zeros()
    A.sort_indices()
    A.indices = A.indices.astype(np.int32)
    A.indptr = A.indptr.astype(np.int32)
    return A


def drop_roundoff(A: sp.csr_matrix, tol: float = DROP_TOL) -> sp.csr_matrix:
    """Symmetrise (assembly and Galerkin products are symmetric up to
    round-off) and remove off-diagonal round-off residue."""
    A = 0.5 * (A + A.T)
    A = sp.coo_matrix(A)
    d = np.abs(A.diagonal())
    off = A.row != A.col
    small = off & (np.abs(A.data) <= tol * np.sqrt(d[A.row] * d[A.col]))
    A.data[small] = 0.0
    return clean_csr(A)


def galerkin(A: sp.csr_matrix, P: sp.csr_matrix) -> sp.csr_matrix:
    return drop_roundoff(sp.csr_matrix(P.T @ A @ P))


def block_field(rng: np.random.Generator, nblocks: int, lo: float, hi: float) -> np.ndarray:
    """(nblocks, nblocks) piecewise-constant coefficient, log10 a ~ U(lo, hi).
    Entry [bj, bi] covers [bi/nb, (bi+1)/nb) x [bj/nb, (bj+1)/nb)."""
    return 10.0 ** rng.uniform(lo, hi, size=(nblocks, nblocks))


def triangle_coef_from_blocks(pts, tris, blocks: np.ndarray) -> np.ndarray:
    nb = blocks.shape[0]
    cen = pts[tris].mean(axis=1)
    bi = np.minimum((cen[:, 0] * nb).astype(np.int64), nb - 1)
    bj = np.minimum((cen[:, 1] * nb).astype(np.int64), nb - 1)
    return blocks[bj, bi]


def levels_for_side(side: int, coarsest_interior: int = 3) -> int:
    """Number of levels when coarsening side -> (side+1)/2 until the interior is
    coarsest_interior x coarsest_interior (33 -> 4 levels, 513 -> 8)."""
    J, s = 1, side
    while s - 2 > coarsest_interior:
        assert s % 2 == 1, "side must be 2^k + 1"
        s = (s + 1) // 2
        J += 1
    assert s - 2 == coarsest_interior, "side must be 2^k + 1"
    return J


def square_hierarchy(side: int, blocks: np.ndarray | None = None, nlevels: int | None = None,
                     coarsening: str = "galerkin") -> Hierarchy:
    """Hierarchy for -div(a grad u) = f on the unit square, "/" P1 mesh.

    blocks: piecewise-constant coefficient (see block_field) or None for a = 1.
    coarsening: "galerkin" (A_{l+1} = P^T A_l P) or "geometric" (rediscretise on
    the coarse mesh with the coefficient sampled at coarse-triangle centroids).
    """
    J = nlevels or levels_for_side(side)
    sides = [side]
    for _ in range(J - 1):
        sides.append((sides[-1] + 1) // 2)

    def assemble(s):
        pts, tris, interior = fem.square_mesh(s)
        coef = 1.0 if blocks is None else triangle_coef_from_blocks(pts, tris, blocks)
        return drop_roundoff(fem.assemble_p1(pts, tris, coef, interior))

    A = [assemble(side)]
    P, R = [], []
    for l in range(J - 1):
        Pl = clean_csr(fem.square_prolongation(sides[l]))
        P.append(Pl)
        R.append(clean_csr(Pl.T))
        if coarsening == "galerkin":
            A.append(galerkin(A[-1], Pl))
        elif coarsening == "geometric":
            A.append(assemble(sides[l + 1]))
        else:
            raise ValueError(coarsening)
    return Hierarchy(A, P, R, meta={"kind": "square", "sides": sides, "coarsening": coarsening})


# ----------------------------------------------------------------------------- L-shape
def lshape_coarse_mesh(rng: np.random.Generator, target_nodes: int = 800):
    """Jittered-grid Delaunay mesh of L = (-1,1)^2 minus (0,1]^2.

    A uniform point lattice of spacing d covering the square is jittered by up
    to d/4 (boundary points slide only along their edge, corners stay), points
    inside the removed quadrant are dropped, the set is triangulated, and
    triangles whose centroid lies in the removed quadrant are discarded.
    """
    from scipy.spatial import Delaunay
    # the L covers 3/4 of the 2x2 square: pick k so that ~target_nodes remain
    k = int(round(np.sqrt(target_nodes / 0.75))) - 1
    d = 2.0 / k
    g = np.linspace(-1.0, 1.0, k + 1)
    X, Y = np.meshgrid(g, g, indexing="xy")
    X, Y = X.ravel(), Y.ravel()
    jx = rng.uniform(-0.25, 0.25, X.shape) * d
    jy = rng.uniform(-0.25, 0.25, Y.shape) * d

    def on(v, c):
        return np.isclose(v, c)

    fixx = on(X, -1) | on(X, 1) | (on(X, 0) & (Y >= 0))
    fixy = on(Y, -1) | on(Y, 1) | (on(Y, 0) & (X >= 0))
    X = X + np.where(fixx, 0.0, jx)
    Y = Y + np.where(fixy, 0.0, jy)
    keep = ~((X > 1e-12) & (Y > 1e-12))
    pts = np.stack([X[keep], Y[keep]], axis=1)
    tri = Delaunay(pts).simplices
    cen = pts[tri].mean(axis=1)
    tri = tri[~((cen[:, 0] > 0) & (cen[:, 1] > 0))]
    # orient counter-clockwise
    p = pts[tri]
    a2 = (p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1]) - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1])
    tri = np.where((a2 < 0)[:, None], tri[:, [0, 2, 1]], tri)
    # boundary: vertices on edges used by exactly one triangle
    e = np.sort(np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]]), axis=1)
    u, c = np.unique(e, axis=0, return_counts=True)
    bnd = np.zeros(len(pts), dtype=bool)
    bnd[u[c == 1].ravel()] = True
    return pts, tri.astype(np.int64), bnd


def rotated_anisotropy(eps: float = 1e-3, angle_deg: float = 30.0) -> np.ndarray:
    t = np.deg2rad(angle_deg)
    Q = np.array([[np.cos(t), -np.sin(t)], [np.sin(t), np.cos(t)]])
    return Q @ np.diag([1.0, eps]) @ Q.T


def interior_map(boundary: np.ndarray) -> np.ndarray:
    m = -np.ones(len(boundary), dtype=np.int64)
    inner = ~boundary
    m[inner] = np.arange(int(inner.sum()))
    return m


def lshape_hierarchy(rng: np.random.Generator, target_nodes: int = 800, refinements: int = 4,
                     tensor: np.ndarray | None = None, coarsening: str = "galerkin") -> Hierarchy:
    """Nested hierarchy on the L-shape: coarse jittered Delaunay mesh refined
    uniformly `refinements` times (levels = refinements + 1)."""
    Kt = rotated_anisotropy() if tensor is None else tensor
    meshes = [lshape_coarse_mesh(rng, target_nodes)]
    parents = []
    for _ in range(refinements):
        p, t, b = meshes[-1]
        pf, tf, bf, par = fem.refine_uniform(p, t, b)
        meshes.append((pf, tf, bf))
        parents.append(par)
    meshes = meshes[::-1]           # finest first
    parents = parents[::-1]
    maps = [interior_map(b) for (_, _, b) in meshes]
    A0 = drop_roundoff(fem.assemble_p1(meshes[0][0], meshes[0][1], Kt, maps[0]))
    A, P, R = [A0], [], []
    for l in range(refinements):
        Pl = clean_csr(fem.nested_prolongation(parents[l], maps[l], maps[l + 1]))
        P.append(Pl)
        R.append(clean_csr(Pl.T))
        if coarsening == "galerkin":
            A.append(galerkin(A[-1], Pl))
        else:
            pc, tc, _ = meshes[l + 1]
            A.append(drop_roundoff(fem.assemble_p1(pc, tc, Kt, maps[l + 1])))
    coords = [m[0][mp >= 0] for m, mp in zip(meshes, maps)]
    return Hierarchy(A, P, R, meta={"kind": "lshape", "coords0": coords[0], "coarsening": coarsening})


def rcm_permute(h: Hierarchy) -> Hierarchy:
    """Reverse Cuthill-McKee renumbering of every level (a locality reordering:
    the operators are the same up to a symmetric permutation)."""
    from scipy.sparse.csgraph import reverse_cuthill_mckee
    perms = [np.asarray(reverse_cuthill_mckee(a, symmetric_mode=True)) for a in h.A]
    A = [clean_csr(a[p][:, p]) for a, p in zip(h.A, perms)]
    P = [clean_csr(Pl[perms[l]][:, perms[l + 1]]) for l, Pl in enumerate(h.P)]
    R = [clean_csr(Pl.T) for Pl in P]
    meta = dict(h.meta)
    meta["perms"] = perms
    return Hierarchy(A, P, R, meta=meta)

"""Helmholtz problems with an impedance boundary, built as input data.

The second model problem of the paper (Sec. 4.2, Helmholtz subsection):
    -Lap u - k^2 u = f in Omega,   du/dn - i k u = 0 on the boundary,
Omega the unit square centred at the origin.  The weak form with P1 elements
gives the complex symmetric matrix
    A = K - k^2 M - i k M_b
(stiffness K, consistent mass M, boundary mass M_b); every vertex is an
unknown (no Dirichlet part).  The paper meshes with nonuniform pygmsh
triangles; here the uniform "/" triangulation of the square stands in for it
(the same mesh family as the diffusion workloads), coarsened geometrically
by uniform derefinement.  P_l is the natural inclusion of nested P1 spaces
(barycentric interpolation on nested meshes), R_l = P_l^T, and A_l is
rediscretised on each mesh (on nested P1 meshes that equals the Galerkin
product P^T A P, which a test checks).

Right-hand sides are load vectors M f_h of smoothed-disk sources (the
training source with one centre and the test source with two, eqs. for the
Helmholtz training and testing sources); further columns move the disks to
seeded random centres.  Nothing here computes any part of the multigrid
method.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from . import fem

R_S = 0.02          # disk radius of the sources
EPS_S = 0.001       # smoothing width of the sources
AMP = 100.0


def mesh(side: int):
    """"/" mesh of [-1/2, 1/2]^2 with `side` points per direction: vertex
    (i, j) has id j*side + i; every vertex is an unknown."""
    pts, tris, _ = fem.square_mesh(side)
    return pts - 0.5, tris


def boundary_edges(side: int) -> np.ndarray:
    """(4 (side - 1), 2) vertex pairs of the boundary segments."""
    s = side
    a = np.arange(s - 1)
    south = np.stack([a, a + 1], 1)
    north = np.stack([(s - 1) * s + a, (s - 1) * s + a + 1], 1)
    west = np.stack([a * s, (a + 1) * s], 1)
    east = np.stack([a * s + s - 1, (a + 1) * s + s - 1], 1)
    return np.concatenate([south, north, west, east], 0)


def _coo(n, r, c, v):
    A = sp.coo_matrix((v, (r, c)), shape=(n, n)).tocsr()
    A.sum_duplicates()
    return A


def matrices(side: int):
    """(K, M, M_b) on the mesh with `side` points per direction."""
    pts, tris = mesh(side)
    n = side * side
    K = fem.assemble_p1(pts, tris, 1.0, np.arange(n))
    p = pts[tris]
    area = 0.5 * np.abs((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1])
                        - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1]))
    me = np.array([[2.0, 1.0, 1.0], [1.0, 2.0, 1.0], [1.0, 1.0, 2.0]]) / 12.0
    M = _coo(n, np.repeat(tris, 3, axis=1).ravel(), np.tile(tris, (1, 3)).ravel(),
             (area[:, None, None] * me).ravel())
    e = boundary_edges(side)
    L = np.linalg.norm(pts[e[:, 0]] - pts[e[:, 1]], axis=1)
    be = np.array([[2.0, 1.0], [1.0, 2.0]]) / 6.0
    Mb = _coo(n, np.repeat(e, 2, axis=1).ravel(), np.tile(e, (1, 2)).ravel(),
              (L[:, None, None] * be).ravel())
    return K, M, Mb


def clean(A) -> sp.csr_matrix:
    A = sp.csr_matrix(A)
    A.sum_duplicates()
    A.eliminate_zeros()
    A.sort_indices()
    A.indices = A.indices.astype(np.int32)
    A.indptr = A.indptr.astype(np.int32)
    return A


def helmholtz_matrix(side: int, k: float) -> sp.csr_matrix:
    """A = K - k^2 M - i k M_b (complex128 CSR, sorted indices).  The stored
    pattern is the triangulation's edges plus the diagonal (the stiffness part
    of the non-edge diagonal pairs is an exact zero on this mesh and is not
    stored)."""
    K, M, Mb = matrices(side)
    A = K.astype(np.complex128) - (k * k) * M - 1j * k * Mb
    # round-off residue of K on non-edges is removed by taking the pattern of M
    A = sp.csr_matrix(A.multiply((M != 0).astype(np.float64)))
    return clean(A)


def prolongation(side_f: int) -> sp.csr_matrix:
    """Nested P1 inclusion from the mesh of (side_f + 1) / 2 points into the
    mesh of side_f points, over all vertices: a fine vertex that is a coarse
    vertex copies it, an edge midpoint takes half of each end."""
    assert side_f % 2 == 1 and side_f >= 3
    side_c = (side_f + 1) // 2
    jj, ii = np.meshgrid(np.arange(side_f), np.arange(side_f), indexing="ij")
    ii, jj = ii.ravel(), jj.ravel()
    r = jj * side_f + ii
    rows, cols = [], []
    for (ix, jx) in ((ii // 2, jj // 2), ((ii + 1) // 2, (jj + 1) // 2)):
        rows.append(r)
        cols.append(jx * side_c + ix)
    P = sp.coo_matrix((np.full(2 * len(r), 0.5), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(side_f * side_f, side_c * side_c)).tocsr()
    return clean(P)


@dataclass
class HelmholtzHierarchy:
    A: list              # [J] complex128 CSR
    P: list              # [J-1] float64 CSR, n_l x n_{l+1}
    R: list              # [J-1] P^T
    sides: list
    k: float

    @property
    def nlevels(self) -> int:
        return len(self.A)

    @property
    def sizes(self):
        return [a.shape[0] for a in self.A]

    def kh(self, l: int) -> float:
        return self.k / (self.sides[l] - 1)


def hierarchy(side: int, k: float, J: int) -> HelmholtzHierarchy:
    sides = [side]
    for _ in range(J - 1):
        assert sides[-1] % 2 == 1 and sides[-1] >= 5
        sides.append((sides[-1] + 1) // 2)
    A = [helmholtz_matrix(s, k) for s in sides]
    P = [prolongation(s) for s in sides[:-1]]
    R = [clean(p.T) for p in P]
    return HelmholtzHierarchy(A, P, R, sides, k)


def smoother_plan(h: HelmholtzHierarchy, threshold: float = 0.5, jacobi=(1, 1), gmres=(1, 2)):
    """Per level l < J-1: ("jacobi" | "gmres", nu_pre, nu_post): Jacobi where
    k h_l <= threshold, GMRES otherwise (the setting the paper takes from
    Elman, Ernst and O'Leary, 2001)."""
    out = []
    for l in range(h.nlevels - 1):
        if h.kh(l) <= threshold:
            out.append(("jacobi",) + tuple(jacobi))
        else:
            out.append(("gmres",) + tuple(gmres))
    return out


def disk_source(pts: np.ndarray, centres) -> np.ndarray:
    """100 (1 - prod_c tanh((|x - c|^2 - r_s^2) / eps_s)) at the points."""
    prod = np.ones(len(pts))
    for c in centres:
        d2 = ((pts - np.asarray(c)[None, :]) ** 2).sum(1)
        prod = prod * np.tanh((d2 - R_S * R_S) / EPS_S)
    return AMP * (1.0 - prod)


def load_vectors(side: int, columns) -> np.ndarray:
    """(n, B) complex load vectors M f_h, one per list of centres."""
    pts, _ = mesh(side)
    _, M, _ = matrices(side)
    F = np.stack([disk_source(pts, cs) for cs in columns], axis=1)
    return (M @ F).astype(np.complex128)


def source_centres(B: int, rng: np.random.Generator):
    """Column 0: the training source (centre at the origin); column 1: the
    test source (centres (0, +-0.25)); further columns: one or two disks at
    uniform random centres in [-0.35, 0.35]^2."""
    cols = [[(0.0, 0.0)], [(0.0, 0.25), (0.0, -0.25)]][:B]
    while len(cols) < B:
        m = int(rng.integers(1, 3))
        cols.append([tuple(rng.uniform(-0.35, 0.35, 2)) for _ in range(m)])
    return cols

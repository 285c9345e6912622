"""P1 finite-element assembly and nested prolongation on triangle meshes.

This module produces the linear systems A u = f that the learnable V-cycle
solves (paper, Sec. 1, eq. (linear_system)), the mesh graph the paper builds
from a triangulation (Sec. 2.1), and the natural-inclusion prolongation of a
coarse P1 space into the uniformly refined fine space (Sec. 2.2).  It holds no
arithmetic of the multigrid method itself: it only generates inputs.

Two mesh families are covered:
  * the structured "/" right-triangle mesh of the unit square (every grid cell
    split along its south-west to north-east diagonal), and
  * arbitrary triangle meshes (used for the jittered Delaunay L-shape), with
    uniform midpoint refinement.
Homogeneous Dirichlet boundary nodes are eliminated; only interior nodes are
unknowns.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

__all__ = [
    "p1_element_matrices",
    "assemble_p1",
    "square_mesh",
    "square_interior_index",
    "square_prolongation",
    "refine_uniform",
]


def p1_element_matrices(pts: np.ndarray, tris: np.ndarray, coef) -> np.ndarray:
    """Element stiffness matrices of -div(K grad u) for P1 triangles.

    pts: (nv, 2) vertex coordinates; tris: (nt, 3) vertex ids.
    coef: scalar, (nt,) per-triangle scalar a (K = a I), or a (2, 2) constant
    tensor K, or (nt, 2, 2) per-triangle tensors.
    Returns (nt, 3, 3) with entry [t, k, l] = |T| grad(phi_k)^T K grad(phi_l).
    """
    p = pts[tris]                                   # (nt, 3, 2)
    x, y = p[..., 0], p[..., 1]
    # b_k = y_{k+1} - y_{k+2}, c_k = x_{k+2} - x_{k+1};  grad phi_k = (b_k, c_k) / (2 |T|_signed)
    b = np.roll(y, -1, axis=1) - np.roll(y, -2, axis=1)
    c = np.roll(x, -2, axis=1) - np.roll(x, -1, axis=1)
    area2 = (x[:, 1] - x[:, 0]) * (y[:, 2] - y[:, 0]) - (x[:, 2] - x[:, 0]) * (y[:, 1] - y[:, 0])
    g = np.stack([b, c], axis=-1) / area2[:, None, None]          # (nt, 3, 2) gradients
    area = 0.5 * np.abs(area2)
    coef = np.asarray(coef, dtype=np.float64)
    if coef.ndim <= 1:
        a = np.broadcast_to(coef, (len(tris),))
        return (a * area)[:, None, None] * np.einsum("tkd,tld->tkl", g, g)
    Kt = np.broadcast_to(coef, (len(tris), 2, 2))
    return area[:, None, None] * np.einsum("tkd,tde,tle->tkl", g, Kt, g)


def assemble_p1(pts, tris, coef, interior: np.ndarray) -> sp.csr_matrix:
    """Assemble the global stiffness matrix restricted to interior nodes.

    interior: (nv,) integer map vertex -> unknown index, -1 for eliminated
    (Dirichlet) vertices.  Exact zeros produced by cancellation are removed, so
    the sparsity pattern is {(i, j): A_ij != 0}.
    """
    Ke = p1_element_matrices(pts, tris, coef)
    rows = np.repeat(tris, 3, axis=1)               # (nt, 9) k-major
    cols = np.tile(tris, (1, 3))
    ri, ci = interior[rows.ravel()], interior[cols.ravel()]
    keep = (ri >= 0) & (ci >= 0)
    n = int(interior.max()) + 1
    A = sp.coo_matrix((Ke.ravel()[keep], (ri[keep], ci[keep])), shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.eliminate_zeros()
    A.sort_indices()
    return A


def square_mesh(side: int):
    """Structured "/" mesh of the unit square with `side` points per direction.

    Vertex (i, j) has id j*side + i and coordinates (i h, j h), h = 1/(side-1).
    Cell (ci, cj) gives the triangles (ci,cj)-(ci+1,cj)-(ci+1,cj+1) and
    (ci,cj)-(ci+1,cj+1)-(ci,cj+1).  Returns (pts, tris, interior_map).
    """
    h = 1.0 / (side - 1)
    jj, ii = np.meshgrid(np.arange(side), np.arange(side), indexing="ij")
    pts = np.stack([ii.ravel() * h, jj.ravel() * h], axis=1)
    ci, cj = np.meshgrid(np.arange(side - 1), np.arange(side - 1), indexing="xy")
    ci, cj = ci.ravel(), cj.ravel()
    v00 = cj * side + ci
    v10 = v00 + 1
    v11 = v00 + side + 1
    v01 = v00 + side
    tris = np.concatenate([np.stack([v00, v10, v11], 1), np.stack([v00, v11, v01], 1)], axis=0)
    return pts, tris, square_interior_index(side)


def square_interior_index(side: int) -> np.ndarray:
    """Vertex -> unknown map of the square: interior (i, j) -> (j-1)*m + (i-1)."""
    m = side - 2
    idx = -np.ones((side, side), dtype=np.int64)    # [j, i]
    idx[1:-1, 1:-1] = np.arange(m * m).reshape(m, m)
    return idx.ravel()


def square_prolongation(side_f: int) -> sp.csr_matrix:
    """Natural inclusion of the coarse P1 space into the fine one on "/" meshes.

    The fine mesh (side_f points) is the uniform midpoint refinement of the
    coarse mesh (side_c = (side_f + 1) / 2 points).  A fine vertex that is a
    coarse vertex copies it; a fine vertex at the midpoint of a coarse edge
    (horizontal, vertical or "/" diagonal) takes half of each end.  Rows are
    interior fine unknowns, columns interior coarse unknowns.
    """
    assert side_f % 2 == 1 and side_f >= 5
    side_c = (side_f + 1) // 2
    fi = square_interior_index(side_f)
    ci = square_interior_index(side_c)
    rows, cols, vals = [], [], []
    jj, ii = np.meshgrid(np.arange(1, side_f - 1), np.arange(1, side_f - 1), indexing="ij")
    ii, jj = ii.ravel(), jj.ravel()
    r = fi[jj * side_f + ii]
    # the two coarse ends (equal for a coinciding vertex)
    ia, ja = ii // 2, jj // 2
    ib, jb = (ii + 1) // 2, (jj + 1) // 2
    for (ix, jx) in ((ia, ja), (ib, jb)):
        # a coinciding vertex lists the same coarse vertex twice, 1/2 each
        c = ci[jx * side_c + ix]
        ok = c >= 0
        rows.append(r[ok]); cols.append(c[ok]); vals.append(np.full(int(ok.sum()), 0.5))
    P = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(int(fi.max()) + 1, int(ci.max()) + 1)).tocsr()
    P.sum_duplicates()
    P.eliminate_zeros()
    P.sort_indices()
    return P


def refine_uniform(pts: np.ndarray, tris: np.ndarray, boundary: np.ndarray):
    """Uniform midpoint refinement of a triangle mesh.

    Each triangle is split into four through its edge midpoints.  Returns
    (pts_f, tris_f, boundary_f, parents) where parents is (nv_f, 2): a fine
    vertex equal to coarse vertex v has parents (v, v); an edge midpoint has
    the two edge ends.  boundary marks Dirichlet vertices; a midpoint is on the
    boundary when its edge is a boundary edge (used by exactly one triangle).
    """
    nv = len(pts)
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]], axis=0)
    e_sorted = np.sort(e, axis=1)
    uniq, inv, counts = np.unique(e_sorted, axis=0, return_inverse=True, return_counts=True)
    inv = inv.ravel()
    mid_id = nv + np.arange(len(uniq))
    pts_f = np.concatenate([pts, 0.5 * (pts[uniq[:, 0]] + pts[uniq[:, 1]])], axis=0)
    nt = len(tris)
    m01, m12, m20 = mid_id[inv[:nt]], mid_id[inv[nt:2 * nt]], mid_id[inv[2 * nt:]]
    v0, v1, v2 = tris[:, 0], tris[:, 1], tris[:, 2]
    tris_f = np.concatenate([
        np.stack([v0, m01, m20], 1), np.stack([m01, v1, m12], 1),
        np.stack([m20, m12, v2], 1), np.stack([m01, m12, m20], 1)], axis=0)
    bnd_edge = counts == 1
    # an edge whose both ends are boundary vertices but is interior (count 2) stays interior
    boundary_f = np.concatenate([boundary, bnd_edge])
    parents = np.concatenate([np.stack([np.arange(nv), np.arange(nv)], 1), uniq], axis=0)
    return pts_f, tris_f, boundary_f, parents


def nested_prolongation(parents: np.ndarray, interior_f: np.ndarray, interior_c: np.ndarray) -> sp.csr_matrix:
    """Prolongation from `refine_uniform` parents: weight 1/2 per parent (a vertex
    that coincides with a coarse one lists it twice, total weight 1)."""
    rows, cols = [], []
    nf = int(interior_f.max()) + 1
    nc = int(interior_c.max()) + 1
    r = interior_f
    for k in range(2):
        c = interior_c[parents[:, k]]
        ok = (r >= 0) & (c >= 0)
        rows.append(r[ok]); cols.append(c[ok])
    rows = np.concatenate(rows); cols = np.concatenate(cols)
    P = sp.coo_matrix((np.full(len(rows), 0.5), (rows, cols)), shape=(nf, nc)).tocsr()
    P.sum_duplicates()
    P.eliminate_zeros()
    P.sort_indices()
    return P

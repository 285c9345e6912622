"""Darcy single-phase flow on the unit square as input data (paper Sec. 4.1).

Pressure equation of the mixed form div u = f, u = -K grad p on a uniform
staggered grid: pressures at the centres of n x n cells, normal velocities on
the faces.  Eliminating the velocities gives the cell-centred scheme
    sum over faces  T_f (p_i - p_j) = h^2 f_i
with face transmissibility T_f the harmonic mean of the two cells' k (face
length over centre distance is 1 on a uniform grid), and on a Dirichlet face
T_f = 2 k_i (half-cell distance) with p_j replaced by g_D.  No-flow Neumann
faces contribute nothing.  The matrix is symmetric positive definite.

Coarse spaces are built by piecewise constant interpolation: the 2 x 2
aggregates of cells (the last row/column of an odd-sized grid forms
aggregates of one cell width) map to one coarse cell, P has one unit entry
per fine row, R = P^T and A_{l+1} = P^T A_l P (Galerkin), as the paper's
Darcy experiment prescribes.  Cell (i, j) (i along x) has index j * n + i.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import hierarchy as H


def cell_centres(n: int):
    h = 1.0 / n
    c = (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(c, c, indexing="xy")
    return X, Y


def inclusion_field(n: int, k_in: float = 1e-6, lo: float = 0.4, hi: float = 0.6) -> np.ndarray:
    """k = k_in on the square [lo, hi]^2, 1 elsewhere (cell centres), the
    paper's training conductivity; shape (n, n) indexed [j, i]."""
    X, Y = cell_centres(n)
    k = np.ones((n, n))
    k[(X >= lo) & (X <= hi) & (Y >= lo) & (Y <= hi)] = k_in
    return k


def two_regions_field(n: int, contrast: float = 1e4) -> np.ndarray:
    """Stand-in for the paper's test field I (two low-conductivity regions,
    contrast 1e4): rectangles [0.15,0.35]x[0.2,0.7] and [0.6,0.85]x[0.35,0.9]."""
    X, Y = cell_centres(n)
    k = np.ones((n, n))
    for (x0, x1, y0, y1) in ((0.15, 0.35, 0.2, 0.7), (0.6, 0.85, 0.35, 0.9)):
        k[(X >= x0) & (X <= x1) & (Y >= y0) & (Y <= y1)] = 1.0 / contrast
    return k


def channels_field(n: int, contrast: float = 1e6) -> np.ndarray:
    """Stand-in for test field II (two high-conductivity channels, contrast
    1e6): horizontal bands 0.25 <= y <= 0.32 and 0.62 <= y <= 0.70 at k =
    contrast, background 1."""
    X, Y = cell_centres(n)
    k = np.ones((n, n))
    for (y0, y1) in ((0.25, 0.32), (0.62, 0.70)):
        k[(Y >= y0) & (Y <= y1)] = contrast
    return k


def random_field(rng: np.random.Generator, n_coarse: int = 40, n: int = 80, decades: float = 4.0,
                 smooth: int = 3) -> np.ndarray:
    """Stand-in for test field III (a heterogeneous field given on 40 x 40 and
    interpolated to 80 x 80): log10 k from seeded normal noise on an
    n_coarse^2 grid, smoothed by `smooth` passes of a 5-point average,
    scaled to span `decades`, then copied to n x n cells (piecewise constant)."""
    z = rng.standard_normal((n_coarse, n_coarse))
    for _ in range(smooth):
        zp = np.pad(z, 1, mode="edge")
        z = (zp[1:-1, 1:-1] + zp[:-2, 1:-1] + zp[2:, 1:-1] + zp[1:-1, :-2] + zp[1:-1, 2:]) / 5.0
    z = (z - z.min()) / max(z.max() - z.min(), 1e-300) * decades - decades / 2
    rep = n // n_coarse
    return 10.0 ** np.kron(z, np.ones((rep, rep)))


def tpfa(k: np.ndarray, g_left: float = 1.0, g_right: float = 0.0, f: np.ndarray | None = None):
    """Cell-centred pressure system (A, b) for cells k[j, i] on the unit
    square: Dirichlet p = g_left at x = 0 and g_right at x = 1, no flow at
    y = 0 and y = 1, source f per cell (default 0).  b = h^2 f + boundary terms."""
    n = k.shape[0]
    assert k.shape == (n, n)
    N = n * n
    idx = np.arange(N).reshape(n, n)
    rows, cols, vals = [], [], []
    diag = np.zeros(N)
    # x faces between (j, i) and (j, i+1); y faces between (j, i) and (j+1, i)
    for a, b_ in ((idx[:, :-1], idx[:, 1:]), (idx[:-1, :], idx[1:, :])):
        ka, kb = k.ravel()[a.ravel()], k.ravel()[b_.ravel()]
        t = 2.0 * ka * kb / (ka + kb)
        rows += [a.ravel(), b_.ravel()]
        cols += [b_.ravel(), a.ravel()]
        vals += [-t, -t]
        np.add.at(diag, a.ravel(), t)
        np.add.at(diag, b_.ravel(), t)
    b = np.zeros(N) if f is None else (np.asarray(f, dtype=float).ravel() / (n * n))
    tl = 2.0 * k[:, 0]
    tr = 2.0 * k[:, -1]
    diag[idx[:, 0]] += tl
    diag[idx[:, -1]] += tr
    b[idx[:, 0]] += tl * g_left
    b[idx[:, -1]] += tr * g_right
    rows.append(np.arange(N))
    cols.append(np.arange(N))
    vals.append(diag)
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))
    return H.clean_csr(A), b


def aggregation_prolongation(n: int) -> sp.csr_matrix:
    """Piecewise constant interpolation from ceil(n/2)^2 coarse cells to n^2
    fine cells: fine cell (j, i) takes the value of coarse cell (j//2, i//2)."""
    nc = (n + 1) // 2
    j, i = np.divmod(np.arange(n * n), n)
    c = (j // 2) * nc + (i // 2)
    P = sp.csr_matrix((np.ones(n * n), (np.arange(n * n), c)), shape=(n * n, nc * nc))
    return H.clean_csr(P)


def darcy_hierarchy(k: np.ndarray, nlevels: int = 7, g_left: float = 1.0, g_right: float = 0.0):
    """(Hierarchy, b): TPFA operator of field k on the finest level,
    aggregation prolongations, R = P^T, Galerkin coarse operators."""
    A0, b = tpfa(k, g_left, g_right)
    A = [H.drop_roundoff(A0)]
    P, R = [], []
    n = k.shape[0]
    for _ in range(nlevels - 1):
        if n < 2:
            raise ValueError("grid too small for the requested number of levels")
        Pl = aggregation_prolongation(n)
        P.append(Pl)
        R.append(H.clean_csr(Pl.T))
        A.append(H.drop_roundoff(H.galerkin(A[-1], Pl)))
        n = (n + 1) // 2
    return H.Hierarchy(A, P, R, {"kind": "darcy-tpfa", "cells": k.shape[0], "interpolation": "piecewise constant"}), b

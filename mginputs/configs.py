"""Seeded synthetic workloads and parameter vectors.

Every random draw uses numpy's PCG64 through
``np.random.default_rng([workload_id, purpose, index])`` so that the CPU
oracle and the GPU path see bit-identical inputs.  Nothing here computes any
part of the multigrid method; it produces matrices, right-hand sides and
parameter vectors.

Parameter vector layout (flat float64), for levels l = 0 .. J-2 (0 = finest):
    [theta_l, eta_l, cB_l[0..KB], cR_l[0..KR], cP_l[0..KP]]
so the length is (J-1) * (2 + (KB+1) + (KR+1) + (KP+1)).  Level J-1 (the
coarsest) is solved exactly and has no parameters (paper Sec. 3, the
parameter set Theta).  The coefficients c_k weight the powers M^k of the
neighbour-mean operator M = D_g^{-1} A_g (K = 1 is SAGEConv with mean
aggregation: w1 = c_0, w2 = c_1).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import hierarchy as H

# purposes for the seed tuple
_COEF, _RHS, _PARAMS, _MESH, _ARRIVAL, _SIZE = 1, 2, 3, 4, 5, 6


def rng(workload: int, purpose: int, index: int = 0) -> np.random.Generator:
    return np.random.default_rng([workload, purpose, index])


def n_params(J: int, KB: int, KR: int, KP: int) -> int:
    return (J - 1) * (2 + (KB + 1) + (KR + 1) + (KP + 1))


def identity_params(J: int, KB: int, KR: int, KP: int, omega: float = 2.0 / 3.0) -> np.ndarray:
    """Identity initialisation: convolutions are the identity map (c_0 = 1,
    c_k = 0), theta = omega, eta = 1 (paper Sec. 3.4)."""
    per = 2 + (KB + 1) + (KR + 1) + (KP + 1)
    p = np.zeros((J - 1, per))
    p[:, 0] = omega
    p[:, 1] = 1.0
    p[:, 2] = 1.0
    p[:, 2 + KB + 1] = 1.0
    p[:, 2 + KB + 1 + KR + 1] = 1.0
    return p.ravel()


def random_params(J: int, KB: int, KR: int, KP: int, seed: int = 0, spread: float = 0.3) -> np.ndarray:
    """Random parameters near the identity initialisation (parity inputs that
    exercise every hop of every convolution)."""
    g = rng(0, _PARAMS, seed)
    p = identity_params(J, KB, KR, KP).reshape(J - 1, -1)
    p[:, 0] = g.uniform(0.5, 0.8, J - 1)
    p[:, 1] = g.uniform(0.8, 1.2, J - 1)
    for off, K in ((2, KB), (2 + KB + 1, KR), (2 + KB + 1 + KR + 1, KP)):
        p[:, off] = g.uniform(0.8, 1.2, J - 1)
        if K:
            p[:, off + 1:off + K + 1] = g.uniform(-spread, spread, (J - 1, K))
    return p.ravel()


@dataclass
class Workload:
    name: str
    hier: H.Hierarchy
    f: np.ndarray            # (n0, B) float64, row-major, B fastest
    params: np.ndarray       # flat float64
    KB: int
    KR: int
    KP: int
    nu_pre: int = 2
    nu_post: int = 2
    rtol: float = 1e-8
    precision: str = "fp64"

    @property
    def B(self) -> int:
        return self.f.shape[1]


def poisson_unit(seed: int = 0, side: int = 33, B: int = 1, K: int = 2) -> Workload:
    """2-D Poisson, P1 on the "/" mesh, h = 1/32 (961 unknowns), 4 levels,
    V(2,2), K-hop convolutions at identity initialisation with omega = 2/3,
    f ~ U(-1, 1) per node, FP64."""
    h = H.square_hierarchy(side)
    f = rng(1, _RHS, seed).uniform(-1.0, 1.0, size=(h.sizes[0], B))
    J = h.nlevels
    return Workload("poisson-33", h, f, identity_params(J, K, K, K), K, K, K, precision="fp64")


def block_diffusion(workload: int, side: int, lo: float, hi: float, B: int, seed: int = 0,
                    nblocks: int = 16, K: int = 3, precision: str = "fp32") -> Workload:
    """-div(a grad u) = f, a piecewise constant on an nblocks x nblocks array
    of square blocks with log10 a ~ U(lo, hi), f ~ N(0, 1)."""
    blocks = H.block_field(rng(workload, _COEF, seed), nblocks, lo, hi)
    h = H.square_hierarchy(side, blocks)
    f = rng(workload, _RHS, seed).standard_normal(size=(h.sizes[0], B))
    J = h.nlevels
    return Workload(f"diffusion-{side}", h, f, identity_params(J, K, K, K), K, K, K, precision=precision)


def diffusion_513(seed: int = 0, B: int = 64, K: int = 3) -> Workload:
    """513 x 513 grid (261 121 unknowns), 8 levels, log10 a ~ U(-3, 3) on 16 x 16
    blocks, 64 right-hand sides ~ N(0, 1), FP32 cycles in FP64 refinement."""
    return block_diffusion(2, 513, -3.0, 3.0, B, seed, K=K)


def training_257(seed: int = 0, B: int = 32, K: int = 3) -> Workload:
    """257 x 257 grid (65 025 unknowns), 7 levels, log10 a ~ U(-2, 2) on 16 x 16
    blocks, 32 right-hand sides ~ N(0, 1), K = 3 (84 parameters)."""
    return block_diffusion(3, 257, -2.0, 2.0, B, seed, K=K)


def lshape_aniso(seed: int = 0, B: int = 1, K: int = 3, refinements: int = 4,
                 target_nodes: int = 800) -> Workload:
    """L-shape, jittered Delaunay coarse mesh (~800 nodes) refined `refinements`
    times, anisotropic diffusion eps = 1e-3 rotated 30 degrees, f ~ U(-1, 1)."""
    h = H.lshape_hierarchy(rng(4, _MESH, seed), target_nodes, refinements)
    f = rng(4, _RHS, seed).uniform(-1.0, 1.0, size=(h.sizes[0], B))
    J = h.nlevels
    return Workload("lshape-aniso", h, f, identity_params(J, K, K, K), K, K, K, precision="fp32")


def darcy_inclusion(seed: int = 0, n: int = 100, nlevels: int = 7, B: int = 8, K: int = 3) -> tuple:
    """Darcy pressure equation (Sec. 4.1): n x n cells, k = 1e-6 on [0.4, 0.6]^2
    and 1 elsewhere, p = 1 / 0 on the left / right, no flow on top and bottom,
    f = 0, piecewise constant interpolation, Galerkin coarsening, nu = 4.
    Returns (Workload with f = the boundary right-hand side in every column,
    u0: seeded random initial iterates (n^2, B))."""
    from . import darcy as D
    h, b = D.darcy_hierarchy(D.inclusion_field(n), nlevels)
    f = np.repeat(b[:, None], B, axis=1)
    u0 = rng(9, _RHS, seed).standard_normal((h.sizes[0], B))
    w = Workload(f"darcy-{n}", h, f, identity_params(nlevels, K, K, K), K, K, K, nu_pre=4, nu_post=4,
                 precision="fp32")
    return w, u0


SERVING_SIDES = (65, 129, 257, 513, 1025)


def serving_request(index: int, stream_seed: int = 0, sides=SERVING_SIDES):
    """Request `index` of a serving stream: (side, blocks, f) with side uniform
    over `sides`, log10 a ~ U(-2, 2) on 16 x 16 blocks, f ~ N(0, 1)."""
    side = int(sides[rng(5, _SIZE, stream_seed * 1_000_003 + index).integers(len(sides))])
    blocks = H.block_field(rng(5, _COEF, stream_seed * 1_000_003 + index), 16, -2.0, 2.0)
    return side, blocks


def serving_rhs(index: int, n: int, stream_seed: int = 0) -> np.ndarray:
    return rng(5, _RHS, stream_seed * 1_000_003 + index).standard_normal(size=(n, 1))


def serving_arrivals(count: int, qps: float, stream_seed: int = 0) -> np.ndarray:
    """Poisson arrivals: cumulative sums of exponential gaps with mean 1/qps."""
    gaps = rng(5, _ARRIVAL, stream_seed).exponential(1.0 / qps, size=count)
    return np.cumsum(gaps)


# ----------------------------------------------------------------------------- Helmholtz (two features)
@dataclass
class HelmholtzWorkload:
    name: str
    hier: object             # helmholtz.HelmholtzHierarchy
    f: np.ndarray            # (n0, B) complex128
    params: np.ndarray       # flat float64, layout of hz_n_params
    KB: int
    KR: int
    KP: int
    plan: list               # [J-1] (kind, nu_pre, nu_post)
    v: int = 4               # GMRES steps of a GMRES smoothing step
    rtol: float = 1e-8

    @property
    def B(self) -> int:
        return self.f.shape[1]


def hz_n_params(J: int, KB: int, KR: int, KP: int) -> int:
    """Per level l < J-1: [theta_l, eta_l, W_B,l[0..KB] (2 x 2 row-major)];
    then the shared W_R[0..KR] and W_P[0..KP]."""
    return (J - 1) * (2 + 4 * (KB + 1)) + 4 * (KR + 1) + 4 * (KP + 1)


def hz_identity_params(J: int, KB: int, KR: int, KP: int, plan, omega: float = 2.0 / 3.0) -> np.ndarray:
    """Identity initialisation with two features: W_0 = I, W_k = 0 (k > 0),
    eta = 1; theta = omega on Jacobi levels and 0 on GMRES levels (a GMRES
    smoothing step then starts from zero: the classical GMRES smoother)."""
    per = 2 + 4 * (KB + 1)
    lv = np.zeros((J - 1, per))
    for l in range(J - 1):
        lv[l, 0] = omega if plan[l][0] == "jacobi" else 0.0
        lv[l, 1] = 1.0
        lv[l, 2:6] = (1.0, 0.0, 0.0, 1.0)
    sh = np.zeros(4 * (KR + 1) + 4 * (KP + 1))
    sh[0:4] = (1.0, 0.0, 0.0, 1.0)
    sh[4 * (KR + 1):4 * (KR + 1) + 4] = (1.0, 0.0, 0.0, 1.0)
    return np.concatenate([lv.ravel(), sh])


def hz_random_params(J: int, KB: int, KR: int, KP: int, plan, seed: int = 0, spread: float = 0.2) -> np.ndarray:
    """Random parameters near the identity initialisation, with off-diagonal
    (real/imaginary mixing) entries in every weight matrix."""
    g = rng(10, _PARAMS, seed)
    per = 2 + 4 * (KB + 1)
    lv = np.zeros((J - 1, per))
    for l in range(J - 1):
        lv[l, 0] = g.uniform(0.5, 0.8) if plan[l][0] == "jacobi" else g.uniform(0.1, 0.6)
        lv[l, 1] = g.uniform(0.8, 1.2)
        W = g.uniform(-spread, spread, (KB + 1, 2, 2))
        W[0] += np.eye(2)
        lv[l, 2:] = W.ravel()
    WR = g.uniform(-spread, spread, (KR + 1, 2, 2))
    WR[0] += np.eye(2)
    WP = g.uniform(-spread, spread, (KP + 1, 2, 2))
    WP[0] += np.eye(2)
    return np.concatenate([lv.ravel(), WR.ravel(), WP.ravel()])


def helmholtz(side: int = 257, k: float = 16.0 * np.pi, J: int = 5, B: int = 16, K: int = 1, seed: int = 0,
              v: int = 4) -> HelmholtzWorkload:
    """Impedance Helmholtz on [-1/2, 1/2]^2 (the "/" P1 mesh with `side`
    points per direction, every vertex an unknown), J levels, smoothed-disk
    sources (column 0 the training source, column 1 the test source, the rest
    at seeded random centres), Jacobi V(1,1) where k h_l <= 0.5 and GMRES(v)
    V(1,2) elsewhere, convolutions of order K at identity initialisation.
    Default: k = 16 pi, h = 1/256 (66 049 unknowns, k h = 0.196), 5 levels."""
    from . import helmholtz as HZ
    h = HZ.hierarchy(side, k, J)
    plan = HZ.smoother_plan(h)
    f = HZ.load_vectors(side, HZ.source_centres(B, rng(10, _RHS, seed)))
    return HelmholtzWorkload(f"helmholtz-{side}", h, f, hz_identity_params(J, K, K, K, plan), K, K, K, plan, v)

"""Trainable parameterisations of Theta -- TEST INFRASTRUCTURE ONLY.

Sec. 4.1 (Darcy experiment) shares one restriction convolution and one
prolongation convolution between all levels (Phi_R,l = Phi_R, Phi_P,l = Phi_P)
and trains two subsets: LMG-RP (only Phi_R, Phi_P; the smoother stays damped
Jacobi) and LMG-RPS (Phi_R, Phi_P, the smoothers Phi_B,l and the scales eta_l;
theta_l fixed).  "full" trains every level's own parameters; "shared" ties
Phi_R/Phi_P and trains everything else per level.

Written out level by level in plain Python; the per-level layout is the
oracle's OParams (theta, eta, cB, cR, cP).  Independent of the HIP package.
"""
from __future__ import annotations

import numpy as np

from .lmg import OParams


def _split_sizes(name, J, KB, KR, KP):
    L = J - 1
    if name == "full":
        return None
    per_level = {"shared": 2 + KB + 1, "rps": 1 + KB + 1, "rp": 0}[name]
    return L, per_level


def expand(name: str, phi, J: int, KB: int, KR: int, KP: int, omega: float = 2.0 / 3.0,
           nu_pre: int = 2, nu_post: int = 2) -> OParams:
    """Per-level parameters from the trainable vector phi (see module doc).
    Order of phi: per level its own entries (shared: theta, eta, cB; rps: eta,
    cB), then cR, then cP; "full" is the per-level layout itself."""
    phi = np.asarray(phi, dtype=np.float64)
    L = J - 1
    if name == "full":
        per = 2 + KB + 1 + KR + 1 + KP + 1
        p = phi.reshape(L, per)
        return OParams(p[:, 0].copy(), p[:, 1].copy(), p[:, 2:3 + KB].copy(), p[:, 3 + KB:4 + KB + KR].copy(),
                       p[:, 4 + KB + KR:].copy(), nu_pre, nu_post)
    _, npl = _split_sizes(name, J, KB, KR, KP)
    theta = np.full(L, omega)
    eta = np.ones(L)
    cB = np.zeros((L, KB + 1))
    cB[:, 0] = 1.0
    pos = 0
    for l in range(L):
        if name == "shared":
            theta[l] = phi[pos]
            eta[l] = phi[pos + 1]
            cB[l] = phi[pos + 2:pos + 3 + KB]
            pos += 3 + KB
        elif name == "rps":
            eta[l] = phi[pos]
            cB[l] = phi[pos + 1:pos + 2 + KB]
            pos += 2 + KB
    cR_shared = phi[pos:pos + KR + 1]
    pos += KR + 1
    cP_shared = phi[pos:pos + KP + 1]
    pos += KP + 1
    assert pos == phi.size, "phi has the wrong length"
    cR = np.array([cR_shared for _ in range(L)])
    cP = np.array([cP_shared for _ in range(L)])
    return OParams(theta, eta, cB, cR, cP, nu_pre, nu_post)  # monomial basis


def grad_phi(name: str, g: OParams, J: int, KB: int, KR: int, KP: int) -> np.ndarray:
    """dL/dphi from the per-level gradient g (chain rule through expand: a
    shared convolution's gradient is the sum of its per-level gradients;
    fixed entries get none)."""
    L = J - 1
    if name == "full":
        return np.concatenate([g.theta[:, None], g.eta[:, None], g.cB, g.cR, g.cP], axis=1).ravel()
    out = []
    for l in range(L):
        if name == "shared":
            out += [g.theta[l], g.eta[l], *g.cB[l]]
        elif name == "rps":
            out += [g.eta[l], *g.cB[l]]
    out += list(np.sum(g.cR, axis=0))
    out += list(np.sum(g.cP, axis=0))
    return np.array(out)

"""Parameter vectors Theta: layout, identity initialisation, level mapping,
trainable parameterisations, files.

Layout (flat float64), per level l = 0 .. J-2 (0 = finest):
    [theta_l, eta_l, cB_l[0..KB], cR_l[0..KR], cP_l[0..KP]]
"""
from __future__ import annotations

import json
import os

import numpy as np


def per_level(KB: int, KR: int, KP: int) -> int:
    return 2 + (KB + 1) + (KR + 1) + (KP + 1)


def identity(J: int, KB: int, KR: int, KP: int, omega: float = 2.0 / 3.0) -> np.ndarray:
    """Identity initialisation: theta = omega, eta = 1, every convolution the
    identity map (paper Sec. 3.4); equals the classical V-cycle."""
    p = np.zeros((J - 1, per_level(KB, KR, KP)))
    p[:, 0] = omega
    p[:, 1] = 1.0
    p[:, 2] = 1.0
    p[:, 2 + KB + 1] = 1.0
    p[:, 2 + KB + 1 + KR + 1] = 1.0
    return p.ravel()


def map_levels(theta: np.ndarray, J_src: int, J_dst: int, KB: int, KR: int, KP: int,
               shift: int = 0) -> np.ndarray:
    """Transfer parameters trained on a J_src-level hierarchy to J_dst levels.

    Target level l takes source level l + shift, clamped to the source's
    parameterised levels: shift = 0 aligns the finest levels, and a target
    level past the deepest source level copies it (the partial-transfer rule
    of Sec. 4.2.3: extra coarse levels copy the deepest compatible source
    weights).  With shift = J_src - J_dst on nested grids levels of equal mesh
    size are matched (the paper matches levels by a mesh-size criterion).
    """
    per = per_level(KB, KR, KP)
    src = np.asarray(theta, dtype=np.float64).reshape(J_src - 1, per)
    out = np.empty((J_dst - 1, per))
    for l in range(J_dst - 1):
        out[l] = src[min(max(l + shift, 0), J_src - 2)]
    return out.ravel()


VARIANTS = ("full", "shared", "rp", "rps")


class Variant:
    """A trainable parameterisation Theta = E phi + t of the per-level layout.

      full    every entry of Theta is trained
      shared  Phi_R and Phi_P are one convolution each for all levels
              (Phi_R,l = Phi_R, Phi_P,l = Phi_P; Sec. 4.1); theta_l, eta_l and
              Phi_B,l per level:  phi = [(theta_l, eta_l, cB_l) for l] + cR + cP
      rp      LMG-RP (Sec. 4.1): only the shared Phi_R, Phi_P are trained; the
              smoother is damped Jacobi (theta = omega, eta = 1, Phi_B = I):
              phi = cR + cP
      rps     LMG-RPS (Sec. 4.1): the shared Phi_R, Phi_P, and per level
              Phi_B,l and eta_l are trained, theta_l = omega is fixed:
              phi = [(eta_l, cB_l) for l] + cR + cP
    E is a 0/1 matrix, so dL/dphi = E^T dL/dTheta (tied entries add up).
    """

    def __init__(self, name: str, J: int, KB: int, KR: int, KP: int, omega: float = 2.0 / 3.0):
        if name not in VARIANTS:
            raise ValueError(f"unknown variant {name!r}; one of {VARIANTS}")
        self.name, self.J, self.KB, self.KR, self.KP, self.omega = name, J, KB, KR, KP, omega
        per = per_level(KB, KR, KP)
        L = J - 1
        oB, oR, oP = 2, 2 + KB + 1, 2 + KB + 1 + KR + 1
        rows, cols = [], []
        t = identity(J, KB, KR, KP, omega).reshape(L, per)
        fixed = np.ones((L, per), dtype=bool)
        col = 0

        def tie(level_entries):
            nonlocal col
            for (l, e) in level_entries:
                rows.append(l * per + e)
                cols.append(col)
                fixed[l, e] = False
            col += 1

        if name == "full":
            for l in range(L):
                for e in range(per):
                    tie([(l, e)])
        else:
            for l in range(L):
                if name == "shared":
                    tie([(l, 0)])
                if name in ("shared", "rps"):
                    tie([(l, 1)])
                    for k in range(KB + 1):
                        tie([(l, oB + k)])
            for k in range(KR + 1):
                tie([(l, oR + k) for l in range(L)])
            for k in range(KP + 1):
                tie([(l, oP + k) for l in range(L)])
        self.nphi = col
        self.E = np.zeros((L * per, col))
        self.E[rows, cols] = 1.0
        self.t = np.where(fixed, t, 0.0).ravel()

    def expand(self, phi):
        """Theta = E phi + t (numpy array or torch tensor; differentiable)."""
        if isinstance(phi, np.ndarray):
            return self.E @ phi + self.t
        import torch
        return torch.as_tensor(self.E, dtype=phi.dtype) @ phi + torch.as_tensor(self.t, dtype=phi.dtype)

    def initial(self, theta=None) -> np.ndarray:
        """phi whose expansion is theta (default: the identity initialisation),
        taking each tied group's mean."""
        theta = identity(self.J, self.KB, self.KR, self.KP, self.omega) if theta is None else np.asarray(theta)
        cnt = self.E.sum(axis=0)
        return (self.E.T @ theta) / cnt


_HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULTS = {("diffusion-513", 3): "k3_diffusion513.npy", ("training-257", 3): "k3_diffusion257_4fields.npy"}
for _side in (65, 129, 257, 513, 1025):
    DEFAULTS[(f"serving-{_side}", 3)] = f"k3_serving{_side}.npy"
DEFAULTS[("darcy-100-rp", 3)] = "k3_darcy100_rp.npy"
DEFAULTS[("darcy-100-rps", 3)] = "k3_darcy100_rps.npy"


def default_file(workload: str, K: int):
    """Shipped parameters trained with this package for a workload, or None."""
    name = DEFAULTS.get((workload, K))
    if name is None:
        return None
    path = os.path.join(_HERE, "theta", name)
    return path if os.path.exists(path) else None


def save(path: str, theta: np.ndarray, meta: dict):
    np.save(path, np.asarray(theta, dtype=np.float64))
    with open(path[:-4] + ".json" if path.endswith(".npy") else path + ".json", "w") as fh:
        json.dump(meta, fh, indent=1)


def load(path: str):
    theta = np.load(path, allow_pickle=False)
    meta_path = path[:-4] + ".json" if path.endswith(".npy") else path + ".json"
    with open(meta_path) as fh:
        meta = json.load(fh)
    return theta, meta

"""Parameter vectors Theta: layout, identity initialisation, level mapping, files.

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
    of Sec. 4.2.4: extra coarse levels copy the deepest compatible source
    weights).  With shift = J_src - J_dst on nested grids levels of equal mesh
    size are matched (the paper matches levels by a mesh-size criterion).
    """
    per = per_level(KB, KR, KP)
    src = np.asarray(theta, dtype=np.float64).reshape(J_src - 1, per)
    out = np.empty((J_dst - 1, per))
    for l in range(J_dst - 1):
        out[l] = src[min(max(l + shift, 0), J_src - 2)]
    return out.ravel()


_HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULTS = {("diffusion-513", 3): "k3_diffusion513.npy", ("training-257", 3): "k3_diffusion257_4fields.npy"}
for _side in (65, 129, 257, 513, 1025):
    DEFAULTS[(f"serving-{_side}", 3)] = f"k3_serving{_side}.npy"


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

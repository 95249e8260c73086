"""Shared helpers of the GPU parity tests (not collected by pytest)."""
import functools

import numpy as np

from oracle import csgd, sampler, siddon
from paper_1709_00953_amd import inputs

TAU_REL = 1e-5      # nnz threshold, fraction of the smallest voxel pitch


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def tau_for(g) -> float:
    return TAU_REL * min(g.vx, g.vy, g.vz if g.is3d else g.vx)


# Parity-scale workloads: small enough for the oracle to finish in seconds,
# large enough to span several back-projection tiles and forward chunks, with
# ragged block edges.
def geom_c1():
    return inputs.config_c1()


def geom_fan_curved():
    return inputs.fan2d(100, 2.56, 120, 160, 4e-3, 500.0, 1000.0, m=6, bx=3, by=2)


def geom_fan_flat():
    return inputs.fan2d(90, 2.8, 90, 170, 4e-3, 500.0, 1000.0, m=5, bx=2, by=3, curved=False,
                        pu_flat=3.2)


def geom_cone():
    return inputs.cone3d(40, 3.2, 120, 60, 6.4, 500.0, 1000.0, m=6, bz=3, bxy=2)


GEOMS = {"c1_par2d": geom_c1, "fan_curved": geom_fan_curved, "fan_flat": geom_fan_flat,
         "cone": geom_cone}


@functools.lru_cache(maxsize=8)
def system(name):
    g = GEOMS[name]()
    return g, csgd.BlockSystem(siddon.system_matrix(g), g)


def phantom_y(g, S, seed, noise=0.01):
    """x_true and y = A_oracle x_true + N(0, (noise max y)^2), float32."""
    x = inputs.phantom_for(g, seed)
    p = S.A @ x
    y = inputs.gaussian_noise(p, noise, seed) if noise > 0 else p.astype(np.float32)
    return x, y

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


def max_rel(a, b) -> float:
    """Element-wise error: max_i |a_i - b_i| / max_i |b_i|."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    mb = float(np.max(np.abs(b))) if b.size else 0.0
    d = float(np.max(np.abs(a - b))) if b.size else 0.0
    return d / mb if mb > 0 else d


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


# Fine pixels on a curved fan (0.5 mm voxels, 1e-3 rad bins, source at
# 500 mm): every view's candidate bins lie within 2e-2 rad of a bin near the
# tile's shadow, so the back-projection forms its ray distances in float32
# in that bin's frame; the coarser fans here keep the float64 form.
def geom_fan_fine():
    return inputs.fan2d(64, 0.5, 120, 96, 1e-3, 500.0, 1000.0, m=6, bx=3, by=2)


def geom_cone():
    return inputs.cone3d(40, 3.2, 120, 60, 6.4, 500.0, 1000.0, m=6, bz=3, bxy=2)


# Rays on voxel faces: odd detectors whose central bin looks through the
# rotation centre, which is a grid corner of an even voxel grid, with views at
# quarter turns.  Parallel rays at every integer offset lie on faces there; in
# the cone the central detector row lies in the face plane z = 0 and the
# central ray runs along an edge.  The diagonal views pass through corners.
def geom_par_axis():
    return inputs.par2d(32, 1.0, 8, 360.0, 47, 1.0, m=4, bx=2, by=2)


def geom_fan_axis():
    return inputs.fan2d(40, 1.0, 8, 61, 8e-3, 100.0, 200.0, m=4, bx=2, by=2)


def geom_fan_flat_axis():
    return inputs.fan2d(40, 1.0, 8, 61, 8e-3, 100.0, 200.0, m=4, bx=2, by=2, curved=False,
                        pu_flat=1.0)


def geom_cone_axis():
    return inputs.cone3d(24, 1.0, 8, 41, 1.0, 100.0, 200.0, m=4, bz=2, bxy=2)


# Row blocks that cut each view group's detector into sub-areas (several row
# blocks per projection, as in the paper's 2D layout).
def geom_fan_split():
    return inputs.fan2d(100, 2.56, 120, 160, 4e-3, 500.0, 1000.0, m=3, bx=3, by=2, u_split=3)


def geom_cone_split():
    return inputs.cone3d(40, 3.2, 120, 60, 6.4, 500.0, 1000.0, m=3, bz=3, bxy=2, v_split=2, u_split=2)


GEOMS = {"c1_par2d": geom_c1, "fan_curved": geom_fan_curved, "fan_fine": geom_fan_fine,
         "fan_flat": geom_fan_flat, "fan_split": geom_fan_split, "cone_split": geom_cone_split,
         "cone": geom_cone, "par_axis": geom_par_axis, "fan_axis": geom_fan_axis,
         "fan_flat_axis": geom_fan_flat_axis, "cone_axis": geom_cone_axis}


@functools.lru_cache(maxsize=len(GEOMS))
def system(name):
    g = GEOMS[name]()
    return g, csgd.BlockSystem(siddon.system_matrix(g), g)


def phantom_y(g, S, seed, noise=0.01):
    """x_true and y = A_oracle x_true + N(0, (noise max y)^2), float32.  The
    parallel-beam case takes 10 ellipses (the small parallel workload), the
    other 2D cases 12 and the cones 20 ellipsoids."""
    x = inputs.phantom_for(g, seed, n_ell=10 if g.kind == inputs.PAR2D else None)
    p = S.A @ x
    y = inputs.gaussian_noise(p, noise, seed) if noise > 0 else p.astype(np.float32)
    return x, y

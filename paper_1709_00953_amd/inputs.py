"""Seeded synthetic workloads for the block-iterative CT solver.

This module only builds *inputs*: scan geometries (per-view source/detector
vectors), the row/column block partitions of Eq. (4) and the tomographic
decomposition of Sec. II-D (detector tiles per view, voxel cuboids), random
ellipse/ellipsoid phantoms and noise.  It holds none of the method's
arithmetic (no projection, no step, no sampling), so both the FP64 oracle and
the HIP path can consume it.

Geometry convention (shared definition, implemented separately by the oracle
and by the library):

* ``kind``: 0 = parallel 2D, 1 = fan 2D flat detector, 2 = fan 2D curved
  (equiangular) detector, 3 = cone 3D flat detector.
* ``views``: float64 array ``[n_views, 12]`` = ``a | c | e_u | e_v`` where
  ``a`` is the ray direction (parallel) or the source position (divergent),
  ``c`` the detector centre, ``e_u``/``e_v`` unit detector axes.
* bin ``iu`` sits at ``u = (iu - (nu-1)/2) * pu`` (mm, or radians for the
  curved detector), ``iv`` likewise along ``e_v``.
* ray index ``i = (view * nv + iv) * nu + iu``; voxel index
  ``j = (iz * ny + iy) * nx + ix``; voxel boxes are half-open.
* A row block is a list of tiles ``(view, u0, u1, v0, v1)``; a column block is
  a voxel box ``(x0, x1, y0, y1, z0, z1)`` (index ranges, half-open).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Tuple

import numpy as np

PAR2D, FAN2D_FLAT, FAN2D_CURVED, CONE3D_FLAT = 0, 1, 2, 3
KIND_NAMES = {PAR2D: "par2d", FAN2D_FLAT: "fan2d_flat",
              FAN2D_CURVED: "fan2d_curved", CONE3D_FLAT: "cone3d_flat"}


@dataclasses.dataclass
class Geometry:
    kind: int
    nx: int
    ny: int
    nz: int
    vx: float
    vy: float
    vz: float
    ox: float
    oy: float
    oz: float
    nu: int
    nv: int
    pu: float
    pv: float
    views: np.ndarray                       # [n_views, 12] float64
    row_blocks: List[np.ndarray]            # each [n_tiles, 5] int32
    col_blocks: np.ndarray                  # [n, 6] int32

    @property
    def n_views(self) -> int:
        return int(self.views.shape[0])

    @property
    def n_rays(self) -> int:
        return self.n_views * self.nu * self.nv

    @property
    def n_vox(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def m(self) -> int:
        return len(self.row_blocks)

    @property
    def n(self) -> int:
        return int(self.col_blocks.shape[0])

    @property
    def is3d(self) -> bool:
        return self.kind == CONE3D_FLAT

    def row_block_rays(self, b: int) -> np.ndarray:
        """Global ray indices of row block ``b`` in tile order, u fastest."""
        out = []
        for (v, u0, u1, v0, v1) in self.row_blocks[b]:
            iv = np.arange(v0, v1)
            iu = np.arange(u0, u1)
            out.append(((v * self.nv + iv[:, None]) * self.nu + iu[None, :]).ravel())
        return np.concatenate(out) if out else np.zeros(0, np.int64)

    def col_block_vox(self, b: int) -> np.ndarray:
        """Global voxel indices of column block ``b`` (x fastest)."""
        x0, x1, y0, y1, z0, z1 = (int(t) for t in self.col_blocks[b])
        iz, iy, ix = np.meshgrid(np.arange(z0, z1), np.arange(y0, y1),
                                 np.arange(x0, x1), indexing="ij")
        return ((iz * self.ny + iy) * self.nx + ix).ravel()


# ----------------------------------------------------------------------------
# scan trajectories
# ----------------------------------------------------------------------------

def _cos_sin(thetas):
    """cos and sin of view angles, exact at quarter turns: float64 leaves
    residues such as cos(pi/2) = 6e-17 there, which would tilt a ray that runs
    along a voxel face by that much and split it between two voxel columns."""
    c, s = np.cos(thetas), np.sin(thetas)
    c[np.abs(c) < 1e-12] = 0.0
    s[np.abs(s) < 1e-12] = 0.0
    return c, s


def _par2d_views(thetas):
    v = np.zeros((len(thetas), 12))
    c, s = _cos_sin(thetas)
    v[:, 0], v[:, 1] = -s, c              # ray direction
    v[:, 6], v[:, 7] = c, s               # detector axis, detector centre at 0
    return v


def _circular_views(thetas, sid, sdd, third_axis=False):
    v = np.zeros((len(thetas), 12))
    c, s = _cos_sin(thetas)
    v[:, 0], v[:, 1] = sid * c, sid * s               # source
    v[:, 3], v[:, 4] = -(sdd - sid) * c, -(sdd - sid) * s  # detector centre
    v[:, 6], v[:, 7] = -s, c                          # e_u
    if third_axis:
        v[:, 11] = 1.0                                # e_v = z
    return v


def sphere_views(n_views, radius, sdd, seed):
    """Random source positions on a sphere (the paper's 3D trajectory, Sec. III-E).

    Detector plane perpendicular to the source-centre line, centre at distance
    ``sdd`` from the source on the far side of the rotation centre.
    """
    rng = np.random.default_rng(seed)
    a = np.arccos(rng.uniform(-1.0, 1.0, n_views))
    b = rng.uniform(0.0, 2 * np.pi, n_views)
    src = radius * np.stack([np.sin(a) * np.cos(b), np.sin(a) * np.sin(b), np.cos(a)], 1)
    n = -src / radius
    ref = np.where(np.abs(n[:, 2:3]) < 0.9, np.array([[0, 0, 1.0]]), np.array([[1.0, 0, 0]]))
    eu = np.cross(n, ref)
    eu /= np.linalg.norm(eu, axis=1, keepdims=True)
    ev = np.cross(n, eu)
    v = np.zeros((n_views, 12))
    v[:, 0:3] = src
    v[:, 3:6] = src + sdd * n
    v[:, 6:9] = eu
    v[:, 9:12] = ev
    return v


# ----------------------------------------------------------------------------
# partitions (Sec. II-D): row blocks = detector tiles of view groups,
# column blocks = voxel cuboids
# ----------------------------------------------------------------------------

def angle_group_blocks(n_views, m, nu, nv, u_split=1, v_split=1):
    """m contiguous view groups (sizes differ by at most one, larger first),
    each optionally crossed with a u_split x v_split detector split."""
    base, extra = divmod(n_views, m)
    sizes = [base + (1 if k < extra else 0) for k in range(m)]
    ub = np.linspace(0, nu, u_split + 1).round().astype(int)
    vb = np.linspace(0, nv, v_split + 1).round().astype(int)
    blocks = []
    start = 0
    for sz in sizes:
        views = range(start, start + sz)
        start += sz
        for a in range(v_split):
            for b in range(u_split):
                blocks.append(np.array([[v, ub[b], ub[b + 1], vb[a], vb[a + 1]] for v in views],
                                       dtype=np.int32))
    return blocks


def detector_area_blocks(n_views, nu, nv, u_split):
    """One row block per (view, detector sub-area): the paper's 2D layout."""
    ub = np.linspace(0, nu, u_split + 1).round().astype(int)
    return [np.array([[v, ub[b], ub[b + 1], 0, nv]], dtype=np.int32)
            for v in range(n_views) for b in range(u_split)]


def box_blocks(nx, ny, nz, sx, sy, sz):
    xb = np.linspace(0, nx, sx + 1).round().astype(int)
    yb = np.linspace(0, ny, sy + 1).round().astype(int)
    zb = np.linspace(0, nz, sz + 1).round().astype(int)
    out = []
    for c in range(sz):
        for b in range(sy):
            for a in range(sx):
                out.append([xb[a], xb[a + 1], yb[b], yb[b + 1], zb[c], zb[c + 1]])
    return np.array(out, dtype=np.int32)


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

def par2d(n=64, pitch=1.0, n_views=90, span_deg=180.0, nu=96, pu=1.0, m=4, bx=2, by=2):
    """Parallel-beam 2D: theta_k = span*k/n_views, rays through u_b*(cos, sin)."""
    th = np.deg2rad(span_deg) * np.arange(n_views) / n_views
    half = n * pitch / 2
    return Geometry(PAR2D, n, n, 1, pitch, pitch, 1.0, -half, -half, 0.0,
                    nu, 1, pu, 1.0, _par2d_views(th),
                    angle_group_blocks(n_views, m, nu, 1), box_blocks(n, n, 1, bx, by, 1))


def fan2d(n=512, pitch=0.5, n_views=720, nu=768, dgamma=1e-3, sid=500.0, sdd=1000.0,
          m=8, bx=4, by=2, curved=True, span_deg=360.0, u_split=1, pu_flat=None):
    th = np.deg2rad(span_deg) * np.arange(n_views) / n_views
    half = n * pitch / 2
    views = _circular_views(th, sid, sdd)
    if curved:
        kind, pu = FAN2D_CURVED, dgamma
    else:
        kind, pu = FAN2D_FLAT, (pu_flat if pu_flat is not None else dgamma * sdd)
    return Geometry(kind, n, n, 1, pitch, pitch, 1.0, -half, -half, 0.0,
                    nu, 1, pu, 1.0, views,
                    angle_group_blocks(n_views, m, nu, 1, u_split=u_split),
                    box_blocks(n, n, 1, bx, by, 1))


def cone3d(n=256, pitch=0.5, n_views=360, nd=384, pd=1.0, sid=500.0, sdd=1000.0,
           m=12, bz=8, bxy=1, span_deg=360.0, u_split=1, v_split=1):
    th = np.deg2rad(span_deg) * np.arange(n_views) / n_views
    half = n * pitch / 2
    return Geometry(CONE3D_FLAT, n, n, n, pitch, pitch, pitch, -half, -half, -half,
                    nd, nd, pd, pd, _circular_views(th, sid, sdd, third_axis=True),
                    angle_group_blocks(n_views, m, nd, nd, u_split=u_split, v_split=v_split),
                    box_blocks(n, n, n, bxy, bxy, bz))


# Configurations of the benchmark suite.
def config_c1():
    """2D parallel, 64^2 at 1 mm, 90 views over [0,180), 96 bins at 1 mm;
    4 angle groups x 4 quadrants."""
    return par2d(64, 1.0, 90, 180.0, 96, 1.0, m=4, bx=2, by=2)


def config_c2():
    """2D fan, curved detector, 512^2 at 0.5 mm, 720 views over 360 deg,
    768 bins at 1e-3 rad, SID 500 / SDD 1000; 8 angle groups x 8 tiles."""
    return fan2d(512, 0.5, 720, 768, 1e-3, 500.0, 1000.0, m=8, bx=4, by=2)


def config_p2():
    """Parity-scale C2: 128^2 at 2 mm, 180 views, 192 bins at 4e-3 rad."""
    return fan2d(128, 2.0, 180, 192, 4e-3, 500.0, 1000.0, m=8, bx=4, by=2)


def config_c3():
    """3D cone, 256^3 at 0.5 mm, 360 views of 384^2 at 1 mm;
    12 projection groups x 8 z-slabs."""
    return cone3d(256, 0.5, 360, 384, 1.0, 500.0, 1000.0, m=12, bz=8)


def config_p3():
    """Parity-scale C3: 48^3 at 128/48 mm, 360 views of 72^2 at 256/48 mm."""
    return cone3d(48, 128.0 / 48, 360, 72, 256.0 / 48, 500.0, 1000.0, m=12, bz=8)


def config_paper2d():
    """The paper's 2D setting (Sec. III): 64^2 pixels of 1, flat 187-pixel
    detector of spacing 1, source and detector centre on circles of radius
    115 (SDD 230), 360 views over 360 degrees; one row block per (view,
    detector half), 720 in all; 2 x 2 image quadrants."""
    n_views, nu = 360, 187
    th = np.deg2rad(360.0) * np.arange(n_views) / n_views
    return Geometry(FAN2D_FLAT, 64, 64, 1, 1.0, 1.0, 1.0, -32.0, -32.0, 0.0,
                    nu, 1, 1.0, 1.0, _circular_views(th, 115.0, 230.0),
                    detector_area_blocks(n_views, nu, 1, 2), box_blocks(64, 64, 1, 2, 2, 1))


def config_paper3d(n=128, nd=202, n_views=720, seed=5300):
    """The paper's 3D setting (Sec. III-E): n^3 voxels over a 32^3 volume, a
    square detector of side 101 (nd x nd pixels), 720 source positions drawn
    at random on a sphere of radius 66, detector plane perpendicular at
    distance 132; every projection one row block (no detector split) x
    2 x 2 x 2 volume blocks."""
    pitch, pd = 32.0 / n, 101.0 / nd
    half = 16.0
    return Geometry(CONE3D_FLAT, n, n, n, pitch, pitch, pitch, -half, -half, -half,
                    nd, nd, pd, pd, sphere_views(n_views, 66.0, 132.0, seed),
                    detector_area_blocks(n_views, nd, nd, 1), box_blocks(n, n, n, 2, 2, 2))


def slice_fan(nn: int, m=4, bx=2, by=2):
    """Batched/served 2D slice of size nn: pixel 256/nn mm, 1.5*nn views over
    360 deg, 1.5*nn bins spanning 0.768 rad."""
    nvw = int(round(1.5 * nn))
    return fan2d(nn, 256.0 / nn, nvw, nvw, 0.768 / nvw, 500.0, 1000.0, m=m, bx=bx, by=by)


def slice_cone(nn: int, m=12, bz=8):
    """Served 3D job: nn^3 voxels at 128/nn mm, 360 views of (1.5 nn)^2 at 256/nn mm."""
    nd = int(round(1.5 * nn))
    return cone3d(nn, 128.0 / nn, 360, nd, 256.0 / nn, 500.0, 1000.0, m=m, bz=bz)


# ----------------------------------------------------------------------------
# phantoms and noise
# ----------------------------------------------------------------------------

def ellipse_phantom(geom: Geometry, n_ell: int, seed: int, scale: float = 0.1) -> np.ndarray:
    """Sum of random ellipses sampled at pixel centres (values in mm^-1).

    Centres U[-0.7, 0.7], semi-axes U[0.05, 0.4] (fractions of the half field
    of view), attenuation U[0.1, 1.0] * ``scale``, rotation U[0, pi).
    """
    rng = np.random.default_rng(seed)
    half = 0.5 * geom.nx * geom.vx
    cx = geom.ox + (np.arange(geom.nx) + 0.5) * geom.vx
    cy = geom.oy + (np.arange(geom.ny) + 0.5) * geom.vy
    X, Y = np.meshgrid(cx, cy, indexing="xy")
    img = np.zeros((geom.ny, geom.nx))
    for _ in range(n_ell):
        x0, y0 = rng.uniform(-0.7, 0.7, 2) * half
        a, b = rng.uniform(0.05, 0.4, 2) * half
        val = rng.uniform(0.1, 1.0) * scale
        phi = rng.uniform(0.0, math.pi)
        dx, dy = X - x0, Y - y0
        c, s = math.cos(phi), math.sin(phi)
        inside = ((dx * c + dy * s) / a) ** 2 + ((-dx * s + dy * c) / b) ** 2 <= 1.0
        img[inside] += val
    return img.reshape(-1)


def _random_rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def ellipsoid_phantom(geom: Geometry, n_ell: int, seed: int, scale: float = 0.1) -> np.ndarray:
    """Sum of random ellipsoids (uniform random rotation) at voxel centres."""
    rng = np.random.default_rng(seed)
    half = 0.5 * geom.nx * geom.vx
    cx = geom.ox + (np.arange(geom.nx) + 0.5) * geom.vx
    cy = geom.oy + (np.arange(geom.ny) + 0.5) * geom.vy
    cz = geom.oz + (np.arange(geom.nz) + 0.5) * geom.vz
    vol = np.zeros((geom.nz, geom.ny, geom.nx), dtype=np.float64)
    Z, Y, X = np.meshgrid(cz, cy, cx, indexing="ij")
    for _ in range(n_ell):
        ctr = rng.uniform(-0.7, 0.7, 3) * half
        ax = rng.uniform(0.05, 0.4, 3) * half
        val = rng.uniform(0.1, 1.0) * scale
        R = _random_rotation(rng)
        d = np.stack([X - ctr[0], Y - ctr[1], Z - ctr[2]], -1)
        loc = d @ R
        inside = ((loc / ax) ** 2).sum(-1) <= 1.0
        vol[inside] += val
    return vol.reshape(-1)


def phantom_for(geom: Geometry, seed: int, n_ell: int | None = None) -> np.ndarray:
    if geom.is3d:
        return ellipsoid_phantom(geom, 20 if n_ell is None else n_ell, seed)
    return ellipse_phantom(geom, 12 if n_ell is None else n_ell, seed)


def gaussian_noise(p: np.ndarray, rel: float, seed: int) -> np.ndarray:
    """y = p + N(0, (rel * max p)^2), rounded to float32."""
    rng = np.random.default_rng(seed + 7919)
    sig = rel * float(np.max(np.abs(p))) if p.size else 0.0
    return (p + rng.normal(0.0, sig, p.shape)).astype(np.float32)


def poisson_noise(p: np.ndarray, photons: float, seed: int) -> np.ndarray:
    """counts ~ Poisson(photons * exp(-p)), clamped >= 1; y = -ln(counts/photons)."""
    rng = np.random.default_rng(seed + 7919)
    cnt = np.maximum(rng.poisson(photons * np.exp(-np.asarray(p, np.float64))), 1)
    return (-np.log(cnt / photons)).astype(np.float32)


def seed_for(config: int, job: int = 0) -> int:
    return 1000 * config + job

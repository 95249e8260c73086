"""Projection-area block densities (oracle side; test infrastructure only).

The paper's own density estimate for importance sampling (Sec. II-C, Alg. 5):
P(I,J) = P_S / P_T, where P_S is the area on the detector sub-areas of row
block I (over the views of I) covered by the projection of the voxel block J,
and P_T is the total projection area of J over the whole scan.  Reading C24:
P_T is the sum of P_S over all row blocks, so that the probabilities of each
column block sum to one also where the detector truncates the projection.

The projection of J's box is taken exactly: the hull of its projected
corners (an interval on a 2D detector, a convex polygon on a flat 3D one,
as the box lies in front of the source), intersected with each tile's
rectangle of bin edges.  Lengths are in detector units (mm, or radians for
the curved detector), areas in mm^2.
"""
from __future__ import annotations

import numpy as np

PAR2D, FAN2D_FLAT, FAN2D_CURVED, CONE3D_FLAT = 0, 1, 2, 3


def _cross(a, b) -> float:
    return float(a[0] * b[1] - a[1] * b[0])


def _corners(geom, box):
    x0, x1, y0, y1, z0, z1 = box
    xs = (geom.ox + x0 * geom.vx, geom.ox + x1 * geom.vx)
    ys = (geom.oy + y0 * geom.vy, geom.oy + y1 * geom.vy)
    if geom.kind != CONE3D_FLAT:
        return [np.array([x, y]) for x in xs for y in ys]
    zs = (geom.oz + z0 * geom.vz, geom.oz + z1 * geom.vz)
    return [np.array([x, y, z]) for x in xs for y in ys for z in zs]


def project_2d(geom, view: int, p) -> float:
    """Detector coordinate u where the ray through point p meets the detector."""
    V = np.asarray(geom.views[view], dtype=np.float64)
    a, c, eu = V[0:2], V[3:5], V[6:8]
    if geom.kind == PAR2D:              # p + t a = c + u e_u
        return _cross(p - c, a) / _cross(eu, a)
    if geom.kind == FAN2D_FLAT:         # a + t (p - a) = c + u e_u
        d = p - a
        return _cross(a - c, d) / _cross(eu, d)
    axis = (c - a) / np.linalg.norm(c - a)  # curved: angle from the central ray
    d = p - a
    return float(np.arctan2(d @ eu, d @ axis))


def project_3d(geom, view: int, p):
    """(u, v) where the ray from the source through p meets the detector plane."""
    V = np.asarray(geom.views[view], dtype=np.float64)
    a, c, eu, ev = V[0:3], V[3:6], V[6:9], V[9:12]
    sdd = np.linalg.norm(c - a)
    n = (c - a) / sdd
    d = p - a
    depth = d @ n
    return np.array([sdd * (d @ eu) / depth, sdd * (d @ ev) / depth])


def _hull(pts):
    """Convex hull, counter-clockwise (Andrew's monotone chain)."""
    pts = sorted(map(tuple, pts))
    if len(pts) <= 2:
        return [np.array(p) for p in pts]

    def half(seq):
        out = []
        for p in seq:
            while len(out) >= 2 and _cross(np.subtract(out[-1], out[-2]), np.subtract(p, out[-2])) <= 0:
                out.pop()
            out.append(p)
        return out

    lower, upper = half(pts), half(reversed(pts))
    return [np.array(p) for p in lower[:-1] + upper[:-1]]


def _clip(poly, axis: int, bound: float, keep_below: bool):
    """Sutherland-Hodgman clip of a polygon by the half-plane x_axis <= bound
    (keep_below) or x_axis >= bound."""
    out = []
    inside = (lambda q: q[axis] <= bound) if keep_below else (lambda q: q[axis] >= bound)
    for k in range(len(poly)):
        p, q = poly[k - 1], poly[k]
        if inside(q):
            if not inside(p):
                t = (bound - p[axis]) / (q[axis] - p[axis])
                out.append(p + t * (q - p))
            out.append(q)
        elif inside(p):
            t = (bound - p[axis]) / (q[axis] - p[axis])
            out.append(p + t * (q - p))
    return out


def _area(poly) -> float:
    if len(poly) < 3:
        return 0.0
    return 0.5 * abs(sum(_cross(poly[k - 1], poly[k]) for k in range(len(poly))))


def bin_edges(n: int, pitch: float, i0: int, i1: int):
    """Detector coordinates of the outer edges of bins [i0, i1)."""
    c0 = 0.5 * (n - 1)
    return (i0 - 0.5 - c0) * pitch, (i1 - 0.5 - c0) * pitch


def tile_overlap(geom, tile, box) -> float:
    """P_S contribution of one tile (view, u0, u1, v0, v1) and a voxel box."""
    view, u0, u1, v0, v1 = (int(t) for t in tile)
    ulo, uhi = bin_edges(geom.nu, geom.pu, u0, u1)
    if geom.kind != CONE3D_FLAT:
        us = [project_2d(geom, view, p) for p in _corners(geom, box)]
        return max(0.0, min(uhi, max(us)) - max(ulo, min(us)))
    vlo, vhi = bin_edges(geom.nv, geom.pv, v0, v1)
    poly = _hull([project_3d(geom, view, p) for p in _corners(geom, box)])
    for axis, bound, below in ((0, ulo, False), (0, uhi, True), (1, vlo, False), (1, vhi, True)):
        poly = _clip(poly, axis, bound, below)
        if not poly:
            return 0.0
    return _area(poly)


def shadow_area_table(geom) -> np.ndarray:
    """P_S for every (row block I, column block J), FP64 [m, n]."""
    out = np.zeros((geom.m, geom.n), dtype=np.float64)
    for I, tiles in enumerate(geom.row_blocks):
        for J, box in enumerate(geom.col_blocks):
            out[I, J] = sum(tile_overlap(geom, t, box) for t in tiles)
    return out


def area_density(geom) -> np.ndarray:
    """P(I,J) = P_S / P_T with P_T = sum_I P_S (reading C24)."""
    S = shadow_area_table(geom)
    tot = S.sum(axis=0)
    P = np.zeros_like(S)
    nz = tot > 0
    P[:, nz] = S[:, nz] / tot[nz]
    return P

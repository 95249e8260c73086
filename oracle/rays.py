"""FP64 rays of a scan geometry (oracle side; test infrastructure only).

One line per detector bin centre (reading C13: no detector-area or
finite-source integration), as the system-matrix definition of Sec. II-A
needs.  Parallel rays are full lines; divergent rays start at the source.
"""
from __future__ import annotations

import numpy as np

PAR2D, FAN2D_FLAT, FAN2D_CURVED, CONE3D_FLAT = 0, 1, 2, 3


def bin_coords(n: int, pitch: float) -> np.ndarray:
    """Centre coordinate of each of ``n`` bins, symmetric about zero."""
    return (np.arange(n, dtype=np.float64) - 0.5 * (n - 1)) * pitch


def rays(geom):
    """Return ``(origin [M,3], direction [M,3], divergent)`` in FP64.

    Ray order: ``i = (view * nv + iv) * nu + iu``.
    """
    V = np.asarray(geom.views, dtype=np.float64)
    nvw = V.shape[0]
    a, c, eu, ev = V[:, 0:3], V[:, 3:6], V[:, 6:9], V[:, 9:12]
    u = bin_coords(geom.nu, geom.pu)
    v = bin_coords(geom.nv, geom.pv) if geom.kind == CONE3D_FLAT else np.zeros(1)
    nv = len(v)
    shape = (nvw, nv, geom.nu, 3)
    if geom.kind == PAR2D:
        pts = c[:, None, None, :] + u[None, None, :, None] * eu[:, None, None, :]
        org = np.broadcast_to(pts, shape)
        dirn = np.broadcast_to(a[:, None, None, :], shape)
        divergent = False
    elif geom.kind == FAN2D_FLAT:
        pts = c[:, None, None, :] + u[None, None, :, None] * eu[:, None, None, :]
        org = np.broadcast_to(a[:, None, None, :], shape)
        dirn = np.broadcast_to(pts, shape) - org
        divergent = True
    elif geom.kind == FAN2D_CURVED:
        axis = c - a
        axis = axis / np.linalg.norm(axis, axis=1, keepdims=True)
        cg, sg = np.cos(u), np.sin(u)
        d = cg[None, :, None] * axis[:, None, :] + sg[None, :, None] * eu[:, None, :]
        org = np.broadcast_to(a[:, None, None, :], shape)
        dirn = np.broadcast_to(d[:, None, :, :], shape)
        divergent = True
    elif geom.kind == CONE3D_FLAT:
        pts = (c[:, None, None, :] + u[None, None, :, None] * eu[:, None, None, :]
               + v[None, :, None, None] * ev[:, None, None, :])
        org = np.broadcast_to(a[:, None, None, :], shape)
        dirn = pts - org
        divergent = True
    else:
        raise ValueError(f"unknown geometry kind {geom.kind}")
    return (np.ascontiguousarray(org.reshape(-1, 3)),
            np.ascontiguousarray(dirn.reshape(-1, 3)), divergent)


def rays_at(geom, idx):
    """Rays of the given ray indices only (same definitions as ``rays``), for
    geometries too large to hold every ray."""
    idx = np.asarray(idx, dtype=np.int64)
    V = np.asarray(geom.views, dtype=np.float64)
    nv = geom.nv if geom.kind == CONE3D_FLAT else 1
    view = idx // (nv * geom.nu)
    iv = (idx // geom.nu) % nv
    iu = idx % geom.nu
    a, c, eu, ev = V[view, 0:3], V[view, 3:6], V[view, 6:9], V[view, 9:12]
    u = ((iu - 0.5 * (geom.nu - 1)) * geom.pu)[:, None]
    if geom.kind == PAR2D:
        return c + u * eu, a.copy(), False
    if geom.kind == FAN2D_FLAT:
        return a.copy(), c + u * eu - a, True
    if geom.kind == FAN2D_CURVED:
        axis = c - a
        axis = axis / np.linalg.norm(axis, axis=1, keepdims=True)
        return a.copy(), np.cos(u) * axis + np.sin(u) * eu, True
    if geom.kind == CONE3D_FLAT:
        v = ((iv - 0.5 * (geom.nv - 1)) * geom.pv)[:, None]
        return a.copy(), c + u * eu + v * ev - a, True
    raise ValueError(f"unknown geometry kind {geom.kind}")

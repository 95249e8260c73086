"""Explicit FP64 system matrix (oracle side; test infrastructure only).

``system_matrix`` builds A (Sec. II-A: A_ij = intersection length of ray i
with voxel j) with the C Siddon traversal in ``siddon.c``; ``clip_length``
is the closed-form length of one line inside one box (slab method) that pins
it.  Both follow reading C12: voxels are half-open, a zero direction
component gives no crossings on that axis.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np
import scipy.sparse as sp

from . import rays as _rays

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "siddon.c")
_LIB = os.path.join(_HERE, "libsiddon_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C row generator with gcc (FP64, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c99",
                               "-fno-fast-math", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        for name in ("siddon_count", "siddon_fill"):
            f = getattr(lib, name)
            f.restype = ctypes.c_int
        lib.siddon_count.argtypes = [ctypes.c_int, P, P, P, ctypes.c_int64, P, P, ctypes.c_int, P]
        lib.siddon_fill.argtypes = [ctypes.c_int, P, P, P, ctypes.c_int64, P, P, ctypes.c_int,
                                    P, P, P]
        lib.siddon_set_threads.argtypes = [ctypes.c_int]
        lib.siddon_set_threads.restype = None
        lib.siddon_max_threads.argtypes = []
        lib.siddon_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def set_threads(n: int) -> int:
    """Threads of the row generator's OpenMP loops (timing only); returns the
    count now in effect."""
    lib = _load()
    lib.siddon_set_threads(int(n))
    return int(lib.siddon_max_threads())


def _vol(geom):
    dims = 3 if geom.kind == _rays.CONE3D_FLAT else 2
    n = np.array([geom.nx, geom.ny, geom.nz], dtype=np.int64)
    lo = np.array([geom.ox, geom.oy, geom.oz], dtype=np.float64)
    h = np.array([geom.vx, geom.vy, geom.vz], dtype=np.float64)
    return dims, n, lo, h


def rows_for(geom, org, dirn, divergent) -> sp.csr_matrix:
    """CSR rows (FP64) for arbitrary lines through the volume of ``geom``."""
    lib = _load()
    dims, n, lo, h = _vol(geom)
    org = np.ascontiguousarray(org, dtype=np.float64)
    dirn = np.ascontiguousarray(dirn, dtype=np.float64)
    M = org.shape[0]
    counts = np.zeros(M, dtype=np.int64)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    if lib.siddon_count(dims, p(n), p(lo), p(h), M, p(org), p(dirn), int(divergent), p(counts)):
        raise MemoryError("siddon_count failed")
    indptr = np.zeros(M + 1, dtype=np.int64)
    np.cumsum(counts, out=indptr[1:])
    nnz = int(indptr[-1])
    indices = np.zeros(nnz, dtype=np.int64)
    data = np.zeros(nnz, dtype=np.float64)
    if lib.siddon_fill(dims, p(n), p(lo), p(h), M, p(org), p(dirn), int(divergent),
                       p(indptr), p(indices), p(data)):
        raise RuntimeError("siddon_fill failed")
    N = geom.nx * geom.ny * geom.nz
    return sp.csr_matrix((data, indices, indptr), shape=(M, N))


def system_matrix(geom) -> sp.csr_matrix:
    """The whole of A for ``geom`` (rows in ray order, FP64)."""
    org, dirn, div = _rays.rays(geom)
    return rows_for(geom, org, dirn, div)


def clip_length(org, dirn, divergent, lo, hi):
    """Closed-form |line ∩ box| for many (line, box) pairs, vectorised.

    ``org``, ``dirn``: [K, D]; ``lo``, ``hi``: [K, D] half-open boxes.  A
    divergent line starts at its origin.  This is the plain definition of
    A_ij, written out independently of the Siddon traversal.
    """
    org = np.asarray(org, dtype=np.float64)
    dirn = np.asarray(dirn, dtype=np.float64)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    K, D = org.shape
    t0 = np.full(K, 0.0 if divergent else -np.inf)
    t1 = np.full(K, np.inf)
    ok = np.ones(K, dtype=bool)
    for k in range(D):
        d = dirn[:, k]
        z = d == 0.0
        inside = (org[:, k] >= lo[:, k]) & (org[:, k] < hi[:, k])
        ok &= ~z | inside
        with np.errstate(divide="ignore", invalid="ignore"):
            ta = np.where(z, -np.inf, (lo[:, k] - org[:, k]) / np.where(z, 1.0, d))
            tb = np.where(z, np.inf, (hi[:, k] - org[:, k]) / np.where(z, 1.0, d))
        t0 = np.maximum(t0, np.minimum(ta, tb))
        t1 = np.minimum(t1, np.maximum(ta, tb))
    L = np.where(ok, np.maximum(t1 - t0, 0.0), 0.0) * np.linalg.norm(dirn, axis=1)
    return L

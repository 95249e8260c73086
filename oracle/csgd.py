"""CSGD / GCSGD (Alg. 4, 5, 6) step by step in FP64 (oracle side; test
infrastructure only).

Every update follows the basic iteration (Alg. 3) on the sub-matrix
``A_{I_G}^J`` of a group G of row blocks:

    g   = (A_{I_G}^J)^T r_{I_G}                         Eq. (7)
    mu  = beta * g^T g / (g^T (A^J)^T A^J g)            Eq. (11), relaxed
    xhat_J += x_J + mu g                                 Alg. 4 / 6
    z^J_{I_G} = A_{I_G}^J (x_J + mu g)                   Alg. 4 / 6

and after each column block (reading C1, default) the residual is refreshed
on the touched rows only, r_It = y_It - sum_j z^j_It (Sec. II-C).  At the end
of an epoch every updated block is set to the mean of its outputs.
Readings: C7 (mu = 0 when g = 0), C9 (x_J is the epoch-start value inside an
epoch), C10 (divisor = number of groups of J in the epoch), C11 (sums over j
ascend).  ``sync='epoch'`` is the simultaneous reading of Sec. II-B: every
column block sees the epoch-start residual, refreshed once at the epoch end.
"""
from __future__ import annotations

from typing import Dict, Tuple

import numpy as np
import scipy.sparse as sp


class BlockSystem:
    """Explicit sub-blocks A_I^J of one system matrix, cut by the partition."""

    def __init__(self, A: sp.csr_matrix, geom):
        self.A = A.tocsr()
        self.geom = geom
        self.M, self.N = A.shape
        self.rows = [geom.row_block_rays(I) for I in range(geom.m)]
        self.vox = [geom.col_block_vox(J) for J in range(geom.n)]
        self._cache: Dict[Tuple[int, int], sp.csr_matrix] = {}
        self._row_cache: Dict[int, sp.csr_matrix] = {}

    def block(self, I: int, J: int) -> sp.csr_matrix:
        key = (I, J)
        if key not in self._cache:
            if I not in self._row_cache:
                self._row_cache[I] = self.A[self.rows[I]].tocsc()
            self._cache[key] = self._row_cache[I][:, self.vox[J]].tocsr()
        return self._cache[key]

    def group(self, G, J: int) -> sp.csr_matrix:
        return sp.vstack([self.block(I, J) for I in G], format="csr")

    def group_rows(self, G) -> np.ndarray:
        return np.concatenate([self.rows[I] for I in G])

    def nnz_table(self, tau: float) -> np.ndarray:
        """nnz(A_I^J): the number of ray-voxel pairs of length > tau (C6)."""
        out = np.zeros((self.geom.m, self.geom.n), dtype=np.int64)
        for I in range(self.geom.m):
            for J in range(self.geom.n):
                out[I, J] = int(np.count_nonzero(self.block(I, J).data > tau))
        return out


def block_fwd(S: BlockSystem, G, J: int, x: np.ndarray) -> np.ndarray:
    """A_{I_G}^J x_J (Alg. 3, last line) on the rows of G, in row order."""
    return S.group(G, J) @ np.asarray(x, dtype=np.float64)[S.vox[J]]


def block_back(S: BlockSystem, G, J: int, r: np.ndarray) -> np.ndarray:
    """(A_{I_G}^J)^T r_{I_G} (Eq. 7) on the voxels of J."""
    rows = S.group_rows(G)
    return S.group(G, J).T @ np.asarray(r, dtype=np.float64)[rows]


class State:
    def __init__(self, S: BlockSystem, y: np.ndarray, x0=None):
        """Initialisation of Alg. 4: x = 0, z^j = 0, r = y.  A non-zero x0 is
        taken as z^j = A^j x0_J and r = y - sum_j z^j, the same invariant."""
        self.S = S
        self.y = np.asarray(y, dtype=np.float64).copy()
        self.x = np.zeros(S.N) if x0 is None else np.asarray(x0, dtype=np.float64).copy()
        self.z = np.zeros((S.geom.n, S.M))
        if x0 is not None:
            for J in range(S.geom.n):
                self.z[J] = S.A[:, S.vox[J]] @ self.x[S.vox[J]]
        self.r = self.y - self.z.sum(axis=0)
        self.updates = 0            # ray-voxel updates (fwd + back), 2 nnz per group


def step_group(st: State, G, J: int, beta: float):
    """One basic computation block on (I_G, J); returns (x_J + mu g, mu)."""
    S = st.S
    AG = S.group(G, J)
    rows = S.group_rows(G)
    vox = S.vox[J]
    g = AG.T @ st.r[rows]
    q = AG @ g
    gg = float(g @ g)
    qq = float(q @ q)
    mu = beta * gg / qq if (gg > 0.0 and qq > 0.0) else 0.0
    xnew = st.x[vox] + mu * g
    st.z[J, rows] = AG @ xnew
    st.updates += 2 * AG.nnz
    return xnew, mu, rows


def step_group_matrix_free(geom, rows: np.ndarray, J: int, x: np.ndarray, r: np.ndarray,
                           beta: float, chunk: int = 1 << 17):
    """The basic computation block of ``step_group`` without a stored A
    (matrix-free mode, for geometries whose A does not fit in memory).

    The rows of A for the rays ``rows`` (global ray indices of the group's
    row blocks, in order) are generated chunk by chunk by the same Siddon
    row generator, cut to the columns of block J and dropped after use; A
    is generated twice, once for g = (A_{I_G}^J)^T r_{I_G} (Eq. 7) and once
    for q = A g and a = A x_J, as the step size (Eq. 11) needs all of g
    first.  z^J_{I_G} = A x_J + mu A g, which is A (x_J + mu g) of
    ``step_group`` up to rounding.  Returns (x_J + mu g, mu, z rows, nnz of
    the block).  Pinned against ``step_group`` on small geometries."""
    from . import rays as _rays
    from . import siddon as _siddon
    rows = np.asarray(rows, dtype=np.int64)
    vox = geom.col_block_vox(J)
    loc = np.full(geom.n_vox, -1, dtype=np.int64)
    loc[vox] = np.arange(len(vox))

    def blocks():
        for a in range(0, len(rows), chunk):
            idx = rows[a:a + chunk]
            org, dirn, div = _rays.rays_at(geom, idx)
            A = _siddon.rows_for(geom, org, dirn, div)
            c = loc[A.indices]
            keep = c >= 0
            rid = np.repeat(np.arange(len(idx)), np.diff(A.indptr))
            AJ = sp.csr_matrix((A.data[keep], (rid[keep], c[keep])), shape=(len(idx), len(vox)))
            yield a, idx, AJ

    g = np.zeros(len(vox))
    nnz = 0
    for _, idx, AJ in blocks():
        g += AJ.T @ np.asarray(r, dtype=np.float64)[idx]
        nnz += AJ.nnz
    xJ = np.asarray(x, dtype=np.float64)[vox]
    q = np.zeros(len(rows))
    ax = np.zeros(len(rows))
    for a, idx, AJ in blocks():
        q[a:a + len(idx)] = AJ @ g
        ax[a:a + len(idx)] = AJ @ xJ
    gg = float(g @ g)
    qq = float(q @ q)
    mu = beta * gg / qq if (gg > 0.0 and qq > 0.0) else 0.0
    return xJ + mu * g, mu, ax + mu * q, nnz


def refresh(st: State, rows: np.ndarray):
    """r_It = y_It - sum_j z^j_It (sum over j ascending)."""
    acc = np.zeros(len(rows))
    for j in range(st.z.shape[0]):
        acc += st.z[j, rows]
    st.r[rows] = st.y[rows] - acc


def epoch(st: State, sched, e: int, sync: str = "column"):
    """One epoch of Alg. 6 (Alg. 4 / 5 are the s = 1 special cases)."""
    S = st.S
    xhat = np.zeros(S.N)
    cnt = np.zeros(S.geom.n, dtype=np.int64)
    touched_all = []
    for J, groups in sched.steps(e):
        touched = []
        for G, beta in groups:
            xnew, _, rows = step_group(st, G, J, beta)
            xhat[S.vox[J]] += xnew
            cnt[J] += 1
            touched.append(rows)
        if touched:
            rows = np.unique(np.concatenate(touched))
            if sync == "column":
                refresh(st, rows)
            else:
                touched_all.append(rows)
    if sync != "column" and touched_all:
        refresh(st, np.unique(np.concatenate(touched_all)))
    for J in range(S.geom.n):
        if cnt[J] > 0:
            st.x[S.vox[J]] = xhat[S.vox[J]] / cnt[J]


def run(S: BlockSystem, y, sched, epochs=None, sync="column", x0=None) -> State:
    st = State(S, y, x0)
    E = sched.n_epochs if epochs is None else epochs
    for e in range(E):
        epoch(st, sched, e, sync)
    return st


def true_rel_residual(S: BlockSystem, y, x) -> float:
    """||y - A x|| / ||y|| with the full A (reading C16)."""
    y = np.asarray(y, dtype=np.float64)
    return float(np.linalg.norm(y - S.A @ x) / np.linalg.norm(y))


def snr_db(x_true, x_est) -> float:
    """Sec. III: 20 log10 ||x_true|| / ||x_true - x_est||."""
    return float(20 * np.log10(np.linalg.norm(x_true) / np.linalg.norm(x_true - x_est)))


def observation_gap_db(S: BlockSystem, y, x_est) -> float:
    """Sec. III: 20 log10 ||y|| / ||y - A x_est||."""
    y = np.asarray(y, dtype=np.float64)
    return float(20 * np.log10(np.linalg.norm(y) / np.linalg.norm(y - S.A @ x_est)))

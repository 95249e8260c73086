"""Block schedule of Alg. 5 / Alg. 6 (oracle side; test infrastructure only).

The schedule depends only on the density table, the parameters and the seed
(never on x or r), so it is drawn up front.  Readings of the paper used here:

* C2  ``select J randomly``: a uniform permutation of the column blocks,
      of which the first ceil(gamma*n) are used (gamma = 1 -> all).
* C3  ``without replacement with probability P(I,J)``: successive weighted
      draws renormalised over the row blocks not yet drawn; blocks of zero
      weight are never drawn, and the draw count is clamped to their number.
* C4  the group loop draws ceil(alpha*m) row blocks in total, cut into
      consecutive groups of s (the last one may be shorter).
* C5  a group's relaxation is beta_G = b * sum_{I in G} P(I,J).
* C6  P(I,J) = nnz(A_I^J) / sum_I' nnz(A_I'^J).
* Mixed sampling (Sec. III-D): row block I of projection p gets the weight
  P_I + theta (P_max(p) - P_I), where P_max(p) is the largest P among the
  row blocks of the same projection (the sub-detector areas of one view, or
  of one set of views) and theta = min(1, epoch * theta_step).  A row block
  with P_I = 0 in a projection with P_max(p) > 0 has weight theta P_max(p),
  so at theta = 1 every sub-area of a projection is equally likely (the
  caption of the sampling-comparison figure); a projection that J does not
  reach at all keeps weight 0.  beta still uses P (C5).

Random numbers come from SplitMix64 (Steele, Lea and Flood, 2014) used as a
counter-based generator: the k-th output for key ``seed`` is
``mix(seed + (k+1) * 0x9E3779B97F4A7C15)``; a uniform double is the top 53
bits times 2^-53.  Within epoch e (0-based) the counter is ``e * 2^32 + k``
where k counts the draws of that epoch in the order they are made.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List

import numpy as np

MASK = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15

DENSITY, UNIFORM, MIXED = 0, 1, 2


def splitmix64(seed: int, ctr: int) -> int:
    z = (seed + (ctr + 1) * GOLDEN) & MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def uniform(seed: int, ctr: int) -> float:
    return (splitmix64(seed, ctr) >> 11) * (1.0 / 9007199254740992.0)


def count_of(frac: float, total: int) -> int:
    """ceil(frac * total) guarded against FP noise, clamped to [1, total]."""
    k = int(math.ceil(frac * total - 1e-9))
    return max(1, min(total, k))


def density_w(w: np.ndarray) -> np.ndarray:
    """P(I,J) = w[I,J] / sum_I w[I,J] for float weights (e.g. projection
    areas), the column sum taken in ascending I (zero column -> zero P)."""
    w = np.asarray(w, dtype=np.float64)
    P = np.zeros(w.shape, dtype=np.float64)
    for J in range(w.shape[1]):
        col = 0.0
        for I in range(w.shape[0]):
            col += float(w[I, J])
        if col > 0:
            P[:, J] = w[:, J] / col
    return P


def density(nnz: np.ndarray) -> np.ndarray:
    """P(I,J) = nnz[I,J] / sum_I nnz[I,J] (zero column -> zero P)."""
    nnz = np.asarray(nnz, dtype=np.int64)
    col = nnz.sum(axis=0)
    P = np.zeros(nnz.shape, dtype=np.float64)
    for J in range(nnz.shape[1]):
        if col[J] > 0:
            P[:, J] = nnz[:, J].astype(np.float64) / float(col[J])
    return P


@dataclasses.dataclass
class Schedule:
    """Flat schedule arrays (epoch -> columns -> groups -> row blocks)."""
    epoch_col_ptr: np.ndarray
    cols: np.ndarray
    col_group_ptr: np.ndarray
    group_rb_ptr: np.ndarray
    rbs: np.ndarray
    beta: np.ndarray

    @property
    def n_epochs(self) -> int:
        return len(self.epoch_col_ptr) - 1

    def steps(self, e: int):
        """Yield ``(J, [(row_blocks, beta), ...])`` for epoch ``e``."""
        for c in range(self.epoch_col_ptr[e], self.epoch_col_ptr[e + 1]):
            groups = []
            for g in range(self.col_group_ptr[c], self.col_group_ptr[c + 1]):
                rb = self.rbs[self.group_rb_ptr[g]:self.group_rb_ptr[g + 1]]
                groups.append((list(int(t) for t in rb), float(self.beta[g])))
            yield int(self.cols[c]), groups


def projection_of(row_blocks) -> np.ndarray:
    """Projection of every row block, for mixed sampling (Sec. III-D).

    Row blocks whose tiles cover the same set of views are sub-detector
    areas of one projection.  Returns, per row block, the index of the first
    row block with the same set of views.
    """
    first = {}
    out = np.zeros(len(row_blocks), dtype=np.int32)
    for I, tiles in enumerate(row_blocks):
        key = tuple(sorted(set(int(t[0]) for t in np.asarray(tiles).reshape(-1, 5))))
        out[I] = first.setdefault(key, I)
    return out


def draw_weights(P: np.ndarray, J: int, theta: float, sampling: int, proj=None) -> List[float]:
    """Weight of every row block in the draws for column block J: P(I,J)
    (importance sampling, Sec. II-C), 1 (uniform), or the mixed weight
    P_I + theta (P_max(p) - P_I) of Sec. III-D, P_max(p) the largest P(., J)
    in I's projection p (0 for a projection J does not reach)."""
    m = P.shape[0]
    if sampling == UNIFORM:
        return [1.0] * m
    if sampling == MIXED:
        pmax = {}
        for I in range(m):
            pmax[proj[I]] = max(pmax.get(proj[I], 0.0), float(P[I, J]))
        return [(float(P[I, J]) + theta * (pmax[proj[I]] - float(P[I, J]))) if pmax[proj[I]] > 0
                else 0.0 for I in range(m)]
    return [float(P[I, J]) for I in range(m)]


def make_schedule(P: np.ndarray, epochs: int, alpha: float, gamma: float, s: int, b: float,
                  seed: int, sampling: int = DENSITY, theta_step: float = 0.0,
                  proj=None) -> Schedule:
    """Draw the whole schedule (Alg. 5 with s = 1, Alg. 6 in general).

    ``proj`` (mixed sampling only): the projection of every row block, as
    ``projection_of`` gives it.
    """
    P = np.asarray(P, dtype=np.float64)
    m, n = P.shape
    if sampling == MIXED:
        if proj is None:
            raise ValueError("mixed sampling needs the projection of every row block")
        proj = [int(p) for p in np.asarray(proj).reshape(-1)]
        if len(proj) != m:
            raise ValueError("proj has the wrong length")
    ecp, cols, cgp, grp, rbs, beta = [0], [], [0], [0], [], []
    for e in range(epochs):
        k = 0
        base = e << 32

        def u():
            nonlocal k
            val = uniform(seed, base + k)
            k += 1
            return val

        perm = list(range(n))
        for i in range(n - 1, 0, -1):
            j = int(math.floor(u() * (i + 1)))
            perm[i], perm[j] = perm[j], perm[i]
        theta = min(1.0, e * theta_step)
        for J in perm[:count_of(gamma, n)]:
            w = draw_weights(P, J, theta, sampling, proj)
            avail = [I for I in range(m) if w[I] > 0]
            K = min(count_of(alpha, m), len(avail))
            draws: List[int] = []
            for _ in range(K):
                W = 0.0
                for I in avail:
                    W += w[I]
                target = u() * W
                acc = 0.0
                pick = avail[-1]
                for I in avail:
                    acc += w[I]
                    if acc > target:
                        pick = I
                        break
                draws.append(pick)
                avail.remove(pick)
            for g0 in range(0, K, s):
                G = draws[g0:g0 + s]
                bsum = 0.0
                for I in G:
                    bsum += P[I, J]
                rbs.extend(G)
                grp.append(len(rbs))
                beta.append(b * bsum)
            cols.append(J)
            cgp.append(len(grp) - 1)
        ecp.append(len(cols))
    i32 = lambda a: np.asarray(a, dtype=np.int32)
    return Schedule(i32(ecp), i32(cols), i32(cgp), i32(grp), i32(rbs),
                    np.asarray(beta, dtype=np.float64))


def full_sweep_schedule(m: int, n: int, epochs: int, beta: float) -> Schedule:
    """Alg. 4 literally: every column block in order, every row block in
    order, one row block per update, constant beta."""
    ecp, cols, cgp, grp, rbs, bet = [0], [], [0], [0], [], []
    for _ in range(epochs):
        for J in range(n):
            for I in range(m):
                rbs.append(I)
                grp.append(len(rbs))
                bet.append(beta)
            cols.append(J)
            cgp.append(len(grp) - 1)
        ecp.append(len(cols))
    i32 = lambda a: np.asarray(a, dtype=np.int32)
    return Schedule(i32(ecp), i32(cols), i32(cgp), i32(grp), i32(rbs), np.asarray(bet))

"""Minimum-image geometry and neighbour sets (oracle).

The neighbour set of atom i is every j != i whose minimum-image squared distance is
below ``r_list**2``, listed in ascending j.  This is the plain definition of the Verlet
list the paper's force routine relies on (Sec. II D; Appendix C mentions the list).

Minimum image, per periodic dimension of length L, with d = x_j - x_i and both
coordinates already in [lo, hi):  d -= L if d >= L/2;  d += L if d < -L/2.
Squared distance:  r2 = (dx*dx + dy*dy) + dz*dz, each product rounded separately.
"""

from __future__ import annotations

import numpy as np


def min_image(d: np.ndarray, L: float, periodic: bool) -> np.ndarray:
    if not periodic:
        return d
    half = 0.5 * L
    return np.where(d >= half, d - L, np.where(d < -half, d + L, d))


def displacements(pos: np.ndarray, box, periodic, i: np.ndarray, j: np.ndarray):
    """Minimum-image vectors r_ij = x_j - x_i for index arrays ``i``, ``j``."""
    dx = min_image(pos[0, j] - pos[0, i], box[0], periodic[0])
    dy = min_image(pos[1, j] - pos[1, i], box[1], periodic[1])
    dz = min_image(pos[2, j] - pos[2, i], box[2], periodic[2])
    return dx, dy, dz


def sq_dist(dx, dy, dz):
    """(dx*dx + dy*dy) + dz*dz in that order (numpy never fuses these)."""
    return (dx * dx + dy * dy) + dz * dz


def _candidate_pairs(pos, lo, hi, periodic, r_list):
    """Unordered candidate pairs (i < j) within ``r_list`` up to a small margin.

    Small systems: brute force over all pairs.  Large systems: scipy's cKDTree (a
    library search used only to propose candidates; the exact test is applied later).
    """
    n = pos.shape[1]
    if n <= 4000:
        i, j = np.triu_indices(n, k=1)
        return i, j
    from scipy.spatial import cKDTree
    box = np.asarray(hi, dtype=np.float64) - np.asarray(lo, dtype=np.float64)
    q = (pos - np.asarray(lo, dtype=np.float64)[:, None]).T.copy()
    size = np.empty(3)
    for k in range(3):
        if periodic[k]:
            q[:, k] = np.mod(q[:, k], box[k])
            q[:, k] = np.where(q[:, k] >= box[k], 0.0, q[:, k])
            size[k] = box[k]
        else:
            shift = q[:, k].min()
            q[:, k] -= shift
            size[k] = q[:, k].max() + 4.0 * r_list + 1.0
    tree = cKDTree(q, boxsize=size)
    pairs = tree.query_pairs(r_list * (1.0 + 1e-9) + 1e-9, output_type="ndarray")
    return pairs[:, 0].astype(np.int64), pairs[:, 1].astype(np.int64)


def neighbor_csr(pos, lo, hi, periodic, r_list):
    """Full neighbour lists within ``r_list`` as CSR ``(offsets[n+1], idx)``.

    Row i holds every j != i with r2(i, j) < r_list**2, in ascending j.
    """
    n = pos.shape[1]
    box = np.asarray(hi, dtype=np.float64) - np.asarray(lo, dtype=np.float64)
    i, j = _candidate_pairs(pos, lo, hi, periodic, r_list)
    dx, dy, dz = displacements(pos, box, periodic, i, j)
    keep = sq_dist(dx, dy, dz) < r_list * r_list
    i, j = i[keep], j[keep]
    # the test is symmetric: r2(j, i) uses -d, whose squares are identical
    ii = np.concatenate([i, j])
    jj = np.concatenate([j, i])
    order = np.lexsort((jj, ii))
    ii, jj = ii[order], jj[order]
    counts = np.bincount(ii, minlength=n)
    offsets = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    return offsets, jj.astype(np.int64)


def pairs_within(pos, lo, hi, periodic, r_cut, csr=None, r_list=None):
    """Directed pairs (i, j), i != j, with r2 < r_cut**2, sorted by (i, j).

    If a CSR list built with a larger radius is given it is filtered; otherwise one is
    built with radius ``r_cut``.
    """
    box = np.asarray(hi, dtype=np.float64) - np.asarray(lo, dtype=np.float64)
    if csr is None:
        csr = neighbor_csr(pos, lo, hi, periodic, r_cut if r_list is None else r_list)
    offsets, idx = csr
    n = pos.shape[1]
    i = np.repeat(np.arange(n, dtype=np.int64), np.diff(offsets))
    j = idx
    dx, dy, dz = displacements(pos, box, periodic, i, j)
    keep = sq_dist(dx, dy, dz) < r_cut * r_cut
    return i[keep], j[keep]

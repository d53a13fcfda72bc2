"""Clusters cut around sampled atoms, for checking large systems one atom at a time.

The sampled atom sits at the origin and every other atom at its minimum-image
displacement from it, computed with the oracle's own formula, so that every quantity of
the sampled atom that depends only on its displacements is reproduced to the last bit.
"""

import numpy as np

import synth
from oracle import geometry


class Cutter:
    """Finds the atoms within a radius of a sampled atom (candidate search with a k-d tree,
    exact test with the oracle's minimum-image displacements) and builds the cluster with
    the sampled atom at the origin."""

    def __init__(self, s):
        from scipy.spatial import cKDTree
        self.s = s
        self.box = s.hi - s.lo
        q = (s.pos - s.lo[:, None]).T.copy()
        size = np.empty(3)
        for d in range(3):
            if s.periodic[d]:
                size[d] = self.box[d]
            else:
                q[:, d] -= q[:, d].min()
                size[d] = q[:, d].max() + 100.0
        self.tree = cKDTree(q, boxsize=size)
        self.q = q

    def cluster(self, i, radius):
        s = self.s
        cand = np.asarray(self.tree.query_ball_point(self.q[i], radius + 1e-6), dtype=np.int64)
        ii = np.full(cand.shape, i)
        dx, dy, dz = geometry.displacements(s.pos, self.box, s.periodic, ii, cand)
        keep = geometry.sq_dist(dx, dy, dz) < radius * radius
        cand, dx, dy, dz = cand[keep], dx[keep], dy[keep], dz[keep]
        order = np.argsort(cand)
        cand, rel = cand[order], np.stack([dx[order], dy[order], dz[order]])
        c = int(np.nonzero(cand == i)[0][0])
        frozen = None if s.frozen is None else s.frozen[cand].copy()
        cl = synth.System(rel, np.full(3, -4 * radius), np.full(3, 4 * radius), (0, 0, 0), frozen=frozen)
        return cl, cand, c

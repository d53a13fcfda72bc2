"""The cluster method of the full-size parity tests, checked against the whole-system
oracle on a small periodic system: rows, centro-symmetry parameter and spread weight bit
for bit, forces and energies to rounding."""

import numpy as np

import synth
from synth import configs
from oracle import ace as oace
from oracle import geometry, hybrid, precision

from cluster_util import Cutter


def test_cluster_matches_whole_system():
    s = configs.bulk(6, seed=3, temperature=300.0, void_radius=4.0)
    prec = synth.PrecisionParams(2.5, 3.0, 1, 3.0, 5.0)
    prm = synth.ace_random(8, 3, oace.num_basis(8, 3), seed=5)
    csr = geometry.neighbor_csr(s.pos, s.lo, s.hi, s.periodic, 5.5)
    pr = precision.compute_precision(s, prec, csr)
    w = pr["w"]
    assert 0 < pr["active"].size < s.n
    ev = hybrid.evaluate(s, synth.eam_cu_like(), prm, w, csr)
    cut = Cutter(s)
    rng = np.random.default_rng(0)
    smp = np.concatenate([rng.choice(np.nonzero(w > 0)[0], 3, replace=False),
                          rng.choice(np.nonzero(w == 0)[0], 2, replace=False)])
    for i in smp:
        cl, idx, c = cut.cluster(i, 10.5)
        ccsr = geometry.neighbor_csr(cl.pos, cl.lo, cl.hi, cl.periodic, 5.5)
        row = np.sort(idx[ccsr[1][ccsr[0][c]:ccsr[0][c + 1]]])
        assert np.array_equal(row, csr[1][csr[0][i]:csr[0][i + 1]])
        c_ref = precision.csp(cl.pos, cl.lo, cl.hi, cl.periodic, ccsr)[c]
        assert c_ref == pr["csp"][i]
        big, bidx, bc = cut.cluster(i, prec.r_hi + 0.5)
        w_ref = precision.spread(big.pos, big.lo, big.hi, big.periodic, pr["w0"][bidx], prec.r_lo, prec.r_hi)[bc]
        assert w_ref == w[i]
        r2 = geometry.sq_dist(cl.pos[0], cl.pos[1], cl.pos[2])
        wc = np.where(r2 < 25.0, w[idx], 0.0)
        evc = hybrid.evaluate(cl, synth.eam_cu_like(), prm, wc)
        assert abs(evc["e_eam"][c] - ev["e_eam"][i]) < 1e-12
        assert np.max(np.abs(evc["f_eam"][:, c] - ev["f_eam"][:, i])) < 1e-12
        assert np.max(np.abs(evc["f_ace"][:, c] - ev["f_ace"][:, i])) < 1e-12
        if w[i] > 0:
            assert abs(evc["e_ace"][c] - ev["e_ace"][i]) < 1e-12

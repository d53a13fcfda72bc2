"""Hybrid energy and forces (oracle).

* Per-atom energy, eq. energy_hyb (Sec. II A), precise-weight form:
      E_i = (1 - w_i) E_i^EAM + w_i E_i^ACE
  (the ACE term is absent when w_i = 0: the precise potential is not evaluated there).
* Forces with the gradient of the switching parameter neglected, eq. F_i_d (Appendix C):
      F_i = -sum_k [ (1 - w_k) d E_k^EAM / d x_i + w_k d E_k^ACE / d x_i ]
  i.e. the negative gradient of sum_k u_k E_k^EAM + w_k E_k^ACE at fixed weights.
  ``f_eam`` and ``f_ace`` are the two weighted parts; ``f`` is their sum.
* E_pot = sum_i E_i, summed exactly rounded (math.fsum).
"""

from __future__ import annotations

import math

import numpy as np
import torch

from . import ace as _ace
from . import eam as _eam
from .geometry import neighbor_csr, pairs_within


def evaluate(system, eam_p, ace_p, w, csr=None, want_forces=True):
    pos, lo, hi, per = system.pos, system.lo, system.hi, system.periodic
    n = pos.shape[1]
    box = np.asarray(hi) - np.asarray(lo)
    w = np.asarray(w, dtype=np.float64)
    u = 1.0 - w
    rc = max(eam_p.rc, ace_p.rc if ace_p is not None else 0.0)
    if csr is None:
        csr = neighbor_csr(pos, lo, hi, per, rc)
    ie, je = pairs_within(pos, lo, hi, per, eam_p.rc, csr)
    pos_t = torch.tensor(pos, dtype=torch.float64, requires_grad=want_forces)
    e_eam_t = _eam.site_energies(pos_t, box, per, ie, je, eam_p, n)
    active = np.nonzero(w > 0.0)[0]
    out = {}
    if want_forces:
        (g,) = torch.autograd.grad((torch.as_tensor(u) * e_eam_t).sum(), pos_t)
        out["f_eam"] = -g.numpy()
    if ace_p is not None and active.size:
        ia, ja = pairs_within(pos, lo, hi, per, ace_p.rc, csr)
        e_ace_t = _ace.site_energies(pos_t, box, per, ia, ja, ace_p, n, active)
        if want_forces:
            (g,) = torch.autograd.grad((torch.as_tensor(w) * e_ace_t).sum(), pos_t)
            out["f_ace"] = -g.numpy()
        e_ace = e_ace_t.detach().numpy()
    else:
        e_ace = np.zeros(n)
        if want_forces:
            out["f_ace"] = np.zeros((3, n))
    e_eam = e_eam_t.detach().numpy()
    e_site = u * e_eam + np.where(w > 0.0, w * e_ace, 0.0)
    out.update(e_eam=e_eam, e_ace=e_ace, e_site=e_site, e_pot=math.fsum(e_site.tolist()),
               rho=_eam.density(pos, box, per, ie, je, eam_p, n), active=active)
    if want_forces:
        out["f"] = out["f_eam"] + out["f_ace"]
    return out

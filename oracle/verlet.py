"""Velocity-Verlet integration with the switching-parameter update (oracle), eq. vv.

One step of length dt (Sec. II C 1):
  1. v(t + dt/2) = v(t) + a(t) dt / 2;   x(t + dt) = x(t) + v(t + dt/2) dt
  2. w(t + dt) recomputed from x(t + dt) (every ``precision_every`` steps; never if 0)
  3. a(t + dt) = F(t + dt) / m with the new weights (plus the external indenter force)
  4. v(t + dt) = v(t + dt/2) + a(t + dt) dt / 2
Frozen atoms are never moved.  Periodic coordinates are wrapped into [lo, hi) after the
drift.  The indenter is a repulsive sphere of radius R: U = (K/3)(R - d)^3 and force
K (R - d)^2 along the outward unit vector, for centre distance d < R (external field,
kept out of the potential-energy sums as the paper prescribes for external forces).
Acceleration units: F [eV/A] / m [amu] * 9648.5332 -> A/ps^2.
"""

from __future__ import annotations

import numpy as np

from . import hybrid as _hyb
from . import precision as _prec
from .geometry import neighbor_csr, min_image

MASS_CU = 63.546  # amu
EV_PER_AMU_A2_PS2 = 9648.5332  # (eV/A)/amu in A/ps^2


def wrap_positions(pos, lo, hi, periodic):
    """Periodic coordinates mapped into [lo, hi)."""
    out = pos.copy()
    for k in range(3):
        if periodic[k]:
            L = hi[k] - lo[k]
            out[k] = lo[k] + np.mod(out[k] - lo[k], L)
            out[k] = np.where(out[k] >= hi[k], lo[k], out[k])
    return out


def indenter(pos, lo, hi, periodic, center, radius, k):
    """(force [3, n], energy) of the spherical indenter."""
    box = np.asarray(hi) - np.asarray(lo)
    d = np.stack([min_image(pos[c] - center[c], box[c], periodic[c]) for c in range(3)])
    dist = np.sqrt((d * d).sum(axis=0))
    inside = dist < radius
    f = np.zeros_like(pos)
    pen = np.where(inside, radius - dist, 0.0)
    safe = np.where(inside, dist, 1.0)
    f[:, inside] = (k * pen[inside] ** 2 / safe[inside]) * d[:, inside]
    return f, float((k / 3.0 * pen ** 3).sum())


def kinetic(v, mass=MASS_CU):
    return 0.5 * mass * float((v * v).sum()) / EV_PER_AMU_A2_PS2


def run(system, eam_p, ace_p, prec_p, dt, n_steps, precision_every=0, w=None,
        indent=None, mass=MASS_CU):
    """Integrate ``n_steps``; returns dict(x, v, w, f, e_pot, e_kin per step incl. t=0)."""
    s = system.copy()
    x = s.pos.copy()
    v = np.zeros_like(x) if s.vel is None else s.vel.copy()
    mobile = np.ones(s.n, bool) if s.frozen is None else ~s.frozen.astype(bool)
    rc = max(eam_p.rc, ace_p.rc if ace_p is not None else 0.0)

    def forces(xx, ww, t):
        s.pos = xx
        ev = _hyb.evaluate(s, eam_p, ace_p, ww)
        f = ev["f"]
        if indent is not None:
            c = np.asarray(indent["center"]) + t * np.asarray(indent["velocity"])
            fi, _ = indenter(xx, s.lo, s.hi, s.periodic, c, indent["radius"], indent["k"])
            f = f + fi
        return f, ev["e_pot"]

    def weights(xx):
        s.pos = xx
        csr = neighbor_csr(xx, s.lo, s.hi, s.periodic, rc)
        return _prec.compute_precision(s, prec_p, csr)["w"]

    if w is None:
        w = weights(x) if prec_p is not None else np.zeros(s.n)
    f, ep = forces(x, w, 0.0)
    e_pot, e_kin = [ep], [kinetic(v[:, mobile], mass)]
    c = 0.5 * dt * EV_PER_AMU_A2_PS2 / mass
    for step in range(1, n_steps + 1):
        v[:, mobile] += c * f[:, mobile]
        x[:, mobile] += dt * v[:, mobile]
        x = wrap_positions(x, s.lo, s.hi, s.periodic)
        if precision_every and step % precision_every == 0:
            w = weights(x)
        f, ep = forces(x, w, step * dt)
        v[:, mobile] += c * f[:, mobile]
        e_pot.append(ep)
        e_kin.append(kinetic(v[:, mobile], mass))
    return dict(x=x, v=v, w=w, f=f, e_pot=np.array(e_pot), e_kin=np.array(e_kin))

"""Velocity-Verlet integration with the switching-parameter update (oracle), eq. vv.

One step of length dt (Sec. II C 1):
  1. v(t + dt/2) = v(t) + a(t) dt / 2;   x(t + dt) = x(t) + v(t + dt/2) dt
  2. w(t + dt) recomputed from x(t + dt) (every ``precision_every`` steps; never if 0)
  3. a(t + dt) = F(t + dt) / m with the new weights (plus the external indenter force)
  4. v(t + dt) = v(t + dt/2) + a(t + dt) dt / 2
Time-averaged weights (``avg``; Appendix B) take one sample per update.  With the "past"
window the sample of step t is taken after that step's forces (the force routine's order
fast potential, precise potential, CSP, lambda of Appendix G), and the weight it forms is
used from step t + 1 on; with the "current" window and with instantaneous weights the
update precedes the forces, as in step 2 above.
The local thermostat (``thermostat``; Sec. II C 2, Appendix C) runs at the end of every
step whose force evaluation uses weights different from the previous one: the forces of
both weight sets at x(t + dt) give the energy errors, and the momenta are rescaled
(``oracle.thermostat``).
Frozen atoms are never moved.  Periodic coordinates are wrapped into [lo, hi) after the
drift.  The indenter is a repulsive sphere of radius R: U = (K/3)(R - d)^3 and force
K (R - d)^2 along the outward unit vector, for centre distance d < R (external field,
kept out of the potential-energy sums as the paper prescribes for external forces).
Acceleration units: F [eV/A] / m [amu] * 9648.5332 -> A/ps^2.
"""

from __future__ import annotations

import numpy as np

from . import averaging as _avg
from . import hybrid as _hyb
from . import precision as _prec
from . import thermostat as _thermo
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
        indent=None, mass=MASS_CU, avg=None, thermostat=None):
    """Integrate ``n_steps``; returns dict(x, v, w, f, e_pot, e_kin per step incl. t=0, and
    per step the thermostat's record).

    ``avg``: dict(n_avg, dw_min, window) for time-averaged weights; ``thermostat``:
    dict(r_omega, omega_max, seed)."""
    s = system.copy()
    x = s.pos.copy()
    v = np.zeros_like(x) if s.vel is None else s.vel.copy()
    mobile = np.ones(s.n, bool) if s.frozen is None else ~s.frozen.astype(bool)
    rc = max(eam_p.rc, ace_p.rc if ace_p is not None else 0.0)
    tas = None
    if avg is not None:
        tas = _avg.TimeAveragedSwitch(avg["n_avg"], avg["dw_min"], avg.get("window", "past"))
    after_forces = tas is not None and tas.window == "past"

    def evaluate(xx, ww):
        s.pos = xx
        return _hyb.evaluate(s, eam_p, ace_p, ww)

    def external(xx, t):
        if indent is None:
            return 0.0
        c = np.asarray(indent["center"]) + t * np.asarray(indent["velocity"])
        return indenter(xx, s.lo, s.hi, s.periodic, c, indent["radius"], indent["k"])[0]

    def weights(xx):
        s.pos = xx
        csr = neighbor_csr(xx, s.lo, s.hi, s.periodic, rc)
        if tas is not None:
            return tas.update(s, prec_p, csr)["w"]
        return _prec.compute_precision(s, prec_p, csr)["w"]

    if w is None:
        w = weights(x) if prec_p is not None else np.zeros(s.n)
    ev = evaluate(x, w)
    f = ev["f"] + external(x, 0.0)
    e_pot, e_kin, records = [ev["e_pot"]], [kinetic(v[:, mobile], mass)], []
    c = 0.5 * dt * EV_PER_AMU_A2_PS2 / mass
    w_used = w  # weights of the last force evaluation
    for step in range(1, n_steps + 1):
        v[:, mobile] += c * f[:, mobile]
        x[:, mobile] += dt * v[:, mobile]
        x = wrap_positions(x, s.lo, s.hi, s.periodic)
        due = bool(precision_every) and step % precision_every == 0
        if due and not after_forces:
            w = weights(x)
        ev = evaluate(x, w)
        v_half = v.copy()
        f = ev["f"] + external(x, step * dt)
        v[:, mobile] += c * f[:, mobile]
        rec = None
        if thermostat is not None and np.any(w != w_used):
            ec = evaluate(x, w_used)
            e_prec = np.where(w > 0.0, ev["e_ace"], ec["e_ace"])
            dE, _, _ = _thermo.energy_errors(w_used, w, ev["e_eam"], e_prec, ec["f"], ev["f"], v_half, dt, mass,
                                             mobile)
            s.pos = x
            rec = _thermo.correct(x, s.lo, s.hi, s.periodic, v, dE, mobile, mass, thermostat["r_omega"],
                                  thermostat["omega_max"], thermostat["seed"], step)
            rec["dE"] = dE
            rec["e_pot_ref"] = ec["e_pot"]  # the constant-weight reference at this step
            v_ref = v_half + c * (ec["f"] + external(x, step * dt))
            rec["e_kin_ref"] = kinetic(v_ref[:, mobile], mass)
        records.append(rec)
        w_used = w
        if due and after_forces:
            w = weights(x)
        e_pot.append(ev["e_pot"])
        e_kin.append(kinetic(v[:, mobile], mass))
    return dict(x=x, v=v, w=w, w_used=w_used, f=f, e_pot=np.array(e_pot), e_kin=np.array(e_kin),
                thermostat=records)

"""Local thermostat (oracle; test infrastructure only, never called by the library).

Energy correction of a weight update, Sec. II C 2 and Appendix C, in the precise-weight form
w = 1 - lambda.  A step whose weights change from w^c (the constant reference, the weights
of the previous force evaluation) to w^d (the updated ones) is finished for both sets at
the same positions x(t+dt); with the gradient of the weights neglected (eq. F_i_d) the
forces are F^c (weights w^c) and F^d (weights w^d), interatomic only (external forces such
as the indenter are left out).  Per mobile atom:
* eq. Delta_V_i:  dV_i = E^c_i - E^d_i = (w^d_i - w^c_i) (E^fast_i - E^precise_i);
* eq. Delta_T_i:  dT_i = sum_a [ dt^2 / (8 m) ((F^c_ia)^2 - (F^d_ia)^2) + (F^c_ia - F^d_ia) v_ia(t+dt/2) dt / 2 ]
  (m in eV ps^2 / A^2, i.e. the mass in amu divided by 9648.5332);
* eq. Delta_E_i:  dE_i = dT_i + dV_i.
Every mobile atom with dE_i != 0 is corrected by rescaling the momenta of a group Omega_i
relative to the group's centre-of-mass velocity (eq. p_resc_omega), with the factor of
eq. beta_omega_i, beta = sqrt(dE_i / K_rel + 1), K_rel = sum_{j in Omega_i} p_rel,j^2 / (2 m_j):
the group's momentum is unchanged and its kinetic energy changes by exactly dE_i.  The
positive root is taken (Appendix C).  A negative radicand (dE_i < -K_rel), or K_rel = 0 with
dE_i != 0, cannot be corrected: that atom's correction is skipped and reported
(Appendix D discusses such cases).

Readings (the paper leaves these open):
* Omega_i is atom i plus a random selection of the mobile atoms j != i within r_omega of i
  (minimum image, r^2 < r_omega^2 at x(t+dt)), at most |Omega| - 1 of them (Appendix F:
  |Omega_i| = 800): all of them if there are fewer, else the |Omega| - 1 with the smallest
  random priority.  The paper draws from the neighbour list of i; r_omega is that list's
  radius.
* The priority of candidate j for atom i at step s is the first 64-bit word of the
  counter-based generator Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11) with counter
  (i, j, s, 0) and key (seed, 0); ties (equal words) go to the smaller j.
* Corrections are applied one after the other, each on the momenta the previous ones left
  (beta depends on the momenta before its rescale, Appendix C).  Order: by colour, then
  by atom index.  The colour of an atom is the parity pattern (cx & 1) + 2 (cy & 1) +
  4 (cz & 1) of its cell in a grid of nc_d = floor(L_d / (2 r_omega)) cells per axis
  (at least 1; a periodic axis with an odd count above 1 uses one cell fewer), cell index
  floor((x_d - lo_d) * (nc_d / L_d)) clamped to [0, nc_d).  Atoms of one colour in
  different cells are at least 2 r_omega apart along some axis, so their groups are
  disjoint and their corrections commute: any order within a colour that keeps each cell's
  atoms ascending gives the same result.
"""

from __future__ import annotations

import math

import numpy as np

from .geometry import displacements, sq_dist

EV_PER_AMU_A2_PS2 = 9648.5332

_M64 = (1 << 64) - 1
_PHILOX_M = (0xD2E7470EE14C6C93, 0xCA5A826395121157)
_PHILOX_W = (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)


def philox4x64_10(ctr, key):
    """Philox4x64 with 10 rounds: counter (4 x 64 bit), key (2 x 64 bit) -> 4 x 64 bit.

    A round maps (c0, c1, c2, c3) to (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1,
    lo(M0 c0)) with 128-bit products; the key is bumped by the Weyl constants before every
    round but the first."""
    c0, c1, c2, c3 = (int(v) & _M64 for v in ctr)
    k0, k1 = (int(v) & _M64 for v in key)
    for r in range(10):
        if r:
            k0 = (k0 + _PHILOX_W[0]) & _M64
            k1 = (k1 + _PHILOX_W[1]) & _M64
        p0 = _PHILOX_M[0] * c0
        p1 = _PHILOX_M[1] * c2
        c0, c1, c2, c3 = (p1 >> 64) ^ c1 ^ k0, p1 & _M64, (p0 >> 64) ^ c3 ^ k1, p0 & _M64
    return c0, c1, c2, c3


def priority(seed: int, step: int, i: int, j: int) -> int:
    """Random priority of candidate j in the group of atom i at step ``step``."""
    return philox4x64_10((i, j, step, 0), (seed, 0))[0]


def energy_errors(w_c, w_d, e_fast, e_precise, f_c, f_d, v_half, dt, mass, mobile):
    """dE_i = dT_i + dV_i of every atom (0 for frozen ones); returns (dE, dV, dT)."""
    w_c = np.asarray(w_c, dtype=np.float64)
    w_d = np.asarray(w_d, dtype=np.float64)
    changed = w_c != w_d
    dV = np.where(changed, (w_d - w_c) * (np.where(changed, e_fast, 0.0) - np.where(changed, e_precise, 0.0)), 0.0)
    a = dt * dt * EV_PER_AMU_A2_PS2 / (8.0 * mass)
    dT = np.zeros_like(dV)
    for c in range(3):
        dT = dT + (a * (f_c[c] * f_c[c] - f_d[c] * f_d[c]) + (f_c[c] - f_d[c]) * v_half[c] * (0.5 * dt))
    mob = np.asarray(mobile, dtype=bool)
    dV = np.where(mob, dV, 0.0)
    dT = np.where(mob, dT, 0.0)
    return dV + dT, dV, dT


def colour_grid(lo, hi, periodic, r_omega):
    """Cells per axis of the colouring grid."""
    nc = []
    for d in range(3):
        L = float(hi[d] - lo[d])
        k = max(1, int(math.floor(L / (2.0 * r_omega))))
        if periodic[d] and k > 1 and k % 2:
            k -= 1
        nc.append(k)
    return nc


def colours(pos, lo, hi, periodic, r_omega):
    """Colour (0..7) and cell index of every atom."""
    nc = colour_grid(lo, hi, periodic, r_omega)
    cell = []
    for d in range(3):
        inv = nc[d] / float(hi[d] - lo[d])
        c = np.floor((pos[d] - lo[d]) * inv).astype(np.int64)
        cell.append(np.clip(c, 0, nc[d] - 1))
    colour = (cell[0] & 1) + 2 * (cell[1] & 1) + 4 * (cell[2] & 1)
    flat = cell[0] + nc[0] * (cell[1] + nc[1] * cell[2])
    return colour, flat


def group(pos, lo, hi, periodic, i, mobile, r_omega, omega_max, seed, step):
    """Omega_i: atom i followed by its selected candidates in ascending index."""
    n = pos.shape[1]
    box = np.asarray(hi, dtype=np.float64) - np.asarray(lo, dtype=np.float64)
    jj = np.arange(n)
    dx, dy, dz = displacements(pos, box, periodic, np.full(n, i), jj)
    r2 = sq_dist(dx, dy, dz)
    cand = np.nonzero(np.asarray(mobile, dtype=bool) & (r2 < r_omega * r_omega) & (jj != i))[0]
    if cand.size + 1 > omega_max:
        keys = [(priority(seed, step, i, int(j)), int(j)) for j in cand]
        keys.sort()
        cand = np.sort(np.array([j for _, j in keys[:omega_max - 1]], dtype=np.int64))
    return np.concatenate([[i], cand]).astype(np.int64)


def rescale_group(v, members, dE, mass):
    """eqs. p_resc_omega, beta_omega_i on the velocities v [3, n] (in place).

    Returns beta, or None when the radicand is negative or the group has no relative
    momentum (the velocities are then left unchanged)."""
    vg = v[:, members]
    vcm = vg.sum(axis=1) / float(members.size)  # equal masses: the plain mean
    rel = vg - vcm[:, None]
    k_rel = 0.5 * mass / EV_PER_AMU_A2_PS2 * float((rel * rel).sum())
    if not k_rel > 0.0:
        return None
    rad = dE / k_rel + 1.0
    if not rad >= 0.0:
        return None
    beta = math.sqrt(rad)
    v[:, members] = vcm[:, None] + beta * rel
    return beta


def correct(pos, lo, hi, periodic, vel, dE, mobile, mass, r_omega, omega_max, seed, step):
    """Applies every correction of one step to ``vel`` (in place); returns a dict with the
    corrected atoms in their order, their group sizes and betas, and the failures."""
    dE = np.asarray(dE, dtype=np.float64)
    todo = np.nonzero((dE != 0.0) & np.asarray(mobile, dtype=bool))[0]
    colour, _ = colours(pos, lo, hi, periodic, r_omega)
    order = todo[np.lexsort((todo, colour[todo]))]
    betas, sizes, failed = [], [], []
    for i in order:
        members = group(pos, lo, hi, periodic, int(i), mobile, r_omega, omega_max, seed, step)
        b = rescale_group(vel, members, float(dE[i]), mass)
        sizes.append(members.size)
        betas.append(b)
        if b is None:
            failed.append(int(i))
    return dict(order=order, sizes=np.array(sizes, dtype=np.int64), betas=betas, failed=failed)


__all__ = ["philox4x64_10", "priority", "energy_errors", "colour_grid", "colours", "group", "rescale_group",
           "correct"]

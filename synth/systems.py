"""Geometry of the synthetic Cu-like test systems (inputs only).

Units are LAMMPS "metal": Angstrom, eV, ps, amu, K.  Positions are stored as a
``float64`` array of shape ``[3, n]`` (structure of arrays: x row, y row, z row),
the layout the library takes on the device.
"""

from __future__ import annotations

import dataclasses

import numpy as np

A_CU = 3.615  # FCC lattice constant of the synthetic copper (Angstrom)
MASS_CU = 63.546  # amu
KB_EV = 8.617333262e-5  # Boltzmann constant, eV/K
# 1 eV/amu expressed in Angstrom^2/ps^2 (CODATA e and u): converts F/m to an acceleration.
EV_PER_AMU_A2_PS2 = 9648.5332


@dataclasses.dataclass
class System:
    """An atomic configuration plus its simulation box.

    ``pos`` is ``[3, n]`` float64, ``lo``/``hi`` are box bounds, ``periodic`` flags per
    dimension, ``frozen`` an optional uint8 mask of atoms that never move and always use
    the fast potential, ``vel`` optional ``[3, n]`` velocities in Angstrom/ps.
    """

    pos: np.ndarray
    lo: np.ndarray
    hi: np.ndarray
    periodic: tuple
    frozen: np.ndarray | None = None
    vel: np.ndarray | None = None
    name: str = ""
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.pos.shape[1])

    @property
    def box(self) -> np.ndarray:
        return self.hi - self.lo

    def copy(self) -> "System":
        return System(
            self.pos.copy(), self.lo.copy(), self.hi.copy(), tuple(self.periodic),
            None if self.frozen is None else self.frozen.copy(),
            None if self.vel is None else self.vel.copy(), self.name, dict(self.meta))


def fcc_positions(nx: int, ny: int, nz: int, a: float = A_CU) -> np.ndarray:
    """Sites of an ``nx x ny x nz`` block of conventional FCC cells, ``[3, 4*nx*ny*nz]``.

    Sites are ordered cell by cell (x fastest, then y, then z), four basis sites per
    cell, so that consecutive indices are spatial neighbours.
    """
    basis = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]])
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    cells = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    pts = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3) * a
    return np.ascontiguousarray(pts.T)


def fcc111_positions(nx: int, ny: int, nz: int, a: float = A_CU):
    """FCC sites in an orthorhombic cell with x=[1-10], y=[11-2], z=[111].

    Returns ``(pos [3, 6*nx*ny*nz], lengths)``; the cell repeats are
    ``a/sqrt(2)``, ``a*sqrt(6)/2`` and ``a*sqrt(3)`` along x, y, z.
    """
    ex = np.array([1.0, -1.0, 0.0]) / np.sqrt(2.0)
    ey = np.array([1.0, 1.0, -2.0]) / np.sqrt(6.0)
    ez = np.array([1.0, 1.0, 1.0]) / np.sqrt(3.0)
    rot = np.stack([ex, ey, ez])
    lengths = np.array([nx * a / np.sqrt(2.0), ny * a * np.sqrt(6.0) / 2.0, nz * a * np.sqrt(3.0)])
    # enumerate conventional cells generously, rotate, keep those inside the box
    span = int(np.ceil(lengths.max() / a)) * 2 + 2
    g = np.arange(-span, span + 1, dtype=np.float64)
    basis = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]])
    out = []
    for b in basis:
        cx, cy, cz = np.meshgrid(g + b[0], g + b[1], g + b[2], indexing="ij")
        p = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1) * a
        q = p @ rot.T
        tol = 1e-7
        keep = np.all((q > -tol) & (q < lengths - tol), axis=1)
        out.append(q[keep])
    q = np.concatenate(out)
    q = np.where(np.abs(q) < 1e-7, 0.0, q)
    order = np.lexsort((q[:, 0], q[:, 1], q[:, 2]))
    q = q[order]
    expect = 6 * nx * ny * nz
    if q.shape[0] != expect:
        raise RuntimeError(f"fcc111 enumeration found {q.shape[0]} sites, expected {expect}")
    return np.ascontiguousarray(q.T), lengths


def remove_random_sites(pos: np.ndarray, k: int, rng: np.random.Generator) -> np.ndarray:
    """Delete ``k`` distinct sites chosen by ``rng.choice`` (one draw)."""
    drop = rng.choice(pos.shape[1], size=k, replace=False)
    keep = np.ones(pos.shape[1], dtype=bool)
    keep[drop] = False
    return np.ascontiguousarray(pos[:, keep])


def remove_sphere(pos: np.ndarray, center, radius: float, box, periodic) -> np.ndarray:
    """Delete every site whose minimum-image distance to ``center`` is below ``radius``."""
    d = pos - np.asarray(center, dtype=np.float64)[:, None]
    for k in range(3):
        if periodic[k]:
            d[k] -= box[k] * np.round(d[k] / box[k])
    r2 = (d * d).sum(axis=0)
    return np.ascontiguousarray(pos[:, r2 >= radius * radius])


def gaussian_displace(pos: np.ndarray, sigma: float, rng: np.random.Generator) -> np.ndarray:
    """Add independent N(0, sigma^2) displacements to every component (one draw)."""
    return pos + rng.normal(0.0, sigma, size=pos.shape)


def thermal_sigma(temperature: float, a: float = A_CU) -> float:
    """Per-component displacement of an uncorrelated-Gaussian thermal proxy.

    Scales 0.083 Angstrom at 300 K with sqrt(T) (classical equipartition of an
    Einstein oscillator).  Used to make hot-looking snapshots without running dynamics.
    """
    return 0.083 * float(np.sqrt(temperature / 300.0))


def wrap_positions(pos: np.ndarray, lo, hi, periodic) -> np.ndarray:
    """Map periodic coordinates into ``[lo, hi)``."""
    out = pos.copy()
    for k in range(3):
        if periodic[k]:
            L = hi[k] - lo[k]
            out[k] = lo[k] + np.mod(out[k] - lo[k], L)
            out[k] = np.where(out[k] >= hi[k], lo[k], out[k])
    return out


def maxwell_velocities(n: int, temperature: float, rng: np.random.Generator,
                       mobile: np.ndarray | None = None, mass: float = MASS_CU) -> np.ndarray:
    """Maxwell-Boltzmann velocities (Angstrom/ps) at exactly ``temperature``.

    Components are drawn N(0, kT/m), the centre-of-mass velocity of the mobile atoms is
    removed, and the result is rescaled so that the kinetic temperature with
    ``3*n_mobile - 3`` degrees of freedom equals ``temperature``.  Immobile atoms get 0.
    """
    var = KB_EV * temperature / mass * EV_PER_AMU_A2_PS2
    v = rng.normal(0.0, np.sqrt(var), size=(3, n))
    if mobile is None:
        mobile = np.ones(n, dtype=bool)
    mobile = mobile.astype(bool)
    v[:, ~mobile] = 0.0
    nm = int(mobile.sum())
    if nm < 2 or temperature <= 0.0:
        return np.zeros((3, n))
    v[:, mobile] -= v[:, mobile].mean(axis=1, keepdims=True)
    ke = 0.5 * mass * (v[:, mobile] ** 2).sum() / EV_PER_AMU_A2_PS2
    t_now = 2.0 * ke / ((3 * nm - 3) * KB_EV)
    v *= np.sqrt(temperature / t_now)
    return v

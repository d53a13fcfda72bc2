"""The five workload families, built from seeded geometry only.

* ``cfg0``   864-site FCC block (6x6x6 cells), 4 random vacancies, sigma = 0.05 A noise.
* ``cfg0_static`` the same without noise (exact-geometry spreading checks).
* ``cfg1``   32x32x32 cells with a 12 A spherical void, 300 K Maxwell velocities.
* ``cfg2``   100x100x100 cells, periodic in x/y, free z surfaces, bottom three (002)
  planes frozen, spherical indenter above the top surface.
* ``cfg3``   16x16x16 cells at 300/800/1200 K (Gaussian thermal proxy), with vacancies,
  and an FCC(111) slab.
* ``cfg4``   training snapshots for the learned indicator (bulk, vacancies, voids, slabs).

Seeds are ``20241105 + index`` unless stated otherwise; every random quantity is drawn
from one ``numpy.random.default_rng`` stream in the order written in each builder.
"""

from __future__ import annotations

import numpy as np

from .systems import (A_CU, System, fcc_positions, fcc111_positions, gaussian_displace,
                      maxwell_velocities, remove_random_sites, remove_sphere, thermal_sigma,
                      wrap_positions)

SEED0 = 20241105


def _periodic_box(nx, ny, nz, a=A_CU):
    return np.zeros(3), np.array([nx * a, ny * a, nz * a])


def cfg0(seed: int = SEED0, sigma: float = 0.05, cells: int = 6, vacancies: int = 4) -> System:
    """6x6x6 FCC cells (a = 3.615 A), periodic, ``vacancies`` random vacancies, then
    Gaussian displacements.  Draw order: vacancy choice, displacements."""
    rng = np.random.default_rng(seed)
    pos = fcc_positions(cells, cells, cells)
    lo, hi = _periodic_box(cells, cells, cells)
    if vacancies:
        pos = remove_random_sites(pos, vacancies, rng)
    if sigma > 0.0:
        pos = gaussian_displace(pos, sigma, rng)
    pos = wrap_positions(pos, lo, hi, (1, 1, 1))
    return System(pos, lo, hi, (1, 1, 1), name=f"cfg0(sigma={sigma},vac={vacancies})")


def cfg0_static(seed: int = SEED0) -> System:
    return cfg0(seed=seed, sigma=0.0)


def bulk(cells: int, seed: int, temperature: float = 0.0, vacancies: int = 0,
         void_radius: float = 0.0, velocities: bool = False, sigma: float | None = None) -> System:
    """Periodic ``cells^3`` FCC block with optional vacancies, a central void, thermal
    displacements (Gaussian proxy at ``temperature``) and Maxwell velocities.
    Draw order: vacancies, displacements, velocities."""
    rng = np.random.default_rng(seed)
    pos = fcc_positions(cells, cells, cells)
    lo, hi = _periodic_box(cells, cells, cells)
    if void_radius > 0.0:
        pos = remove_sphere(pos, 0.5 * (lo + hi), void_radius, hi - lo, (1, 1, 1))
    if vacancies:
        pos = remove_random_sites(pos, vacancies, rng)
    s = thermal_sigma(temperature) if sigma is None else sigma
    if s > 0.0:
        pos = gaussian_displace(pos, s, rng)
    pos = wrap_positions(pos, lo, hi, (1, 1, 1))
    vel = maxwell_velocities(pos.shape[1], temperature, rng) if velocities else None
    return System(pos, lo, hi, (1, 1, 1), vel=vel,
                  name=f"bulk{cells}(T={temperature},vac={vacancies},void={void_radius})")


def cfg1(seed: int = SEED0 + 1, cells: int = 32, void_radius: float = 12.0,
         temperature: float = 300.0) -> System:
    """32^3 cells, sites within 12 A of the box centre removed, 300 K Maxwell velocities
    on the perfect lattice."""
    return bulk(cells, seed, temperature=temperature, void_radius=void_radius,
                velocities=True, sigma=0.0)


def slab100(nx: int, ny: int, nz: int, seed: int, temperature: float = 300.0,
            frozen_planes: int = 3, vacuum: float = 10.0, sigma: float | None = None,
            velocities: bool = True) -> System:
    """FCC block periodic in x/y with free (001) surfaces.  The lowest ``frozen_planes``
    (002) planes are frozen.  The box extends ``vacuum`` beyond the atoms in z."""
    rng = np.random.default_rng(seed)
    a = A_CU
    pos = fcc_positions(nx, ny, nz)
    zmin, zmax = pos[2].min(), pos[2].max()
    frozen = (pos[2] < zmin + (frozen_planes - 0.5) * 0.5 * a).astype(np.uint8)
    s = 0.0 if sigma is None else sigma
    if s > 0.0:
        d = rng.normal(0.0, s, size=pos.shape)
        d[:, frozen.astype(bool)] = 0.0
        pos = pos + d
    lo = np.array([0.0, 0.0, zmin - vacuum])
    hi = np.array([nx * a, ny * a, zmax + vacuum])
    pos = wrap_positions(pos, lo, hi, (1, 1, 0))
    vel = maxwell_velocities(pos.shape[1], temperature, rng, mobile=~frozen.astype(bool)) \
        if velocities else None
    sysm = System(pos, lo, hi, (1, 1, 0), frozen=frozen, vel=vel,
                  name=f"slab100({nx}x{ny}x{nz},T={temperature})")
    sysm.meta["z_top"] = float(zmax)
    return sysm


def cfg2(seed: int = SEED0 + 2, cells: int = 100, temperature: float = 300.0,
         radius: float = 40.0, k: float = 10.0, speed: float = 0.2) -> System:
    """Nanoindentation-like block: ``cells^3`` FCC cells, x/y periodic, z free, bottom
    three (002) planes frozen, 300 K Maxwell velocities, spherical indenter of radius
    ``radius`` whose centre starts at (Lx/2, Ly/2, z_top + radius) and moves -z."""
    s = slab100(cells, cells, cells, seed, temperature=temperature)
    L = s.hi - s.lo
    s.meta.update(indenter=dict(radius=radius, k=k,
                                center=[s.lo[0] + 0.5 * L[0], s.lo[1] + 0.5 * L[1],
                                        s.meta["z_top"] + radius],
                                velocity=[0.0, 0.0, -speed]))
    s.name = f"cfg2({cells}^3 indentation)"
    return s


def cfg3(kind: str, seed: int = SEED0 + 3, cells: int = 16) -> System:
    """Differentiation workloads on 16^3 cells: ``T300``/``T800``/``T1200`` thermal
    snapshots, ``vac`` (8 vacancies at 300 K) and ``slab111`` (FCC(111) slab at 300 K)."""
    if kind.startswith("T"):
        return bulk(cells, seed, temperature=float(kind[1:]))
    if kind == "vac":
        return bulk(cells, seed, temperature=300.0, vacancies=8)
    if kind == "slab111":
        rng = np.random.default_rng(seed)
        pos, L = fcc111_positions(16, 10, 17)  # 16,320 sites, the closest to 16,384
        pos = gaussian_displace(pos, thermal_sigma(300.0), rng)
        lo = np.array([0.0, 0.0, -10.0])
        hi = np.array([L[0], L[1], L[2] + 10.0])
        pos = wrap_positions(pos, lo, hi, (1, 1, 0))
        return System(pos, lo, hi, (1, 1, 0), name="slab111(300K)")
    raise ValueError(kind)


def cfg4_snapshot(index: int, seed: int = SEED0 + 4, cells: int = 16) -> System:
    """Starting state of training snapshot ``index`` (0..199): structure family =
    index % 4 (bulk, 1 % vacancies, 8 A void, (100) slab), target temperature
    T = {300, 600, 900, 1200}[(index // 4) % 4].  Atoms sit on their lattice sites with
    Maxwell velocities at 2T; integrating it with the fast potential (``meta['md_steps']``
    steps of 1 fs) brings it to about T by equipartition."""
    fam = index % 4
    T = [300.0, 600.0, 900.0, 1200.0][(index // 4) % 4]
    sd = seed * 1000 + index
    if fam == 0:
        s = bulk(cells, sd, temperature=2 * T, velocities=True, sigma=0.0)
    elif fam == 1:
        s = bulk(cells, sd, temperature=2 * T, vacancies=int(round(0.01 * 4 * cells ** 3)), velocities=True,
                 sigma=0.0)
    elif fam == 2:
        s = bulk(cells, sd, temperature=2 * T, void_radius=8.0, velocities=True, sigma=0.0)
    else:
        s = slab100(cells, cells, cells, sd, temperature=2 * T, frozen_planes=0, sigma=0.0, velocities=True)
    s.meta["temperature"] = T
    s.meta["md_steps"] = 500
    return s

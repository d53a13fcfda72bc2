"""Pins of the oracle's EAM2 copper potential (Appendix E, parameters of Table III) against
the properties the paper prints for it in Table II (CPU only).

Table II gives, for the original EAM2 parameters and for the paper's refit, the FCC lattice
constant, the cohesive energy, the elastic constants C11, C12, C44, the vacancy formation
energy and the (111), (100) and (110) surface energies (the LaTeX source carries them to
full precision; the table rounds).  They are computed here from the oracle's pair, density
and embedding functions:
* bulk values by lattice sums over a perfect FCC crystal: minimising the energy per atom
  over the lattice constant, and central second differences of the energy density under
  small homogeneous strains (a monatomic Bravais lattice has no internal relaxation, so
  these are the elastic constants);
* the vacancy and surface energies on relaxed structures: one site removed from a periodic
  6x6x6-cell crystal, or a slab periodic in its plane with two free faces, relaxed at fixed
  cell by L-BFGS on the oracle's energy with its autograd forces.
Atoms next to a vacancy or in a surface have less than unit density, where the embedding's
q2..q4 terms act, so the defect energies pin them.  The relaxed <100> dumbbell and
tetrahedral interstitials (Table II) bring neighbours to 2.17-2.20 A, inside the reach of the
first short-range repulsion S_1 (2.24 A); its share of their energy is 1e-4 eV for the
original set.  Parity unpinned: S_2 and S_3 act only below 1.80 and 1.20 A, which no printed
value reaches.
"""

import numpy as np
import pytest
import torch
from scipy.optimize import minimize, minimize_scalar

import synth
from oracle import eam as oeam
from oracle import geometry

EV_PER_A3_IN_GPA = 160.21766208

EV_PER_A2_IN_J_PER_M2 = 16.02176634

# Table II (EAM original, EAM fit)
TABLE2 = {
    "original": dict(a0=3.61492887282983, e_coh=-3.55786833489833, c11=171.453901566772, c12=124.157217644317,
                     c44=76.2101973267168),
    "fit": dict(a0=3.63045256622797, e_coh=-3.69569662929878, c11=171.288636692165, c12=120.145974948912,
                c44=80.5610917066166),
}
# Table II: relaxed vacancy formation energy (eV) and surface energies (J/m^2)
TABLE2_DEFECTS = {
    "original": dict(vacancy=1.27349604826122, s111=1.24430605633688, s100=1.35153002045502,
                     s110=1.48217604297006),
    "fit": dict(vacancy=1.0588710171005, s111=0.88024354655695, s100=0.97649687173991, s110=1.12251374356068),
}
# Table II: interstitial formation energies (eV): <100> dumbbell, octahedral, tetrahedral
TABLE2_INTERSTITIALS = {
    "original": dict(dumbbell=3.08094456110825, octahedral=3.2558783098782, tetrahedral=3.5655217348783),
    "fit": dict(dumbbell=2.96618403515875, octahedral=3.13034901463887, tetrahedral=3.42395856517813),
}


def _lattice_vectors(reach=2.5):
    """FCC lattice vectors in units of a, 0 < |u| < reach."""
    k = np.arange(-3, 4)
    cells = np.array([(i, j, l) for i in k for j in k for l in k], float)
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    u = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3)
    norm = np.linalg.norm(u, axis=1)
    return u[(norm > 1e-9) & (norm < reach)]


U = _lattice_vectors()


def _energy(p, a, strain=None):
    """Energy per atom of the (strained) perfect crystal: xi(sum zeta) + 1/2 sum Phi."""
    R = U * a
    if strain is not None:
        R = R @ (np.eye(3) + strain).T
    r = torch.as_tensor(np.linalg.norm(R, axis=1))
    r = r[r < p.rc]
    rho = oeam.pair_rho(r, p).sum().reshape(1)
    return float(oeam.embed(rho, p)[0] + 0.5 * oeam.pair_phi(r, p).sum())


def _properties(p):
    res = minimize_scalar(lambda a: _energy(p, a), bounds=(3.5, 3.7), method="bounded", options={"xatol": 1e-12})
    a0 = res.x
    e0 = _energy(p, a0)
    vol = a0 ** 3 / 4.0
    h = 1e-4

    def second(direction):
        return (_energy(p, a0, h * direction) + _energy(p, a0, -h * direction) - 2.0 * e0) / (h * h * vol)

    e11 = np.zeros((3, 3))
    e11[0, 0] = 1.0
    e12 = np.diag([1.0, 1.0, 0.0])
    g23 = np.zeros((3, 3))
    g23[1, 2] = g23[2, 1] = 0.5  # engineering shear strain 1 in the 23 plane
    c11 = second(e11) * EV_PER_A3_IN_GPA
    c11_plus_c12 = 0.5 * second(e12) * EV_PER_A3_IN_GPA
    c44 = second(g23) * EV_PER_A3_IN_GPA
    return dict(a0=a0, e_coh=e0, c11=c11, c12=c11_plus_c12 - c11, c44=c44)


@pytest.mark.parametrize("name,params", [("original", synth.eam2_original()), ("fit", synth.eam2_fit300k())])
def test_eam2_bulk_properties_match_table2(name, params):
    got = _properties(params)
    want = TABLE2[name]
    assert abs(got["a0"] - want["a0"]) < 2e-5, (got["a0"], want["a0"])
    assert abs(got["e_coh"] - want["e_coh"]) < 1e-4, (got["e_coh"], want["e_coh"])
    for c in ("c11", "c12", "c44"):
        assert abs(got[c] - want[c]) < 0.1, (c, got[c], want[c])


def test_eam2_density_term_underflows_and_taper_vanishes():
    # Appendix E's second density term exp(-beta2 (r - r04)) with beta2 = 535.661 /A and
    # r04 = -261.984 A is below the smallest double for every r > 0: it contributes nothing
    p = synth.eam2_original()
    r = torch.tensor([0.5, 2.5, 5.0], dtype=torch.float64)
    assert torch.all(torch.exp(-p.beta2 * (r - p.r04)) == 0.0)
    # pair and density vanish at and beyond the cutoff; the embedding is xi0 + f0 at unit density
    rc = torch.tensor([p.rc, p.rc + 0.3], dtype=torch.float64)
    assert torch.all(oeam.pair_phi(rc, p) == 0.0) and torch.all(oeam.pair_rho(rc, p) == 0.0)
    fit = synth.eam2_fit300k()
    one = torch.ones(1, dtype=torch.float64)
    assert float(oeam.embed(one, fit)[0]) == fit.xi0 + fit.f0


# ------------------------------------------------------------- relaxed defect energies
def _total_energy_and_grad(p, lo, hi, per, n, skin=1.0):
    """x (flattened [3, n]) -> (sum_i E_i, dE/dx) with the oracle's site energies; the pair
    candidates within r_c + skin are refreshed when an atom has moved more than skin/2."""
    box = np.asarray(hi) - np.asarray(lo)
    cache = {}

    def f(x):
        pos = x.reshape(3, n)
        if "ref" not in cache or np.abs(pos - cache["ref"]).max() > 0.5 * skin:
            cache["csr"] = geometry.neighbor_csr(pos, lo, hi, per, p.rc + skin)
            cache["ref"] = pos.copy()
        i, j = geometry.pairs_within(pos, lo, hi, per, p.rc, cache["csr"])
        pt = torch.tensor(pos, dtype=torch.float64, requires_grad=True)
        e = oeam.site_energies(pt, box, per, i, j, p, n).sum()
        (g,) = torch.autograd.grad(e, pt)
        return float(e.detach()), g.numpy().ravel()
    return f


def _relaxed(p, pos, lo, hi, per):
    n = pos.shape[1]
    f = _total_energy_and_grad(p, lo, hi, per, n)
    res = minimize(f, pos.ravel(), jac=True, method="L-BFGS-B",
                   options=dict(maxiter=4000, gtol=1e-8, ftol=0.0, maxcor=30))
    e, g = f(res.x)
    assert np.abs(g).max() < 1e-6, "relaxation did not converge"
    return e, f(pos.ravel())[0]


def _oriented_cell(a, frame):
    """Sites of the orthorhombic FCC cell whose axes are the integer directions `frame`,
    and its edge lengths (the shortest lattice translation along each axis)."""
    F = np.asarray(frame, dtype=float)
    R = F / np.linalg.norm(F, axis=1)[:, None]
    edges = []
    for v in F:
        # lattice translations are half-integer combinations with an even sum of doubles
        k = next(k for k in range(1, 7) if int(round((v * k).sum())) % 2 == 0)
        edges.append(np.linalg.norm(v * k / 2.0))
    edges = np.array(edges)
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    r = np.arange(-6, 7)
    pts = (np.array([(i, j, l) for i in r for j in r for l in r], float)[:, None, :] + basis[None]).reshape(-1, 3)
    q = pts @ R.T
    keep = np.all((q >= -1e-7) & (q < edges - 1e-7), axis=1)
    return q[keep] * a, edges * a


SURFACES = {  # plane: (cell axes with the normal last, repeats); periodic edges >= 2 (r_c + skin)
    "s100": (([1, 0, 0], [0, 1, 0], [0, 0, 1]), (4, 4, 6)),
    "s110": (([0, 0, 1], [1, -1, 0], [1, 1, 0]), (4, 6, 8)),
    "s111": (([1, -1, 0], [1, 1, -2], [1, 1, 1]), (6, 4, 4)),
}


@pytest.mark.parametrize("name,params", [("original", synth.eam2_original()), ("fit", synth.eam2_fit300k())])
def test_eam2_relaxed_vacancy_formation_energy(name, params):
    pr = _properties(params)
    cells = 8
    pos = synth.fcc_positions(cells, cells, cells, pr["a0"])
    n = pos.shape[1]
    lo, hi, per = np.zeros(3), np.full(3, cells * pr["a0"]), (1, 1, 1)
    e_perfect = _total_energy_and_grad(params, lo, hi, per, n)(pos.ravel())[0]
    e_rel, e_unrel = _relaxed(params, pos[:, 1:].copy(), lo, hi, per)
    ef = e_rel - (n - 1) / n * e_perfect
    want = TABLE2_DEFECTS[name]["vacancy"]
    print(f"{name}: vacancy formation {ef:.5f} eV (unrelaxed {e_unrel - (n - 1) / n * e_perfect:.5f}), "
          f"Table II {want:.5f}")
    # 2,048-site periodic cell at the lattice constant: the printed values are reproduced
    # to 1e-5 eV at this size (the relaxation energy converges as 1/volume)
    assert abs(ef - want) < 1e-4


@pytest.mark.parametrize("surface", sorted(SURFACES))
@pytest.mark.parametrize("name,params", [("original", synth.eam2_original()), ("fit", synth.eam2_fit300k())])
def test_eam2_relaxed_surface_energies(name, params, surface):
    pr = _properties(params)
    frame, (nx, ny, nz) = SURFACES[surface]
    cell, edges = _oriented_cell(pr["a0"], frame)
    vac = 12.0
    shifts = [np.array([i * edges[0], j * edges[1], k * edges[2] + vac])
              for i in range(nx) for j in range(ny) for k in range(nz)]
    pos = np.concatenate([cell + s for s in shifts]).T.copy()
    lo = np.zeros(3)
    hi = np.array([nx * edges[0], ny * edges[1], nz * edges[2] + 2 * vac])
    n = pos.shape[1]
    e_rel, _ = _relaxed(params, pos, lo, hi, (1, 1, 0))
    gamma = (e_rel - n * pr["e_coh"]) / (2.0 * hi[0] * hi[1]) * EV_PER_A2_IN_J_PER_M2
    want = TABLE2_DEFECTS[name][surface]
    print(f"{name} {surface}: {gamma:.5f} J/m^2, Table II {want:.5f}")
    assert abs(gamma - want) < 2e-4


@pytest.mark.parametrize("kind", ["dumbbell", "octahedral", "tetrahedral"])
@pytest.mark.parametrize("name,params", [("original", synth.eam2_original()), ("fit", synth.eam2_fit300k())])
def test_eam2_relaxed_interstitial_formation_energies(name, params, kind):
    pr = _properties(params)
    a, cells = pr["a0"], 8
    pos = synth.fcc_positions(cells, cells, cells, a)
    n = pos.shape[1]
    lo, hi, per = np.zeros(3), np.full(3, cells * a), (1, 1, 1)
    e_perfect = _total_energy_and_grad(params, lo, hi, per, n)(pos.ravel())[0]
    centre = np.full(3, cells // 2 * a)
    k = int(np.argmin(((pos - centre[:, None]) ** 2).sum(axis=0)))
    site = pos[:, k].copy()
    if kind == "dumbbell":  # two atoms share site k along [100]; symmetric start
        extra = np.stack([site + [0.3 * a, 0, 0], site - [0.3 * a, 0, 0]], axis=1)
        pos = np.concatenate([np.delete(pos, k, axis=1), extra], axis=1)
    elif kind == "octahedral":
        pos = np.concatenate([pos, (site + [0.5 * a, 0, 0])[:, None]], axis=1)
    else:
        pos = np.concatenate([pos, (site + [0.25 * a, 0.25 * a, 0.25 * a])[:, None]], axis=1)
    e_rel, _ = _relaxed(params, pos, lo, hi, per)
    ef = e_rel - pos.shape[1] / n * e_perfect
    want = TABLE2_INTERSTITIALS[name][kind]
    print(f"{name} {kind}: {ef:.5f} eV, Table II {want:.5f}")
    assert abs(ef - want) < 1e-4

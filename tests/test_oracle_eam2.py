"""Pins of the oracle's EAM2 copper potential (Appendix D) against the bulk properties the
paper prints for it (CPU only).

Appendix D, Table III gives, for the original EAM2 parameters and for the paper's refit,
the FCC lattice constant, the cohesive energy and the elastic constants C11, C12, C44 (the
LaTeX source carries them to full precision; the table rounds).  They are computed here
from the oracle's pair, density and embedding functions by lattice sums over a perfect FCC
crystal: minimising the energy per atom over the lattice constant, and central second
differences of the energy density under small homogeneous strains (a monatomic Bravais
lattice has no internal relaxation, so these are the elastic constants).
Parity unpinned: the short-range repulsions S_n act only below 2.24 A and the embedding
terms q2..q4 only below unit density; no printed value reaches them.
"""

import numpy as np
import pytest
import torch
from scipy.optimize import minimize_scalar

import synth
from oracle import eam as oeam

EV_PER_A3_IN_GPA = 160.21766208

# Appendix D, Table III (EAM original, EAM fit)
TABLE3 = {
    "original": dict(a0=3.61492887282983, e_coh=-3.55786833489833, c11=171.453901566772, c12=124.157217644317,
                     c44=76.2101973267168),
    "fit": dict(a0=3.63045256622797, e_coh=-3.69569662929878, c11=171.288636692165, c12=120.145974948912,
                c44=80.5610917066166),
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
def test_eam2_bulk_properties_match_table3(name, params):
    got = _properties(params)
    want = TABLE3[name]
    assert abs(got["a0"] - want["a0"]) < 2e-5, (got["a0"], want["a0"])
    assert abs(got["e_coh"] - want["e_coh"]) < 1e-4, (got["e_coh"], want["e_coh"])
    for c in ("c11", "c12", "c44"):
        assert abs(got[c] - want[c]) < 0.1, (c, got[c], want[c])


def test_eam2_density_term_underflows_and_taper_vanishes():
    # Appendix D's second density term exp(-beta2 (r - r04)) with beta2 = 535.661 /A and
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

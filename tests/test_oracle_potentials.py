"""Pins of the oracle's EAM, ACE and hybrid energies and forces (CPU only)."""

import math

import numpy as np
import pytest
import torch
from scipy.special import sph_harm_y

import synth
from synth import configs
from oracle import ace, eam, geometry, hybrid

A = synth.A_CU


# ------------------------------------------------------------------------- helpers
def _perfect(cells=4, a=A):
    pos = synth.fcc_positions(cells, cells, cells, a)
    return synth.System(pos, np.zeros(3), np.full(3, cells * a), (1, 1, 1))


def _total(system, eam_p, ace_p, w, sites_near=None):
    """sum_i (1-w_i) E_i^EAM + w_i E_i^ACE, optionally only over ``sites_near``."""
    ev = hybrid.evaluate(system, eam_p, ace_p, w, want_forces=False)
    e = ev["e_site"]
    if sites_near is not None:
        return math.fsum(e[sites_near].tolist())
    return math.fsum(e.tolist())


def _near(system, i, r):
    d = system.pos - system.pos[:, [i]]
    for k in range(3):
        if system.periodic[k]:
            d[k] -= system.box[k] * np.round(d[k] / system.box[k])
    return np.nonzero((d * d).sum(0) < r * r)[0]


def _fd_check(system, eam_p, ace_p, w, atoms, h=1e-5, tol=1e-7):
    ev = hybrid.evaluate(system, eam_p, ace_p, w)
    for i in atoms:
        near = _near(system, i, 5.6)  # sites whose energy depends on atom i
        for c in range(3):
            sp = system.copy()
            sp.pos[c, i] += h
            sm = system.copy()
            sm.pos[c, i] -= h
            fd = -(_total(sp, eam_p, ace_p, w, near) - _total(sm, eam_p, ace_p, w, near)) / (2 * h)
            assert ev["f"][c, i] == pytest.approx(fd, abs=tol), (i, c)


def _ace(n_max=8, l_max=3, seed=11, anchored=False):
    return synth.ace_random(n_max, l_max, ace.num_basis(n_max, l_max), seed, anchored=anchored)


# -------------------------------------------------------------------------- EAM
def test_eam_perfect_lattice_closed_form():
    p = synth.eam_cu_like()
    s = _perfect(4)
    ev = hybrid.evaluate(s, p, None, np.zeros(s.n))
    # shells inside r_c = 5 A: 12 at a/sqrt2, 6 at a, 24 at a sqrt(3/2)
    shells = [(12, A / math.sqrt(2)), (6, A), (24, A * math.sqrt(1.5))]

    def psi(x):
        return x ** 4 / (1 + x ** 4) if x < 0 else 0.0
    rho = sum(k * math.exp(-p.beta * (r - p.r0)) * psi((r - p.rc) / p.h) for k, r in shells)
    pair = sum(k * p.A * math.exp(-p.alpha * (r - p.r0)) * psi((r - p.rc) / p.h) for k, r in shells)
    e = -math.sqrt(rho) + 0.5 * pair
    assert np.allclose(ev["e_eam"], e, rtol=0, atol=1e-12)
    assert np.max(np.abs(ev["f"])) < 1e-12


@pytest.mark.parametrize("maker", [synth.eam_cu_like, synth.eam_anchor, synth.eam_label_anchor])
def test_eam_stress_free_at_a(maker):
    # the amplitudes were chosen for zero pressure at a = 3.615 A: dE/da = 0
    p = maker()
    def e_of(a):
        q = synth.EamParams(p.A, p.alpha, p.beta, p.r0, p.rc, p.h)  # r0 fixed
        s = _perfect(4, a)
        return hybrid.evaluate(s, q, None, np.zeros(s.n), want_forces=False)["e_eam"].mean()
    h = 1e-5
    dE = (e_of(A + h) - e_of(A - h)) / (2 * h)
    assert abs(dE) < 1e-8
    assert e_of(A) < e_of(A * 1.01) and e_of(A) < e_of(A * 0.99)


def test_eam_forces_fd_and_momentum():
    s = configs.cfg0()
    p = synth.eam_cu_like()
    w = np.random.default_rng(5).uniform(0, 1, s.n)  # frozen weights
    ev = hybrid.evaluate(s, p, None, np.zeros(s.n))
    assert np.max(np.abs(ev["f"].sum(axis=1))) < 1e-11
    _fd_check(s, p, None, np.zeros(s.n), atoms=[0, 401])
    ev = hybrid.evaluate(s, p, None, w)
    assert np.max(np.abs(ev["f_eam"].sum(axis=1))) < 1e-11


# -------------------------------------------------------------------------- ACE parts
def test_real_sph_harm_matches_scipy():
    rng = np.random.default_rng(0)
    u = rng.normal(size=(50, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    Y = ace.real_sph_harm(torch.as_tensor(u), 4).numpy()
    theta = np.arccos(u[:, 2])
    phi = np.arctan2(u[:, 1], u[:, 0])
    for l in range(5):
        for m in range(-l, l + 1):
            Yc = sph_harm_y(l, abs(m), theta, phi)  # complex, Condon-Shortley phase
            if m > 0:
                ref = math.sqrt(2) * (-1) ** m * Yc.real
            elif m < 0:
                ref = math.sqrt(2) * (-1) ** m * Yc.imag
            else:
                ref = Yc.real
            assert np.allclose(Y[:, l * l + l + m], ref, atol=1e-13), (l, m)


def test_chebyshev_radial_matches_numpy():
    r = torch.linspace(0.5, 5.2, 40, dtype=torch.float64)
    g = ace.chebyshev_radial(r, 10, 5.0, 0.5).numpy()
    x = 2 * r.numpy() / 5.0 - 1
    t = np.where(r.numpy() < 5.0, ((r.numpy() - 5) / .5) ** 4 / (1 + ((r.numpy() - 5) / .5) ** 4), 0)
    for k in range(10):
        assert np.allclose(g[:, k], np.polynomial.chebyshev.chebval(x, [0] * k + [1]) * t, atol=1e-13)


def _w3j000(l1, l2, l3):
    g2 = l1 + l2 + l3
    if g2 % 2:
        return 0.0
    g = g2 // 2
    f = math.factorial
    v = math.sqrt(f(g2 - 2 * l1) * f(g2 - 2 * l2) * f(g2 - 2 * l3) / f(g2 + 1))
    return (-1) ** g * v * f(g) / (f(g - l1) * f(g - l2) * f(g - l3))


def test_gaunt_closed_forms():
    G = ace.gaunt(4)
    for (l1, l2, l3), g in G.items():
        # m = 0 entries: Racah's closed form through the 3j symbol (l1 l2 l3; 0 0 0)
        ref = math.sqrt((2 * l1 + 1) * (2 * l2 + 1) * (2 * l3 + 1) / (4 * math.pi)) \
            * _w3j000(l1, l2, l3) ** 2
        assert g[l1, l2, l3] == pytest.approx(ref, abs=1e-13)
        # symmetry under exchange of the first two slots
        assert np.allclose(g, np.transpose(G[(l2, l1, l3)], (1, 0, 2)), atol=1e-14)
    for l in range(5):  # Y_00 = 1/sqrt(4 pi): orthonormality
        assert np.allclose(G[(l, 0, l)][:, 0, :], np.eye(2 * l + 1) / math.sqrt(4 * math.pi),
                           atol=1e-14)


def test_basis_sizes():
    assert ace.num_basis(8, 3) == 2344
    assert ace.num_basis(10, 4) == 7895


def _single_env(nbrs):
    pos = np.concatenate([np.zeros((3, 1)), np.asarray(nbrs, float).T], axis=1)
    return synth.System(pos, np.full(3, -50.0), np.full(3, 50.0), (0, 0, 0))


@pytest.mark.parametrize("nl", [(8, 3), (10, 4)])
def test_b2_addition_theorem(nl):
    n_max, l_max = nl
    rng = np.random.default_rng(3)
    nb = rng.normal(size=(7, 3))
    nb *= (rng.uniform(2.2, 4.8, 7) / np.linalg.norm(nb, axis=1))[:, None]
    s = _single_env(nb)
    prm = _ace(n_max, l_max)
    i, j = geometry.pairs_within(s.pos, s.lo, s.hi, s.periodic, prm.rc)
    A_ = ace.atomic_base(torch.as_tensor(s.pos), s.box, s.periodic, i, j, prm, [0])
    B = ace.product_basis(A_, n_max, l_max)[0].numpy()
    r = np.linalg.norm(nb, axis=1)
    u = nb / r[:, None]
    g = ace.chebyshev_radial(torch.as_tensor(r), n_max, 5.0, 0.5).numpy()
    col = n_max
    for n1 in range(n_max):
        for n2 in range(n1, n_max):
            for l in range(l_max + 1):
                R1 = g @ prm.W[l, n1]
                R2 = g @ prm.W[l, n2]
                Pl = np.polynomial.legendre.legval(u @ u.T, [0] * l + [1])
                ref = (R1[:, None] * R2[None, :] * Pl).sum() * (2 * l + 1) / (4 * np.pi) / 36.0
                assert B[col] == pytest.approx(ref, rel=1e-10, abs=1e-15)
                col += 1


@pytest.mark.parametrize("nl", [(8, 3), (10, 4)])
def test_b3_single_neighbour_closed_form(nl):
    """One neighbour in a generic direction: every real Gaunt entry, m != 0 included,
    enters sum_m G Y Y Y, which the closed form fixes through (l1 l2 l3; 0 0 0)^2."""
    n_max, l_max = nl
    v = np.array([[1.3, -2.0, 1.7]])
    s = _single_env(v)
    prm = _ace(n_max, l_max)
    i, j = geometry.pairs_within(s.pos, s.lo, s.hi, s.periodic, prm.rc)
    A_ = ace.atomic_base(torch.as_tensor(s.pos), s.box, s.periodic, i, j, prm, [0])
    B = ace.product_basis(A_, n_max, l_max)[0].numpy()
    r = np.linalg.norm(v)
    g = ace.chebyshev_radial(torch.tensor([r]), n_max, 5.0, 0.5).numpy()[0]
    spec = ace.basis_spec(n_max, l_max)
    seen = set()
    for col, sp in enumerate(spec):
        if sp[0] != "3":
            continue
        (n1, l1), (n2, l2), (n3, l3) = [divmod(p, l_max + 1) for p in sp[1:]]
        seen.add(tuple(sorted((l1, l2, l3))))
        R = [g @ prm.W[l, n] for n, l in ((n1, l1), (n2, l2), (n3, l3))]
        ref = R[0] * R[1] * R[2] / 6.0 ** 3 * (2 * l1 + 1) * (2 * l2 + 1) * (2 * l3 + 1) \
            / (4 * np.pi) ** 2 * _w3j000(l1, l2, l3) ** 2
        assert B[col] == pytest.approx(ref, rel=1e-9, abs=1e-16), sp
    if l_max == 4:  # every degree triple with an l = 4 block is reached
        assert {(0, 4, 4), (1, 3, 4), (2, 2, 4), (2, 4, 4), (3, 3, 4), (4, 4, 4)} <= seen


def test_gaunt_l4_entries_from_a_rotated_single_neighbour():
    """The single-neighbour sum of a (l1, l2, 4) block over random directions: a wrong m != 0
    entry of the l = 4 Gaunt tables makes sum_m G Y Y Y depend on the direction."""
    G = ace.gaunt(4)
    rng = np.random.default_rng(12)
    dirs = rng.normal(size=(6, 3))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    for (l1, l2, l3), g in G.items():
        if 4 not in (l1, l2, l3):
            continue
        ref = (2 * l1 + 1) * (2 * l2 + 1) * (2 * l3 + 1) / (4 * np.pi) ** 2 * _w3j000(l1, l2, l3) ** 2
        for u in dirs:
            Y = ace.real_sph_harm(torch.as_tensor(u[None, :]), 4).numpy()[0]
            ys = [Y[l * l:(l + 1) ** 2] for l in (l1, l2, l3)]
            val = np.einsum("abc,a,b,c->", g, ys[0], ys[1], ys[2])
            assert val == pytest.approx(ref, rel=1e-12, abs=1e-14), (l1, l2, l3)


def test_perfect_fcc_only_cubic_invariants_survive():
    s = _perfect(3)
    prm = _ace(8, 3)
    i, j = geometry.pairs_within(s.pos, s.lo, s.hi, s.periodic, prm.rc)
    A_ = ace.atomic_base(torch.as_tensor(s.pos), s.box, s.periodic, i, j, prm, [0, 5])
    for l in (1, 2, 3):  # inversion kills odd l; cubic symmetry has no l = 2 invariant
        assert np.max(np.abs(A_[l].numpy())) < 1e-14
    assert np.max(np.abs(A_[0].numpy())) > 1e-3


# ---------------------------------------------------------------- ACE energy, forces
def test_ace_forces_fd():
    s = configs.cfg0()
    prm = _ace(8, 3)
    w = np.ones(s.n)
    _fd_check(s, synth.eam_cu_like(), prm, w, atoms=[3, 500], tol=1e-7)


def test_hybrid_forces_fd_random_weights():
    s = configs.cfg0()
    prm = _ace(8, 3, anchored=True)
    rng = np.random.default_rng(9)
    w = np.where(rng.uniform(size=s.n) < 0.5, 0.0, rng.uniform(size=s.n))
    _fd_check(s, synth.eam_cu_like(), prm, w, atoms=[10, 222], tol=1e-7)


def _cluster(seed=4):
    s = configs.cfg0(seed=seed)
    keep = _near(s, 100, 9.0)
    pos = s.pos[:, keep].copy()
    pos -= pos.mean(axis=1, keepdims=True)
    return synth.System(pos, np.full(3, -60.0), np.full(3, 60.0), (0, 0, 0))


@pytest.mark.parametrize("nl", [(8, 3), (10, 4)])
def test_invariance_rotation_translation_permutation(nl):
    s = _cluster()
    prm = _ace(*nl)
    eam_p = synth.eam_cu_like()
    w = np.random.default_rng(1).uniform(0, 1, s.n)
    ev = hybrid.evaluate(s, eam_p, prm, w)
    q, _ = np.linalg.qr(np.random.default_rng(2).normal(size=(3, 3)))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    r = s.copy()
    r.pos = q @ s.pos + np.array([[1.5], [-2.0], [0.7]])
    er = hybrid.evaluate(r, eam_p, prm, w)
    assert er["e_pot"] == pytest.approx(ev["e_pot"], rel=1e-12)
    assert np.allclose(er["f"], q @ ev["f"], atol=1e-11)
    perm = np.random.default_rng(3).permutation(s.n)
    p = s.copy()
    p.pos = s.pos[:, perm]
    ep = hybrid.evaluate(p, eam_p, prm, w[perm])
    assert ep["e_pot"] == pytest.approx(ev["e_pot"], rel=1e-12)
    assert np.allclose(ep["f"], ev["f"][:, perm], atol=1e-11)
    assert np.max(np.abs(ev["f"].sum(axis=1))) < 1e-11


def test_weight_limits_and_uniform_mixing():
    s = configs.cfg0()
    eam_p = synth.eam_cu_like()
    prm = _ace(8, 3)
    e0 = hybrid.evaluate(s, eam_p, prm, np.zeros(s.n))
    pure = hybrid.evaluate(s, eam_p, None, np.zeros(s.n))
    assert np.array_equal(e0["f"], pure["f"]) and e0["e_pot"] == pure["e_pot"]
    e1 = hybrid.evaluate(s, eam_p, prm, np.ones(s.n))
    assert np.array_equal(e1["e_site"], e1["e_ace"])
    assert np.allclose(e1["f"], e1["f_ace"], atol=0)
    c = 0.3
    ec = hybrid.evaluate(s, eam_p, prm, np.full(s.n, c))
    assert np.allclose(ec["f"], (1 - c) * pure["f"] + c * e1["f"], atol=1e-13)
    # non-uniform weights: the force is not the per-atom mix of the two force fields
    w = np.random.default_rng(0).uniform(size=s.n)
    ew = hybrid.evaluate(s, eam_p, prm, w)
    mixed = (1 - w) * pure["f"] + w * e1["f"]
    assert np.max(np.abs(ew["f"] - mixed)) > 1e-3


def test_potential_energy_jump_identity():
    # Appendix C, eq. Delta_V_i in the precise-weight form: at fixed positions a weight
    # change w -> w' changes E_pot by sum_i (w'_i - w_i)(E_i^ACE - E_i^EAM)
    s = configs.cfg0()
    eam_p = synth.eam_cu_like()
    prm = _ace(8, 3, anchored=True)
    rng = np.random.default_rng(4)
    w = np.where(rng.uniform(size=s.n) < 0.6, 0.0, rng.uniform(size=s.n))
    w2 = np.where(rng.uniform(size=s.n) < 0.6, 0.0, rng.uniform(size=s.n))
    full = hybrid.evaluate(s, eam_p, prm, np.ones(s.n), want_forces=False)
    a = hybrid.evaluate(s, eam_p, prm, w, want_forces=False)
    b = hybrid.evaluate(s, eam_p, prm, w2, want_forces=False)
    dv = math.fsum(((w2 - w) * (full["e_ace"] - full["e_eam"])).tolist())
    assert b["e_pot"] - a["e_pot"] == pytest.approx(dv, abs=1e-10)


def test_coefficient_gradients_fd():
    s = configs.cfg0()
    prm = _ace(8, 3)
    i, j = geometry.pairs_within(s.pos, s.lo, s.hi, s.periodic, prm.rc)
    w = np.random.default_rng(2).uniform(size=s.n)
    sites = np.arange(0, s.n, 7)
    c1 = torch.tensor(prm.c1, requires_grad=True)
    c2 = torch.tensor(prm.c2, requires_grad=True)
    e = ace.site_energies(torch.as_tensor(s.pos), s.box, s.periodic, i, j, prm, s.n, sites, c1, c2)
    tot = (torch.as_tensor(w) * e).sum()
    g1, g2 = torch.autograd.grad(tot, (c1, c2))
    h = 1e-6
    for k in (0, 50, 900, 2300):
        for cvec, g in ((prm.c1, g1), (prm.c2, g2)):
            orig = cvec[k]
            vals = []
            for sgn in (1, -1):
                cvec[k] = orig + sgn * h
                ee = ace.site_energies(torch.as_tensor(s.pos), s.box, s.periodic, i, j, prm, s.n, sites)
                vals.append(float((torch.as_tensor(w) * ee).sum()))
            cvec[k] = orig
            assert float(g[k]) == pytest.approx((vals[0] - vals[1]) / (2 * h), rel=1e-6, abs=1e-9)


def test_anchor_with_zero_coefficients_is_eam():
    s = configs.cfg0()
    prm = synth.AceParams(8, 3, np.zeros((4, 8, 8)), np.zeros(2344), np.zeros(2344),
                          anchor=synth.eam_anchor())
    e = hybrid.evaluate(s, synth.eam_anchor(), prm, np.ones(s.n))
    ref = hybrid.evaluate(s, synth.eam_anchor(), None, np.zeros(s.n))
    assert np.allclose(e["e_ace"], ref["e_eam"], atol=1e-14)
    assert np.allclose(e["f"], ref["f"], atol=1e-13)

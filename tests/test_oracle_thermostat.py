"""Pins of the oracle's local thermostat (Sec. II C 2, Appendix C; CPU only).

* The counter-based generator is Philox4x64-10 as numpy's Philox bit generator computes it
  (numpy advances its counter by one before each block of four words).
* One group rescale keeps the group's momentum, multiplies its relative kinetic energy by
  beta^2 and changes the kinetic energy by exactly dE (eqs. p_resc_omega, beta_omega_i);
  a negative radicand leaves the momenta alone and is reported.
* dV and dT equal the differences of site energies and of kinetic energies computed the
  long way (blend site energies; velocities after the second half kick with each force).
* Whole step: a step whose weights change, finished with the updated weights and the
  thermostat, has the total energy of the same step with constant weights (the paper's
  claim of energy conservation within numerical precision), and without the thermostat it
  does not.  Total momentum is unchanged by the correction.
* Atoms of one colour in different cells of the colouring grid have disjoint groups.
* Over 12 steps with weights recomputed every step, the total energy with the thermostat
  equals the constant-weight reference at every step and follows the integration error;
  without it, it drifts ten times further.
"""

import math

import numpy as np
import pytest

import synth
from synth import configs
from oracle import ace as oace
from oracle import geometry, hybrid, precision, thermostat, verlet

CONV = 9648.5332
M = synth.MASS_CU


def test_philox_matches_numpy_generator():
    # the Random123 known answer for a zero counter and key
    assert thermostat.philox4x64_10((0, 0, 0, 0), (0, 0)) == (
        0x16554D9ECA36314C, 0xDB20FE9D672D0FDC, 0xD7E772CEE186176B, 0x7E68B68AEC7BA23B)
    rng = np.random.default_rng(3)
    for _ in range(20):
        key = [int(v) for v in rng.integers(0, 2 ** 63, size=2)]
        ctr = [int(v) for v in rng.integers(0, 2 ** 63, size=4)]
        g = np.random.Philox(key=key, counter=ctr)
        got = [int(v) for v in g.random_raw(4)]
        ctr1 = [ctr[0] + 1] + ctr[1:]
        assert list(thermostat.philox4x64_10(ctr1, key)) == got


def test_rescale_group_momentum_and_energy():
    rng = np.random.default_rng(4)
    v = rng.normal(0.0, 3.0, size=(3, 50))
    members = np.array(sorted(rng.choice(50, size=17, replace=False)))
    for dE in (0.013, -0.004, 0.0):
        w = v.copy()
        p0 = w[:, members].sum(axis=1)
        ke0 = 0.5 * M / CONV * float((w[:, members] ** 2).sum())
        rel0 = w[:, members] - w[:, members].mean(axis=1, keepdims=True)
        krel0 = 0.5 * M / CONV * float((rel0 ** 2).sum())
        beta = thermostat.rescale_group(w, members, dE, M)
        assert beta is not None
        assert np.allclose(w[:, members].sum(axis=1), p0, rtol=0, atol=1e-12)
        ke1 = 0.5 * M / CONV * float((w[:, members] ** 2).sum())
        assert ke1 - ke0 == pytest.approx(dE, abs=1e-13)
        rel1 = w[:, members] - w[:, members].mean(axis=1, keepdims=True)
        assert 0.5 * M / CONV * float((rel1 ** 2).sum()) == pytest.approx(beta * beta * krel0, rel=1e-13)
        others = np.setdiff1d(np.arange(50), members)
        assert np.array_equal(w[:, others], v[:, others])
        if dE == 0.0:
            assert beta == 1.0


def test_negative_radicand_is_reported_and_skipped():
    rng = np.random.default_rng(5)
    v = rng.normal(0.0, 1.0, size=(3, 12))
    members = np.arange(12)
    rel = v - v.mean(axis=1, keepdims=True)
    krel = 0.5 * M / CONV * float((rel ** 2).sum())
    w = v.copy()
    assert thermostat.rescale_group(w, members, -1.5 * krel, M) is None
    assert np.array_equal(w, v)
    # exactly -K_rel: beta = 0, every relative momentum removed
    w = v.copy()
    assert thermostat.rescale_group(w, members, -krel * (1.0 - 1e-15), M) == pytest.approx(0.0, abs=1e-6)
    # no relative momentum: nothing to rescale
    same = np.ones((3, 12))
    assert thermostat.rescale_group(same.copy(), members, 0.01, M) is None


def _system(cells=8, seed=11):
    s = configs.bulk(cells, seed, temperature=600.0, vacancies=3, velocities=True)
    return s


def test_group_selection():
    s = _system()
    mobile = np.ones(s.n, bool)
    mobile[::7] = False
    r_om, cap = 6.0, 40
    for i in (0, 101, 1500):
        g = thermostat.group(s.pos, s.lo, s.hi, s.periodic, i, mobile, r_om, cap, seed=9, step=3)
        dx, dy, dz = geometry.displacements(s.pos, s.box, s.periodic, np.full(s.n, i), np.arange(s.n))
        r2 = geometry.sq_dist(dx, dy, dz)
        cand = np.nonzero(mobile & (r2 < r_om ** 2) & (np.arange(s.n) != i))[0]
        assert cand.size > cap  # the random selection is exercised
        assert g[0] == i and g.size == cap
        sel = g[1:]
        assert np.all(np.isin(sel, cand)) and np.all(np.diff(sel) > 0)
        pri = {int(j): thermostat.priority(9, 3, i, int(j)) for j in cand}
        worst_taken = max(pri[int(j)] for j in sel)
        assert all(pri[int(j)] > worst_taken for j in np.setdiff1d(cand, sel))
        # another step draws another subset; a radius with few candidates takes them all
        g2 = thermostat.group(s.pos, s.lo, s.hi, s.periodic, i, mobile, r_om, cap, seed=9, step=4)
        assert not np.array_equal(g, g2)
        g3 = thermostat.group(s.pos, s.lo, s.hi, s.periodic, i, mobile, 3.0, cap, seed=9, step=3)
        small = np.nonzero(mobile & (r2 < 9.0) & (np.arange(s.n) != i))[0]
        assert np.array_equal(g3[1:], small)


def test_colour_classes_have_disjoint_groups():
    rng = np.random.default_rng(6)
    L = np.array([61.0, 49.0, 75.0])
    per = (1, 1, 0)
    pos = rng.uniform(0.0, 1.0, size=(3, 3000)) * L[:, None]
    r_om = 6.0
    nc = thermostat.colour_grid(np.zeros(3), L, per, r_om)
    assert nc == [4, 4, 6]  # 61/12 = 5 (odd, periodic) -> 4; 49/12 -> 4; 75/12 -> 6
    colour, cell = thermostat.colours(pos, np.zeros(3), L, per, r_om)
    for c in range(8):
        idx = np.nonzero(colour == c)[0]
        a, b = np.triu_indices(idx.size, k=1)
        a, b = idx[a], idx[b]
        other = cell[a] != cell[b]
        dx, dy, dz = geometry.displacements(pos, L, per, a[other], b[other])
        assert np.all(np.sqrt(geometry.sq_dist(dx, dy, dz)) >= 2.0 * r_om)


def _evaluate(s, x, w, eam_p, ace_p):
    t = s.copy()
    t.pos = x
    return hybrid.evaluate(t, eam_p, ace_p, w)


def _one_step_setup():
    s = _system(cells=6, seed=12)
    eam_p = synth.eam_cu_like()
    ace_p = synth.ace_random(8, 3, oace.num_basis(8, 3), seed=5, anchored=True)
    csr = geometry.neighbor_csr(s.pos, s.lo, s.hi, s.periodic, 5.5)
    w_c = precision.compute_precision(s, synth.precision_cfg0(), csr)["w"]
    rng = np.random.default_rng(13)
    # the update: some weights change by a minimum step, some switch on or off
    w_d = w_c.copy()
    pick = rng.choice(s.n, size=60, replace=False)
    w_d[pick[:30]] = np.clip(w_d[pick[:30]] + rng.choice([-0.1, 0.1], size=30), 0.0, 1.0)
    w_d[pick[30:45]] = 0.0
    w_d[pick[45:]] = 1.0
    dt = 1e-3
    c = 0.5 * dt * CONV / M
    ev0 = _evaluate(s, s.pos, w_c, eam_p, ace_p)
    v_half = s.vel + c * ev0["f"]
    x1 = verlet.wrap_positions(s.pos + dt * v_half, s.lo, s.hi, s.periodic)
    ec = _evaluate(s, x1, w_c, eam_p, ace_p)
    ed = _evaluate(s, x1, w_d, eam_p, ace_p)
    return s, eam_p, ace_p, w_c, w_d, dt, c, v_half, x1, ec, ed


def _kin(v):
    return 0.5 * M / CONV * math.fsum((v * v).ravel().tolist())


def test_energy_errors_equal_the_long_way():
    s, eam_p, ace_p, w_c, w_d, dt, c, v_half, x1, ec, ed = _one_step_setup()
    e_prec = np.where(w_d > 0.0, ed["e_ace"], ec["e_ace"])
    mobile = np.ones(s.n, bool)
    dE, dV, dT = thermostat.energy_errors(w_c, w_d, ed["e_eam"], e_prec, ec["f"], ed["f"], v_half, dt, M, mobile)
    # dV: site energies of the blend with each weight set
    assert np.allclose(dV, ec["e_site"] - ed["e_site"], rtol=0, atol=1e-12)
    assert np.count_nonzero(dV) == np.count_nonzero(w_c != w_d)
    # dT: kinetic energies after the second half kick with each force
    vc = v_half + c * ec["f"]
    vd = v_half + c * ed["f"]
    tk = 0.5 * M / CONV * ((vc * vc).sum(axis=0) - (vd * vd).sum(axis=0))
    assert np.allclose(dT, tk, rtol=0, atol=1e-13)
    assert np.count_nonzero(dT) > np.count_nonzero(dV)  # neighbours of changed sites too
    assert np.array_equal(dE, dV + dT)


@pytest.mark.parametrize("r_omega,cap", [(6.0, 40), (9.0, 800)])
def test_corrected_step_has_the_reference_energy(r_omega, cap):
    s, eam_p, ace_p, w_c, w_d, dt, c, v_half, x1, ec, ed = _one_step_setup()
    mobile = np.ones(s.n, bool)
    vc = v_half + c * ec["f"]
    vd = v_half + c * ed["f"]
    e_ref = ec["e_pot"] + _kin(vc)
    e_dyn = ed["e_pot"] + _kin(vd)
    e_prec = np.where(w_d > 0.0, ed["e_ace"], ec["e_ace"])
    dE, _, _ = thermostat.energy_errors(w_c, w_d, ed["e_eam"], e_prec, ec["f"], ed["f"], v_half, dt, M, mobile)
    p_before = vd.sum(axis=1)
    v = vd.copy()
    rec = thermostat.correct(x1, s.lo, s.hi, s.periodic, v, dE, mobile, M, r_omega, cap, seed=21, step=1)
    assert not rec["failed"]
    assert rec["order"].size == np.count_nonzero(dE)
    assert abs(e_dyn - e_ref) > 1e-3  # the update's energy error is real
    e_fix = ed["e_pot"] + _kin(v)
    print(f"dynamic - reference {e_dyn - e_ref:.3e} eV, corrected - reference {e_fix - e_ref:.3e} eV")
    assert abs(e_fix - e_ref) < 1e-9
    assert np.allclose(v.sum(axis=1), p_before, rtol=0, atol=1e-9)


def test_dynamic_weights_conserve_energy_with_the_thermostat():
    """Weights recomputed every step (instantaneous, linear switch 0.2-0.5 A^2 on a thermal
    crystal: thermal CSP noise moves many partial weights every step).  At every step the
    corrected total energy equals that of the same step with the previous weights held
    constant, so the total energy follows the integrator's own error; without the
    thermostat each update adds its energy error and the total drifts."""
    s = configs.bulk(5, 17, temperature=900.0, vacancies=2, velocities=True)
    eam_p = synth.eam_cu_like()
    ace_p = synth.ace_random(8, 3, oace.num_basis(8, 3), seed=5, anchored=True)
    prec = synth.precision_cfg0()
    dt, steps = 5e-4, 12
    runs = {}
    for on in (False, True):
        th = dict(r_omega=6.0, omega_max=60, seed=3) if on else None
        runs[on] = verlet.run(s, eam_p, ace_p, prec, dt, steps, precision_every=1, thermostat=th)
    ref = verlet.run(s, eam_p, ace_p, prec, dt, steps, precision_every=0)
    e = {on: r["e_pot"] + r["e_kin"] for on, r in runs.items()}
    for k, rec in enumerate(runs[True]["thermostat"], start=1):
        assert rec is not None and not rec["failed"]
        assert abs(e[True][k] - (rec["e_pot_ref"] + rec["e_kin_ref"])) < 1e-9 * s.n
    drift = {on: np.abs(v - v[0]).max() / s.n for on, v in e.items()}
    e_ref = ref["e_pot"] + ref["e_kin"]
    drift_ref = np.abs(e_ref - e_ref[0]).max() / s.n
    print(f"max |E - E0| per atom: constant weights {drift_ref:.2e}, dynamic {drift[False]:.2e}, "
          f"dynamic + thermostat {drift[True]:.2e} eV")
    assert drift[True] < 3.0 * drift_ref + 1e-8
    assert drift[False] > 10.0 * drift[True]

"""The local thermostat on the GPU (Sec. II C 2, Appendix C) against the oracle.

* Energy errors from the oracle's forces and energies: within 1e-12 eV, the same atoms
  exactly zero.
* The correction on seeded synthetic velocities and energy errors: the same atoms
  corrected in the same groups (the draw is integer work), velocities within 1e-12 of
  their scale; several colour grids (one cell, eight cells, 64 cells), frozen atoms and a
  free surface; a negative radicand reported and skipped on both sides; too many
  candidates refused.
* The integrator with the thermostat against the oracle's trajectory (instantaneous
  weights every step, and time-averaged weights over the past window), float64 ACE.
* A longer run: with the thermostat the total energy follows the constant-weight
  integration error, without it it drifts; total momentum is kept.
"""

import numpy as np
import pytest
import torch

import synth
from synth import configs
from oracle import ace as oace
from oracle import thermostat, verlet

from test_oracle_thermostat import _one_step_setup

pytestmark = pytest.mark.gpu
M = synth.MASS_CU


@pytest.fixture(scope="module")
def ops_ctx():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2411_03002_amd import ops
    return ops, ops.Context(0)


def _case(msg):
    print(f"\n[case] {msg}", flush=True)


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def test_energy_errors_parity(ops_ctx):
    ops, ctx = ops_ctx
    _case("thermostat energy errors")
    s, eam_p, ace_p, w_c, w_d, dt, c, v_half, x1, ec, ed = _one_step_setup()
    e_prec = np.where(w_d > 0.0, ed["e_ace"], ec["e_ace"])
    mobile = np.ones(s.n, bool)
    ref, _, _ = thermostat.energy_errors(w_c, w_d, ed["e_eam"], e_prec, ec["f"], ed["f"], v_half, dt, M, mobile)
    got = ops.thermostat_energy_errors(ctx, _dev(w_c), _dev(w_d), _dev(ed["e_eam"]), _dev(e_prec), _dev(ed["f"]),
                                       _dev(ec["f"] - ed["f"]), _dev(v_half), dt, M).cpu().numpy()
    assert np.array_equal(got == 0.0, ref == 0.0)
    assert np.abs(got - ref).max() < 1e-12, np.abs(got - ref).max()
    # frozen atoms carry no error
    fz = np.zeros(s.n, np.uint8)
    fz[::5] = 1
    got = ops.thermostat_energy_errors(ctx, _dev(w_c), _dev(w_d), _dev(ed["e_eam"]), _dev(e_prec), _dev(ed["f"]),
                                       _dev(ec["f"] - ed["f"]), _dev(v_half), dt, M,
                                       frozen=torch.as_tensor(fz, device="cuda")).cpu().numpy()
    assert np.all(got[fz == 1] == 0.0)
    assert np.abs(got[fz == 0] - ref[fz == 0]).max() < 1e-12


def _bulk(cells, seed):
    return configs.bulk(cells, seed, temperature=600.0, vacancies=3, velocities=True)


def _slab():
    return configs.slab100(8, 8, 6, seed=41, temperature=600.0, sigma=0.1)


CASES = {
    # system, r_omega, omega_max, fraction corrected
    "bulk8_draw_8cells": (lambda: _bulk(8, 51), 6.0, 40, 0.3),
    "bulk8_all_one_cell": (lambda: _bulk(8, 52), 9.0, 800, 0.1),
    "bulk12_draw_64cells": (lambda: _bulk(12, 53), 5.0, 50, 0.2),
    "slab_frozen_free_z": (_slab, 6.0, 30, 0.3),
}


def _inputs(s, frac, seed):
    rng = np.random.default_rng(seed)
    dE = np.where(rng.uniform(size=s.n) < frac, rng.normal(0.0, 2e-3, size=s.n), 0.0)
    if s.vel is None:
        s.vel = synth.maxwell_velocities(s.n, 600.0, rng, None if s.frozen is None else ~s.frozen.astype(bool))
    return dE


@pytest.mark.parametrize("case", list(CASES))
def test_correction_parity(ops_ctx, case):
    ops, ctx = ops_ctx
    make, r_om, cap, frac = CASES[case]
    _case(f"thermostat correction {case}")
    s = make()
    dE = _inputs(s, frac, 7)
    mobile = np.ones(s.n, bool) if s.frozen is None else ~s.frozen.astype(bool)
    params = dict(r_omega=r_om, omega_max=cap, seed=12345)
    v_ref = s.vel.copy()
    rec = thermostat.correct(s.pos, s.lo, s.hi, s.periodic, v_ref, dE, mobile, M, r_om, cap, 12345, 9)
    atoms = ops.device_atoms(s)
    vel = _dev(s.vel)
    out = ops.thermostat_correct(ctx, atoms, vel, _dev(dE), params, 9, M)
    v = vel.cpu().numpy()
    print(f"{s.n} atoms, {out['corrected']} corrections, groups of {rec['sizes'].min()}..{rec['sizes'].max()}, "
          f"max |dv| {np.abs(v - v_ref).max():.2e}", flush=True)
    assert out["corrected"] == len(rec["order"]) - len(rec["failed"]) and out["failed"] == 0
    assert np.abs(v - v_ref).max() < 1e-12 * np.abs(v_ref).max()
    assert not np.array_equal(v_ref, s.vel)


@pytest.mark.parametrize("batch", [1, 37])
def test_correction_parity_in_batches(ops_ctx, batch):
    # groups drawn a few at a time: a colour cell's corrections span several batches, and
    # the order (colour, cell, atom) and the result stay those of the oracle
    ops, ctx = ops_ctx
    _case(f"thermostat correction in batches of {batch} groups")
    s = _bulk(12, 53)
    dE = _inputs(s, 0.2, 7)
    mobile = np.ones(s.n, bool)
    v_ref = s.vel.copy()
    rec = thermostat.correct(s.pos, s.lo, s.hi, s.periodic, v_ref, dE, mobile, M, 5.0, 50, 12345, 9)
    atoms = ops.device_atoms(s)
    vel = _dev(s.vel)
    out = ops.thermostat_correct(ctx, atoms, vel, _dev(dE), dict(r_omega=5.0, omega_max=50, seed=12345,
                                                                 group_batch=batch), 9, M)
    v = vel.cpu().numpy()
    print(f"{out['corrected']} corrections, max |dv| {np.abs(v - v_ref).max():.2e}", flush=True)
    assert out["corrected"] == len(rec["order"]) - len(rec["failed"]) and out["failed"] == 0
    assert np.abs(v - v_ref).max() < 1e-12 * np.abs(v_ref).max()


def test_negative_radicand_reported(ops_ctx):
    ops, ctx = ops_ctx
    _case("thermostat negative radicand")
    s = _bulk(8, 54)
    dE = _inputs(s, 0.05, 8)
    bad = int(np.nonzero(dE == 0.0)[0][17])
    dE[bad] = -50.0  # far beyond any group's relative kinetic energy
    mobile = np.ones(s.n, bool)
    v_ref = s.vel.copy()
    rec = thermostat.correct(s.pos, s.lo, s.hi, s.periodic, v_ref, dE, mobile, M, 6.0, 40, 3, 1)
    assert rec["failed"] == [bad]
    atoms = ops.device_atoms(s)
    vel = _dev(s.vel)
    from paper_2411_03002_amd import binding as B
    with pytest.raises(B.ApxError):
        ops.thermostat_correct(ctx, atoms, vel, _dev(dE), dict(r_omega=6.0, omega_max=40, seed=3), 1, M)
    vel = _dev(s.vel)
    out = ops.thermostat_correct(ctx, atoms, vel, _dev(dE), dict(r_omega=6.0, omega_max=40, seed=3), 1, M,
                                 allow_radicand=True)
    assert out["status"] == B.APX_ERADICAND and out["failed"] == 1
    assert out["corrected"] == len(rec["order"]) - 1
    assert np.abs(vel.cpu().numpy() - v_ref).max() < 1e-12 * np.abs(v_ref).max()


def test_candidate_overflow_refused(ops_ctx):
    ops, ctx = ops_ctx
    _case("thermostat candidate capacity")
    s = configs.bulk(14, 55, temperature=300.0, velocities=True)
    dE = np.zeros(s.n)
    dE[100] = 1e-3
    from paper_2411_03002_amd import binding as B
    with pytest.raises(B.ApxError) as e:
        ops.thermostat_correct(ctx, ops.device_atoms(s), _dev(s.vel), _dev(dE),
                               dict(r_omega=24.0, omega_max=800, seed=1), 0, M)
    assert e.value.code == B.APX_ECAPACITY


def _md_setup(s):
    eam_p = synth.eam_cu_like()
    ace_p = synth.ace_random(8, 3, oace.num_basis(8, 3), seed=5, anchored=True)
    return eam_p, ace_p, synth.precision_cfg0()


@pytest.mark.parametrize("mode", ["instantaneous", "averaged_past"])
def test_integrator_with_thermostat_matches_oracle(ops_ctx, mode):
    ops, ctx = ops_ctx
    _case(f"integrator with the thermostat, {mode}")
    s = configs.bulk(5, 17, temperature=900.0, vacancies=2, velocities=True)
    eam_p, ace_p, prec = _md_setup(s)
    th = dict(r_omega=6.0, omega_max=60, seed=3)
    dt, steps = 5e-4, 6
    if mode == "instantaneous":
        every, avg, kw = 1, None, {}
    else:
        # every step, no minimum step: the averaged weights move at every update
        every, avg = 1, dict(n_avg=3, dw_min=0.0, window="past")
        kw = dict(avg_samples=3, avg_dw_min=0.0, avg_window="past")
    ref = verlet.run(s, eam_p, ace_p, prec, dt, steps, precision_every=every, avg=avg, thermostat=th)
    atoms = ops.device_atoms(s)
    model = ops.AceModel(ctx, ace_p)
    md = ops.MD(ctx, atoms, eam_p, model, prec, dt=dt, skin=0.5, max_nb=80, precision_every=every,
                ace_precision="fp64", mode="adaptive", thermostat=th, **kw)
    pos = atoms.pos.clone()
    vel = _dev(s.vel)
    f, w = md.init(pos)
    st = md.step(pos, vel, f, w, steps)
    md.close()
    n_ref = sum(len(r["order"]) for r in ref["thermostat"] if r is not None)
    dx = np.abs(pos.cpu().numpy() - ref["x"]).max()
    dv = np.abs(vel.cpu().numpy() - ref["v"]).max()
    print(f"{st['thermo_corrected']} corrections over {st['thermo_steps']} steps (oracle {n_ref}); "
          f"max |dx| {dx:.2e} A, max |dv| {dv:.2e} A/ps", flush=True)
    assert st["thermo_corrected"] == n_ref and n_ref > 0 and st["thermo_failed"] == 0
    assert dx < 1e-10 and dv < 1e-8
    assert np.abs(w.cpu().numpy() - ref["w"]).max() < 1e-9
    e_tot = st["e_pot"] + st["e_kin"]
    assert abs(e_tot - (ref["e_pot"][-1] + ref["e_kin"][-1])) < 1e-8 * s.n


def test_energy_conserved_with_thermostat(ops_ctx):
    ops, ctx = ops_ctx
    _case("integrator energy with and without the thermostat, 4,000 atoms, 40 steps")
    s = configs.bulk(10, 18, temperature=900.0, vacancies=5, velocities=True)
    eam_p, ace_p, prec = _md_setup(s)
    model = ops.AceModel(ctx, ace_p)
    res = {}
    for name, every, th in (("constant", 0, None), ("dynamic", 1, None),
                            ("thermostat", 1, dict(r_omega=6.0, omega_max=80, seed=5))):
        atoms = ops.device_atoms(s)
        md = ops.MD(ctx, atoms, eam_p, model, prec, dt=5e-4, skin=0.5, max_nb=80, precision_every=every,
                    ace_precision="fp64", mode="adaptive", thermostat=th)
        pos = atoms.pos.clone()
        vel = _dev(s.vel)
        p0 = vel.sum(dim=1).cpu().numpy()
        f, w = md.init(pos)
        e = []
        for _ in range(40):
            st = md.step(pos, vel, f, w, 1)
            e.append(st["e_pot"] + st["e_kin"])
        md.close()
        e = np.array(e)
        res[name] = (np.abs(e - e[0]).max() / s.n, np.abs(vel.sum(dim=1).cpu().numpy() - p0).max())
    print({k: f"drift {v[0]:.2e} eV/atom, |dP| {v[1]:.1e}" for k, v in res.items()}, flush=True)
    assert res["thermostat"][0] < 3.0 * res["constant"][0] + 1e-8
    assert res["dynamic"][0] > 5.0 * res["thermostat"][0]
    # the rescale keeps each group's momentum: no more drift than the integration's rounding
    assert res["thermostat"][1] < 10.0 * res["constant"][1] + 1e-9

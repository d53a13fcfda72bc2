"""Pins of the oracle's integrator, indenter and learned-indicator pieces (CPU only)."""

import math

import numpy as np
import pytest

import synth
from synth import configs
from oracle import ace, geometry, hybrid, mlp, verlet


def test_nve_energy_conservation_fixed_weights():
    # Sec. II C 2: with the weights held constant the dynamics is conservative
    s = configs.cfg0()
    s.vel = synth.maxwell_velocities(s.n, 300.0, np.random.default_rng(1))
    prm = synth.ace_random(8, 3, ace.num_basis(8, 3), 11, anchored=True)
    w = np.zeros(s.n)
    w[:40] = np.linspace(0.1, 1.0, 40)
    errs = []
    for dt, nst in ((1e-3, 16), (5e-4, 32)):
        out = verlet.run(s, synth.eam_cu_like(), prm, None, dt=dt, n_steps=nst, w=w)
        etot = out["e_pot"] + out["e_kin"]
        errs.append(np.max(np.abs(etot - etot[0])))
        assert out["e_kin"][-1] != out["e_kin"][0]  # something moved
    assert errs[0] / s.n < 1e-5
    # velocity Verlet is second order: halving dt cuts the energy error about 4x
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_nve_eam_100fs():
    s = configs.cfg0()
    s.vel = synth.maxwell_velocities(s.n, 300.0, np.random.default_rng(2))
    out = verlet.run(s, synth.eam_cu_like(), None, None, dt=1e-3, n_steps=100, w=np.zeros(s.n))
    etot = out["e_pot"] + out["e_kin"]
    assert np.max(np.abs(etot - etot[0])) / s.n < 1e-5


def test_time_reversibility():
    s = configs.cfg0()
    s.vel = synth.maxwell_velocities(s.n, 300.0, np.random.default_rng(3))
    eam_p = synth.eam_cu_like()
    fwd = verlet.run(s, eam_p, None, None, dt=1e-3, n_steps=20, w=np.zeros(s.n))
    b = s.copy()
    b.pos = fwd["x"]
    b.vel = -fwd["v"]
    back = verlet.run(b, eam_p, None, None, dt=1e-3, n_steps=20, w=np.zeros(s.n))
    d = back["x"] - s.pos
    d -= s.box[:, None] * np.round(d / s.box[:, None])
    assert np.max(np.abs(d)) < 1e-9


def test_indenter_force_is_minus_gradient():
    rng = np.random.default_rng(0)
    pos = rng.uniform(0, 30, size=(3, 40))
    lo, hi = np.zeros(3), np.full(3, 30.0)
    c = np.array([15.0, 15.0, 20.0])
    f, _ = verlet.indenter(pos, lo, hi, (1, 1, 0), c, 10.0, 10.0)
    h = 1e-6
    for i in range(0, 40, 5):
        for k in range(3):
            p1 = pos.copy()
            p1[k, i] += h
            p2 = pos.copy()
            p2[k, i] -= h
            u1 = verlet.indenter(p1, lo, hi, (1, 1, 0), c, 10.0, 10.0)[1]
            u2 = verlet.indenter(p2, lo, hi, (1, 1, 0), c, 10.0, 10.0)[1]
            assert f[k, i] == pytest.approx(-(u1 - u2) / (2 * h), abs=1e-6)


def test_mlp_gradient_fd():
    rng = np.random.default_rng(0)
    params = mlp.init_params(3)
    params = [p + 0.1 * rng.normal(size=p.shape) for p in params]
    x = rng.normal(size=(17, 4))
    y = rng.normal(size=17)
    loss, g = mlp.loss_and_grad(params, x, y)
    h = 1e-6
    for k in range(8):
        flat = params[k].reshape(-1)
        for idx in rng.choice(flat.size, min(4, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = mlp.loss_and_grad(params, x, y)[0]
            flat[idx] = old - h
            lm = mlp.loss_and_grad(params, x, y)[0]
            flat[idx] = old
            assert g[k].reshape(-1)[idx] == pytest.approx((lp - lm) / (2 * h), rel=1e-6, abs=1e-9)


def test_adam_first_step_is_signed_lr():
    params = [np.array([1.0, -2.0, 0.5])]
    grads = [np.array([0.3, -4.0, 1e-3])]
    m, v = [np.zeros(3)], [np.zeros(3)]
    mlp.adam_step(params, grads, m, v, t=1, lr=0.01)
    # bias-corrected first step: mhat = g, vhat = g^2 -> update lr * g / (|g| + eps)
    assert np.allclose(params[0], [1.0 - 0.01, -2.0 + 0.01, 0.5 - 0.01 * 1e-3 / (1e-3 + 1e-8)],
                       atol=1e-15)


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -7, -3.14159, 65504.0],
                    dtype=np.float32)
    out = mlp.to_bf16(vals)
    # bfloat16 keeps 8 significand bits: 1 + 2^-8 is a tie -> even (1.0); 1 + 3*2^-8 -> 1 + 2^-6
    assert out[0] == 1.0 and out[1] == 1.0 and out[2] == np.float32(1.0 + 2 ** -6)
    assert out[3] == np.float32(1.0 + 2 ** -7)
    assert out[4] == np.float32(-3.140625)
    assert out[5] == np.float32(65536.0)


def test_features_on_perfect_lattice():
    s = synth.System(synth.fcc_positions(4, 4, 4), np.zeros(3), np.full(3, 4 * synth.A_CU), (1, 1, 1))
    csr = geometry.neighbor_csr(s.pos, s.lo, s.hi, s.periodic, 5.5)
    ev = hybrid.evaluate(s, synth.eam_cu_like(), None, np.zeros(s.n))
    f = mlp.features(s.pos, s.lo, s.hi, s.periodic, csr, ev["rho"], np.zeros(s.n), ev["f"])
    assert np.all(f[:, 2] == 12.0)  # nearest-neighbour shell at a/sqrt2 = 2.556 < 3.08 A
    assert np.allclose(f[:, 3], 0.0, atol=1e-12)
    assert np.allclose(f[:, 0], f[0, 0])

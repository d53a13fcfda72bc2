"""Time-averaged switching on the GPU against the oracle, bit for bit.

A sequence of calls on perturbed positions (more calls than ring slots, so the rings
wrap; a minimum step that holds some weights) compares every output of every call:
the instantaneous and averaged CSP, w0, the spread weight, its mean, the filtered
weight, the mask and the active list.  The integrator's averaged weights are compared
with the oracle at every weight update of a short run.
"""

import numpy as np
import pytest
import torch

import synth
from synth import configs
from oracle import ace as oace
from oracle import averaging, geometry

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ops_ctx():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2411_03002_amd import ops
    return ops, ops.Context(0)


def _case(msg):
    print(f"\n[case] {msg}", flush=True)


def _slab():
    return configs.slab100(4, 4, 6, seed=31, temperature=300.0, sigma=0.1, velocities=False)


def _bulk():
    return configs.bulk(8, seed=32, temperature=0.0, vacancies=2)


CASES = {
    # system, n_avg, dw_min, calls, noise (A)
    "slab_n4_dw005": (_slab, 4, 0.05, 9, 0.1),
    "bulk_vac_n3_dw01": (_bulk, 3, 0.1, 7, 0.08),
    "slab_n1_dw0": (_slab, 1, 0.0, 3, 0.1),
}


def _positions(s, base, rng, noise):
    """The base positions with fresh Gaussian displacements of the mobile atoms."""
    d = rng.normal(0.0, noise, size=base.shape)
    if s.frozen is not None:
        d[:, s.frozen.astype(bool)] = 0.0
    return synth.wrap_positions(base + d, s.lo, s.hi, s.periodic)


def _compare(out, ref):
    for key in ("csp", "csp_avg", "w0", "w_min", "w_avg", "w"):
        a = out[key].cpu().numpy()
        b = ref[key]
        same = (a == b) | (np.isinf(a) & np.isinf(b))
        assert same.all(), (key, np.nonzero(~same)[0][:5], a[~same][:5], b[~same][:5])
    assert np.array_equal(out["mask"].cpu().numpy(), ref["mask"])
    assert np.array_equal(out["active"].cpu().numpy(), ref["active"])


@pytest.mark.parametrize("case", list(CASES))
def test_time_averaged_switching_parity(ops_ctx, case):
    ops, ctx = ops_ctx
    make, n_avg, dw, calls, noise = CASES[case]
    _case(f"time-averaged switching {case}")
    s = make()
    p = synth.precision_static()
    rng = np.random.default_rng(77)
    ora = averaging.TimeAveragedSwitch(n_avg, dw)
    dev = ops.TimeAveragedSwitch(s.n, n_avg, dw)
    held = 0
    base = s.pos.copy()
    for k in range(calls):
        s.pos = _positions(s, base, rng, noise)
        atoms = ops.device_atoms(s)
        nl = ops.build_neighbors(ctx, atoms, 5.5)
        out = dev.update(ctx, atoms, nl, p)
        ref = ora.update(s, p, geometry.neighbor_csr(s.pos, s.lo, s.hi, s.periodic, 5.5))
        _compare(out, ref)
        held += int(np.sum(ref["w"] != ref["w_avg"]))
    assert dev.samples == calls
    print(f"{s.n} atoms, {calls} calls, detected {int(ref['mask'].sum())}, weights held by the minimum step {held}",
          flush=True)
    assert ref["mask"].sum() > 0
    if dw > 0:
        assert held > 0


def test_given_csp_and_extra_weight(ops_ctx):
    ops, ctx = ops_ctx
    _case("time-averaged switching, given CSP and extra detection weight")
    s = _slab()
    p = synth.precision_static()
    rng = np.random.default_rng(5)
    ora = averaging.TimeAveragedSwitch(3, 0.05)
    dev = ops.TimeAveragedSwitch(s.n, 3, 0.05)
    atoms = ops.device_atoms(s)
    nl = ops.build_neighbors(ctx, atoms, 5.5)
    csr = geometry.neighbor_csr(s.pos, s.lo, s.hi, s.periodic, 5.5)
    for k in range(5):
        c = rng.uniform(0.0, 4.0, size=s.n)
        c[rng.choice(s.n, 3, replace=False)] = np.inf
        extra = np.where(rng.uniform(size=s.n) < 0.05, rng.uniform(0.0, 1.0, size=s.n), 0.0)
        out = dev.update(ctx, atoms, nl, p, w0_extra=torch.as_tensor(extra, device="cuda"),
                         csp=torch.as_tensor(c, device="cuda"))
        ref = ora.update(s, p, csr, w0_extra=extra, csp=c)
        _compare(out, ref)


def test_argument_errors(ops_ctx):
    ops, ctx = ops_ctx
    _case("time-averaged switching, argument errors")
    from paper_2411_03002_amd import binding as B
    s = _slab()
    atoms = ops.device_atoms(s)
    nl = ops.build_neighbors(ctx, atoms, 5.5)
    p = synth.precision_static()
    for n_avg, dw in ((4, -0.1), (4, float("nan"))):
        dev = ops.TimeAveragedSwitch(s.n, n_avg, dw)
        with pytest.raises(B.ApxError):
            dev.update(ctx, atoms, nl, p)
        assert dev.samples == 0
    dev = ops.TimeAveragedSwitch(s.n, 1, 0.0)
    dev.n_avg = 0
    with pytest.raises(B.ApxError):
        dev.update(ctx, atoms, nl, p)
    dev.n_avg = 5000
    with pytest.raises(B.ApxError):
        dev.update(ctx, atoms, nl, p)


def test_integrator_time_averaged_weights(ops_ctx):
    """The integrator samples at apx_md_init and after the drift of every second step; its
    weights after each update equal the oracle's pipeline on the same positions."""
    ops, ctx = ops_ctx
    _case("integrator with time-averaged weights, slab, 12 steps")
    s = configs.slab100(4, 4, 6, seed=33, temperature=600.0, sigma=0.1)
    p = synth.precision_static()
    prm = synth.ace_random(8, 3, oace.num_basis(8, 3), seed=5, anchored=True)
    atoms = ops.device_atoms(s)
    model = ops.AceModel(ctx, prm)
    md = ops.MD(ctx, atoms, synth.eam_cu_like(), model, p, dt=1e-3, skin=0.5, max_nb=80, precision_every=2,
                ace_precision="fp64", mode="adaptive", avg_samples=3, avg_dw_min=0.05)
    pos = atoms.pos.clone()
    vel = torch.as_tensor(s.vel, device="cuda").contiguous()
    ora = averaging.TimeAveragedSwitch(3, 0.05)

    def check(w):
        s.pos = pos.cpu().numpy()
        ref = ora.update(s, p, geometry.neighbor_csr(s.pos, s.lo, s.hi, s.periodic, 5.5))
        assert np.array_equal(w.cpu().numpy(), ref["w"])
        return ref

    f, w = md.init(pos)
    check(w)
    for step in range(1, 13):
        st = md.step(pos, vel, f, w, 1)
        if step % 2 == 0:
            ref = check(w)
            assert st["n_active"] == ref["active"].size
    md.close()
    assert ref["active"].size > 0

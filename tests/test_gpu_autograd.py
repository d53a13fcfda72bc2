"""The ACE adjoint behind torch.autograd.Function on the differentiation workloads
(16x16x16-cell systems at 300/800/1200 K, with vacancies, and an FCC(111) slab):
forces against central finite differences of the library's own float64 energy
(h = 1e-5 A) and against the oracle's gradient on sampled atoms; coefficient
gradients against finite differences."""

import numpy as np
import pytest
import torch

import synth
from synth import configs
from oracle import ace as oace
from oracle import geometry

pytestmark = pytest.mark.gpu

KINDS = ["T300", "T800", "T1200", "vac", "slab111"]


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2411_03002_amd import autograd, ops
    ctx = ops.Context(0)
    prm = synth.ace_random(10, 4, oace.num_basis(10, 4), seed=33)
    model = ops.AceModel(ctx, prm)
    return ops, autograd, ctx, prm, model


def _setup(env, kind):
    ops, autograd, ctx, prm, model = env
    s = configs.cfg3(kind)
    print(f"\n[case] autograd {kind} n={s.n}", flush=True)
    w = torch.as_tensor(np.random.default_rng(1).uniform(0.2, 1.0, s.n), device="cuda")
    runner = autograd.AceRunner(ctx, model, s.lo, s.hi, s.periodic, w=w, precision="fp64", r_list=5.5)
    pos = torch.as_tensor(s.pos, device="cuda").clone().requires_grad_(True)
    c1 = torch.tensor(prm.c1, dtype=torch.float64, requires_grad=True)
    c2 = torch.tensor(prm.c2, dtype=torch.float64, requires_grad=True)
    return s, runner, pos, c1, c2, w


@pytest.mark.parametrize("kind", KINDS)
def test_forces_match_finite_differences_and_oracle(env, kind):
    ops, autograd, ctx, prm, model = env
    s, runner, pos, c1, c2, w = _setup(env, kind)
    e = autograd.ace_energy(pos, c1.detach(), c2.detach(), runner)
    (g,) = torch.autograd.grad(e, pos)
    g = g.cpu().numpy()
    rng = np.random.default_rng(7)
    atoms = rng.choice(s.n, 4, replace=False)
    h = 1e-5
    with torch.no_grad():
        for i in atoms:
            for c in range(3):
                p = pos.detach().clone()
                p[c, i] += h
                ep = autograd.ace_energy(p, c1.detach(), c2.detach(), runner).item()
                p[c, i] -= 2 * h
                em = autograd.ace_energy(p, c1.detach(), c2.detach(), runner).item()
                fd = (ep - em) / (2 * h)
                assert g[c, i] == pytest.approx(fd, abs=2e-6), (i, c)
    # oracle gradient of the same weighted energy on the sampled atoms: only sites within
    # the cutoff of atom i depend on x_i
    wn = w.cpu().numpy()
    i_all, j_all = geometry.pairs_within(s.pos, s.lo, s.hi, s.periodic, prm.rc)
    for i in atoms:
        sites = np.unique(np.concatenate([[i], j_all[i_all == i]]))
        pt = torch.tensor(s.pos, dtype=torch.float64, requires_grad=True)
        es = oace.site_energies(pt, s.box, s.periodic, i_all, j_all, prm, s.n, sites)
        (go,) = torch.autograd.grad((torch.as_tensor(wn) * es).sum(), pt)
        assert np.allclose(g[:, i], go.numpy()[:, i], atol=1e-10, rtol=0), (i, g[:, i], go.numpy()[:, i])


@pytest.mark.parametrize("kind", ["T300", "slab111"])
def test_coefficient_gradient_finite_differences(env, kind):
    ops, autograd, ctx, prm, model = env
    s, runner, pos, c1, c2, w = _setup(env, kind)
    e = autograd.ace_energy(pos.detach(), c1, c2, runner)
    g1, g2 = torch.autograd.grad(e, (c1, c2))
    h = 1e-6
    rng = np.random.default_rng(3)
    idx = list(rng.choice(len(prm.c1), 5, replace=False)) + [0, 20, 7000]
    for k in idx:
        for cvec, g in ((c1, g1), (c2, g2)):
            with torch.no_grad():
                base = cvec[k].item()
                cvec[k] = base + h
                ep = autograd.ace_energy(pos.detach(), c1.detach().clone(), c2.detach().clone(), runner).item()
                cvec[k] = base - h
                em = autograd.ace_energy(pos.detach(), c1.detach().clone(), c2.detach().clone(), runner).item()
                cvec[k] = base
            fd = (ep - em) / (2 * h)
            assert g[k].item() == pytest.approx(fd, rel=1e-5, abs=1e-6), (k, g[k].item(), fd)
    # restore the model's coefficients
    runner.sync_coeffs(torch.tensor(prm.c1), torch.tensor(prm.c2))


def test_float32_adjoint_matches_float64(env):
    ops, autograd, ctx, prm, model = env
    s, runner, pos, c1, c2, w = _setup(env, "T800")
    runner.sync_coeffs(torch.tensor(prm.c1), torch.tensor(prm.c2))
    e64 = autograd.ace_energy(pos, c1.detach(), c2.detach(), runner)
    (g64,) = torch.autograd.grad(e64, pos)
    runner.precision = "fp32"
    e32 = autograd.ace_energy(pos, c1.detach(), c2.detach(), runner)
    (g32,) = torch.autograd.grad(e32, pos)
    runner.precision = "fp64"
    err = (g32 - g64).abs().max().item()
    print(f"fp32 adjoint force error {err * 1e3:.5f} meV/A, energy error {abs(e32.item() - e64.item()):.3e} eV")
    assert err < 1e-2  # the stated budget
    assert err < 1e-5, "float32 adjoint force error above its rounding bound"

"""Learned precision indicator kernels against the CPU oracle: features, float32 forward,
gradients of the mean squared error, Adam, bfloat16 inference; and a training smoke test."""

import numpy as np
import pytest
import torch

import synth
from synth import configs
from oracle import geometry, hybrid, mlp as omlp, precision

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ops_ctx():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2411_03002_amd import ops
    return ops, ops.Context(0)


def _std(x, mu, sd):
    # the kernels standardise in float32: (f - mu) / sd
    return ((x.astype(np.float32) - mu.astype(np.float32)) / sd.astype(np.float32)).astype(np.float64)


def _params(seed=3, scale=0.3):
    ps = omlp.init_params(seed)
    rng = np.random.default_rng(seed + 1)
    ps = [p + scale * rng.normal(size=p.shape) for p in ps]
    flat = np.concatenate([p.ravel() for p in ps]).astype(np.float32)
    # the oracle works from exactly the float32 values the device holds
    out, k = [], 0
    for p in ps:
        out.append(flat[k:k + p.size].astype(np.float64).reshape(p.shape))
        k += p.size
    return flat, out


@pytest.mark.parametrize("name", ["void", "slab"])
def test_features_match_oracle(ops_ctx, name):
    ops, ctx = ops_ctx
    print(f"\n[case] features {name}", flush=True)
    s = configs.bulk(8, seed=6, temperature=600.0, void_radius=6.0) if name == "void" else \
        configs.slab100(4, 4, 6, seed=5, temperature=300.0, sigma=0.05)
    atoms = ops.device_atoms(s)
    nl = ops.build_neighbors(ctx, atoms, 5.5)
    e = ops.eam_forces(ctx, atoms, nl, synth.eam_cu_like(), None)
    pr = ops.compute_precision(ctx, atoms, nl, synth.precision_hyb1())
    feat = ops.features(ctx, atoms, nl, e["rho"], pr["csp"], e["f"]).cpu().numpy()
    csr = geometry.neighbor_csr(s.pos, s.lo, s.hi, s.periodic, 5.5)
    ev = hybrid.evaluate(s, synth.eam_cu_like(), None, np.zeros(s.n), csr)
    c = precision.csp(s.pos, s.lo, s.hi, s.periodic, csr, frozen=s.frozen)
    ref = omlp.features(s.pos, s.lo, s.hi, s.periodic, csr, ev["rho"], c, ev["f"]).astype(np.float32)
    assert np.array_equal(feat[:, 1], ref[:, 1])  # CSP (capped) and coordination are exact
    assert np.array_equal(feat[:, 2], ref[:, 2])
    assert np.allclose(feat[:, [0, 3]], ref[:, [0, 3]], rtol=1e-6, atol=1e-7)


def test_forward_gradients_adam(ops_ctx):
    ops, ctx = ops_ctx
    print("\n[case] mlp forward/gradients/adam", flush=True)
    rng = np.random.default_rng(0)
    n = 1000
    feat = np.stack([rng.uniform(1.5, 4.0, n), rng.uniform(0, 30, n), rng.integers(6, 13, n),
                     rng.uniform(0, 1.2, n)], axis=1).astype(np.float32)
    target = rng.normal(-4.0, 1.0, n).astype(np.float32)
    mu, sd = feat.mean(0), feat.std(0)
    flat, ps = _params()
    net = ops.Mlp(ctx, flat, mu, sd)
    ft = torch.as_tensor(feat, device="cuda")
    tt = torch.as_tensor(target, device="cuda")
    x = _std(feat, mu, sd)
    y_ref, _ = omlp.forward(ps, x)
    y = net.forward(ft).cpu().numpy()
    assert np.allclose(y, y_ref, rtol=1e-4, atol=1e-4)
    g, loss = net.gradients(ft, tt)
    loss_ref, g_ref = omlp.loss_and_grad(ps, x, target.astype(np.float64))
    assert loss.item() == pytest.approx(loss_ref, rel=1e-4)
    gflat = g.cpu().numpy()
    gref = np.concatenate([a.ravel() for a in g_ref])
    scale = np.abs(gref).max()
    assert np.allclose(gflat, gref, rtol=1e-3, atol=1e-5 * scale)
    # Adam on both sides from the same gradient
    p_ref = [p.copy() for p in ps]
    m = [np.zeros_like(p) for p in ps]
    v = [np.zeros_like(p) for p in ps]
    for t in (1, 2, 3):
        g, _ = net.gradients(ft, tt)
        gg = g.cpu().numpy().astype(np.float64)
        grads, k = [], 0
        for p in p_ref:
            grads.append(gg[k:k + p.size].reshape(p.shape))
            k += p.size
        net.adam_step(g, lr=1e-3)
        omlp.adam_step(p_ref, grads, m, v, t, lr=1e-3)
        # keep the oracle on the device's float32 parameter values
        got = net.params()
        ref_flat = np.concatenate([p.ravel() for p in p_ref])
        assert np.allclose(got, ref_flat, rtol=0, atol=2e-6)
        k = 0
        for idx, p in enumerate(p_ref):
            p_ref[idx] = got[k:k + p.size].astype(np.float64).reshape(p.shape)
            k += p.size


def test_bf16_inference(ops_ctx):
    ops, ctx = ops_ctx
    print("\n[case] mlp bf16 inference", flush=True)
    rng = np.random.default_rng(1)
    n = 5003  # not a multiple of the 64-atom tile
    feat = np.stack([rng.uniform(1.5, 4.0, n), rng.uniform(0, 30, n), rng.integers(6, 13, n),
                     rng.uniform(0, 1.2, n)], axis=1).astype(np.float32)
    mu, sd = feat.mean(0), feat.std(0)
    flat, ps = _params(seed=9, scale=0.2)
    net = ops.Mlp(ctx, flat, mu, sd)
    y = net.infer_bf16(torch.as_tensor(feat, device="cuda")).cpu().numpy()
    x = _std(feat, mu, sd).astype(np.float32)
    y_ref = omlp.forward_bf16(ps, x)
    y32, _ = omlp.forward(ps, x.astype(np.float64))
    err = np.abs(y - y_ref)
    assert np.max(err / (np.abs(y_ref) + 0.1)) < 1e-2, err.max()
    # and bf16 stays close to the float32 network
    assert np.max(np.abs(y - y32)) < 0.1


def test_training_reduces_loss(ops_ctx):
    ops, ctx = ops_ctx
    print("\n[case] mlp training", flush=True)
    rng = np.random.default_rng(2)
    n = 20000
    feat = rng.normal(size=(n, 4)).astype(np.float32)
    target = (np.tanh(feat[:, 0]) - 0.5 * feat[:, 3] ** 2 + 0.3 * feat[:, 1] * feat[:, 2]).astype(np.float32)
    flat = np.concatenate([p.ravel() for p in omlp.init_params(0)]).astype(np.float32)
    net = ops.Mlp(ctx, flat, np.zeros(4), np.ones(4))
    ft = torch.as_tensor(feat, device="cuda")
    tt = torch.as_tensor(target, device="cuda")
    g = torch.Generator().manual_seed(0)
    losses = []
    for epoch in range(6):
        perm = torch.randperm(n, generator=g).to(torch.int32).cuda()
        for b in range(0, n, 1024):
            loss = net.train_step(ft, tt, perm[b:b + 1024], lr=3e-3)
        losses.append(loss.item())
    pred = net.forward(ft).cpu().numpy()
    mse = float(((pred - target) ** 2).mean())
    print("losses", [round(v, 4) for v in losses], "final mse", mse)
    assert mse < 0.1 * float(target.var())


def test_learned_weight_matches_oracle(ops_ctx):
    """apx_mlp_weight on seeded predictions and features (a third of them outside the
    training range, some on its bounds) against the oracle's learned weight."""
    ops, ctx = ops_ctx
    print("\n[case] learned detection weight", flush=True)
    rng = np.random.default_rng(21)
    n = 70001
    fmin = np.array([0.5, 0.0, 6.0, 0.0], dtype=np.float32)
    fmax = np.array([3.0, 50.0, 14.0, 4.0], dtype=np.float32)
    feat = np.stack([rng.uniform(0.3, 3.2, n), rng.uniform(0, 52, n), rng.integers(5, 16, n),
                     rng.uniform(0, 4.3, n)], axis=1).astype(np.float32)
    feat[:50, 3] = fmax[3]
    feat[50:100, 0] = fmin[0]
    pred = rng.uniform(np.log(1.5e-3), np.log(0.05), n).astype(np.float32)
    flat, _ = _params()
    net = ops.Mlp(ctx, flat, np.zeros(4), np.ones(4))
    net.set_range(fmin, fmax)
    tau_lo, tau_hi = 5e-3, 1e-2
    got = net.weight(torch.as_tensor(pred, device="cuda"), torch.as_tensor(feat, device="cuda"), tau_lo,
                     tau_hi).cpu().numpy()
    ref = omlp.learned_w0(pred, feat, fmin, fmax, tau_lo, tau_hi)
    assert np.array_equal(got > 0, ref > 0)
    assert np.array_equal(got == 1.0, ref == 1.0)
    assert np.abs(got - ref).max() < 1e-13
    inside = np.all((feat >= fmin) & (feat <= fmax), axis=1)
    assert 0.2 < inside.mean() < 0.8 and ((ref > 0) & (ref < 1)).sum() > 1000
    # apx_mlp_precision is the bfloat16 inference followed by this weight
    ft = torch.as_tensor(feat, device="cuda")
    p2, w2 = net.precision(ft, tau_lo, tau_hi)
    assert torch.equal(p2, net.infer_bf16(ft))
    assert torch.equal(w2, net.weight(p2, ft, tau_lo, tau_hi))


def test_labels_and_feature_stats_match_oracle(ops_ctx):
    ops, ctx = ops_ctx
    print("\n[case] learned labels and feature statistics", flush=True)
    rng = np.random.default_rng(22)
    n = 100003
    fp = rng.normal(0.0, 0.5, size=(3, n))
    ff = fp + rng.normal(0.0, 0.01, size=(3, n)) * (rng.uniform(size=n) < 0.7)
    dF, lab = ops.mlp_labels(ctx, torch.as_tensor(fp, device="cuda"), torch.as_tensor(ff, device="cuda"))
    dF_ref, lab_ref = omlp.labels(fp, ff)
    assert np.allclose(dF.cpu().numpy(), dF_ref, rtol=1e-15, atol=0)
    lab = lab.cpu().numpy()
    ulp = np.abs(lab.view(np.int32) - lab_ref.view(np.int32))
    assert ulp.max() <= 1, ulp.max()
    feat = np.stack([rng.uniform(1.5, 4.0, n), rng.uniform(0, 50, n), rng.integers(6, 13, n),
                     rng.exponential(0.3, n)], axis=1).astype(np.float32)
    st = ops.feature_stats(ctx, torch.as_tensor(feat, device="cuda"))
    ref = omlp.feature_stats(feat)
    for k in ("mean", "sd"):
        assert np.allclose(st[k], ref[k], rtol=1e-12, atol=0), k
    for k in ("min", "max"):
        assert np.array_equal(st[k], ref[k]), k


def test_weighted_sum(ops_ctx):
    import math
    ops, ctx = ops_ctx
    print("\n[case] weighted energy sum", flush=True)
    rng = np.random.default_rng(23)
    for n in (0, 1, 2047, 300001):
        w = np.where(rng.uniform(size=n) < 0.5, 0.0, rng.uniform(size=n))
        e = rng.normal(-3.5, 0.2, size=n)
        got = ops.weighted_sum(ctx, torch.as_tensor(w, device="cuda"), torch.as_tensor(e, device="cuda")).item()
        ref = math.fsum((w * e).tolist())
        assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)), (n, got, ref)
        got1 = ops.weighted_sum(ctx, None, torch.as_tensor(e, device="cuda")).item()
        assert abs(got1 - math.fsum(e.tolist())) <= 1e-12 * max(1.0, abs(got1)), n

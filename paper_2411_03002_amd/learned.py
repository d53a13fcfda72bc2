"""Learned precision indicator: data generation, training and deployment.

The paper allows the detection argument of the switching function to be replaced by
another criterion (Appendix B, after eq. lambda_1_i).  Here a 4-64-64-64-1 network is
trained, with the library's own kernels, to predict log(|F_ACE - F_EAM| + 1e-3) from
cheap per-atom descriptors; the labels are produced by the method itself (full-ACE and
pure-EAM forces from the library).  Deployed, its prediction becomes an additional
detection weight combined with the centro-symmetry weight by max (the centro-symmetry
criterion stays as fallback: atoms with features outside the training range use it
alone), followed by the usual spreading.

Every step of the method (labels, input statistics, training, inference, weights) runs in
libapx.so; this module orders the calls.  `assess` is the evaluation of a result, not part
of the method.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np
import torch

from . import ops

EPS_LABEL = 1e-3  # eV/A offset inside the logarithm of the label


def glorot_params(seed: int) -> np.ndarray:
    """Initial parameters (float32, layer order W1 b1 W2 b2 W3 b3 W4 b4): Glorot-uniform
    weights drawn layer by layer from default_rng(seed), zero biases."""
    rng = np.random.default_rng(seed)
    out = []
    for a, b in zip((4, 64, 64, 64), (64, 64, 64, 1)):
        lim = math.sqrt(6.0 / (a + b))
        out.append(rng.uniform(-lim, lim, size=(b, a)).ravel())
        out.append(np.zeros(b))
    return np.concatenate(out).astype(np.float32)


@dataclasses.dataclass
class Snapshot:
    feat: torch.Tensor   # [n, 4] float32
    label: torch.Tensor  # [n] float32, log(|dF| + 1e-3)
    dF: torch.Tensor     # [n] float64, |F_ACE - F_EAM| (eV/A)
    csp: torch.Tensor    # [n] float64


def thermalize(ctx: ops.Context, system, eam, steps: int) -> ops.DeviceAtoms:
    """Integrates ``system`` (positions and velocities) with the fast potential for
    ``steps`` steps of 1 fs and returns the final positions on the device."""
    atoms = ops.device_atoms(system)
    md = ops.MD(ctx, atoms, eam, None, None, dt=1e-3, mode="eam", precision_every=0)
    pos = atoms.pos.clone()
    vel = torch.as_tensor(system.vel, dtype=torch.float64, device=pos.device).contiguous()
    f, w = md.init(pos)
    md.step(pos, vel, f, w, steps)
    md.close()
    return ops.DeviceAtoms(pos, atoms.lo, atoms.hi, atoms.periodic, atoms.frozen)


def snapshot(ctx: ops.Context, system, eam, ace: ops.AceModel, prec, precision: str = "fp32") -> Snapshot:
    """Features and labels of one configuration (all atoms); ``system`` is a synthetic
    system or atoms already on the device."""
    atoms = system if isinstance(system, ops.DeviceAtoms) else ops.device_atoms(system)
    nl = ops.build_neighbors(ctx, atoms, 5.5)
    e = ops.eam_forces(ctx, atoms, nl, eam, None)
    pr = ops.compute_precision(ctx, atoms, nl, dataclasses.replace(prec, r_hi=0.0) if dataclasses.is_dataclass(prec) else prec)
    feat = ops.features(ctx, atoms, nl, e["rho"], pr["csp"], e["f"])
    everyone = torch.arange(atoms.n, dtype=torch.int32, device=atoms.pos.device)
    a = ops.ace_energy_forces(ctx, atoms, nl, ace, everyone, None, precision)
    dF, label = ops.mlp_labels(ctx, a["f"], e["f"])
    return Snapshot(feat, label, dF, pr["csp"])


def train(ctx: ops.Context, feat: torch.Tensor, label: torch.Tensor, *, epochs: int = 20, batch: int = 4096,
          lr: float = 1e-3, seed: int = 0, log=None) -> ops.Mlp:
    """Adam on the mean squared error with shuffled mini-batches; returns the network with
    its input standardisation and feature range set from the training data."""
    st = ops.feature_stats(ctx, feat)
    sd = np.maximum(st["sd"], 1e-6)
    net = ops.Mlp(ctx, glorot_params(seed), st["mean"], sd)
    net.set_range(st["min"], st["max"])
    n = feat.shape[0]
    g = torch.Generator().manual_seed(seed)
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).to(torch.int32).to(feat.device)
        for b in range(0, n, batch):
            loss = net.train_step(feat, label, perm[b:b + batch], lr)
        if log is not None:
            log(f"epoch {ep + 1}: last batch mse {loss.item():.4f}")
    return net


def weights(ctx: ops.Context, atoms: ops.DeviceAtoms, nl: ops.NeighborList, prec, eam, net: ops.Mlp | None,
            tau_lo: float, tau_hi: float) -> dict:
    """Precision weights from the centro-symmetry criterion alone, or combined with the
    learned one (net given)."""
    if net is None:
        return ops.compute_precision(ctx, atoms, nl, prec)
    e = ops.eam_forces(ctx, atoms, nl, eam, None)
    first = ops.compute_precision(ctx, atoms, nl, dataclasses.replace(prec, r_hi=0.0))
    feat = ops.features(ctx, atoms, nl, e["rho"], first["csp"], e["f"])
    pred, w0x = net.precision(feat, tau_lo, tau_hi)
    out = ops.compute_precision(ctx, atoms, nl, prec, w0_extra=w0x, csp=first["csp"])
    out["pred"] = pred
    out["w0_learned"] = w0x
    return out


def assess(w: torch.Tensor, dF: torch.Tensor, f_hyb: torch.Tensor, f_ace: torch.Tensor, tau_lo: float,
           tau_hi: float) -> dict:
    """Misassignment statistics of a weight field against the true force difference:
    false negatives (|dF| > tau_hi but w = 0), false positives (|dF| < tau_lo but w > 0),
    and the hybrid force error on the atoms that need the precise potential."""
    need = dF > tau_hi
    fn = need & (w <= 0)
    fp = (dF < tau_lo) & (w > 0)
    err = (f_hyb - f_ace).norm(dim=0)
    e_need = err[need]
    return dict(n=int(w.numel()), active=int((w > 0).sum().item()), need=int(need.sum().item()),
                false_negative=int(fn.sum().item()), false_positive=int(fp.sum().item()),
                force_err_need_rms_meV=float(e_need.pow(2).mean().sqrt().item() * 1e3) if e_need.numel() else 0.0,
                force_err_need_max_meV=float(e_need.max().item() * 1e3) if e_need.numel() else 0.0,
                force_err_all_rms_meV=float(err.pow(2).mean().sqrt().item() * 1e3))

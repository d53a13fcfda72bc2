"""Learned precision indicator (oracle): features, MLP forward/backward, Adam, BF16.

The paper lets the detection argument of eq. lambda_1_i be replaced by another
criterion (Appendix B, the remark after eq. lambda_1_i; Sec. II B).  The learned
criterion is a fully connected network 4-64-64-64-1 with tanh hidden units and a
linear output:
    h1 = tanh(W1 x + b1), h2 = tanh(W2 h1 + b2), h3 = tanh(W3 h2 + b3), y = W4 h3 + b4
on standardised per-atom inputs x = (f - mu) / sigma, f = [rho_EAM, min(CSP, 50),
coordination (neighbours closer than 3.08 A), |F_EAM|].  Its target is
log(|F_ACE - F_EAM| + 1e-3) and the loss is the mean squared error over a batch.
Adam: m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2; p -= lr mhat / (sqrt(vhat) + 1e-8).
BF16 inference: weights and every layer input rounded to bfloat16 (nearest-even),
products summed in float32, tanh in float32.

Detection weight of the learned criterion (Appendix B: eq. lambda_1_i with its argument
replaced; the argument must be 0 for atoms that need the precise potential and 1 for the
others).  The network predicts y = log(|dF| + 1e-3), so the predicted force gap is
exp(y) - 1e-3 and, in the precise-weight form,
    w0 = 1 - f_cut((exp(y) - 1e-3 - tau_lo) / (tau_hi - tau_lo))
with f_cut of Appendix B; an atom with any feature outside the range seen in training
gets 0 here and keeps the centro-symmetry weight alone (the criterion's fallback).
"""

from __future__ import annotations

import numpy as np

from .geometry import displacements, sq_dist
from .precision import f_cut

LAYERS = (4, 64, 64, 64, 1)
COORD_R = 3.08
CSP_CAP = 50.0


def features(pos, lo, hi, periodic, csr, rho, csp, f_eam):
    """[n, 4] float64 features (f_eam is the unweighted EAM force [3, n])."""
    n = pos.shape[1]
    box = np.asarray(hi) - np.asarray(lo)
    offsets, idx = csr
    i = np.repeat(np.arange(n), np.diff(offsets))
    dx, dy, dz = displacements(pos, box, periodic, i, idx)
    close = sq_dist(dx, dy, dz) < COORD_R * COORD_R
    coord = np.bincount(i[close], minlength=n).astype(np.float64)
    fn = np.sqrt((f_eam * f_eam).sum(axis=0))
    return np.stack([rho, np.minimum(csp, CSP_CAP), coord, fn], axis=1)


def init_params(seed: int):
    """Glorot-uniform weights (as inputs; drawn in layer order), zero biases."""
    rng = np.random.default_rng(seed)
    ps = []
    for a, b in zip(LAYERS[:-1], LAYERS[1:]):
        lim = np.sqrt(6.0 / (a + b))
        ps.append(rng.uniform(-lim, lim, size=(b, a)))
        ps.append(np.zeros(b))
    return ps


def forward(params, x):
    """Returns (y [n], cache)."""
    acts = [x]
    h = x
    for k in range(3):
        h = np.tanh(h @ params[2 * k].T + params[2 * k + 1])
        acts.append(h)
    y = (h @ params[6].T + params[7])[:, 0]
    return y, acts


def loss_and_grad(params, x, target):
    """Mean squared error and its gradient with respect to every parameter."""
    y, acts = forward(params, x)
    nb = x.shape[0]
    r = y - target
    loss = float((r * r).mean())
    g = [None] * 8
    dy = (2.0 / nb) * r[:, None]  # [n, 1]
    g[6] = dy.T @ acts[3]
    g[7] = dy.sum(axis=0)
    delta = dy @ params[6]  # [n, 64]
    for k in (2, 1, 0):
        dz = delta * (1.0 - acts[k + 1] ** 2)
        g[2 * k] = dz.T @ acts[k]
        g[2 * k + 1] = dz.sum(axis=0)
        delta = dz @ params[2 * k]
    return loss, g


def adam_step(params, grads, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); updates params, m, v in place."""
    for k in range(len(params)):
        m[k] = b1 * m[k] + (1.0 - b1) * grads[k]
        v[k] = b2 * v[k] + (1.0 - b2) * grads[k] * grads[k]
        mh = m[k] / (1.0 - b1 ** t)
        vh = v[k] / (1.0 - b2 ** t)
        params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)


def to_bf16(a):
    """Round float32 values to the nearest bfloat16 (ties to even), returned as float32."""
    a = np.asarray(a, dtype=np.float32)
    b = a.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32)
    return np.where(np.isnan(a), a, out)


def forward_bf16(params, x):
    """Inference with bf16 weights/activations and float32 sums."""
    h = to_bf16(x)
    for k in range(3):
        W = to_bf16(params[2 * k]).astype(np.float32)
        h = np.tanh((h.astype(np.float32) @ W.T + np.float32(params[2 * k + 1])).astype(np.float32))
        h = to_bf16(h)
    W = to_bf16(params[6]).astype(np.float32)
    return (h.astype(np.float32) @ W.T + np.float32(params[7]))[:, 0].astype(np.float32)


def learned_w0(pred, feat, fmin, fmax, tau_lo, tau_hi):
    """Precise weight from predictions ``pred`` [n] (float32 log force gaps) and features
    ``feat`` [n, 4] (float32): the predicted gap exp(pred) - 1e-3 (float64) switched by
    1 - f_cut((gap - tau_lo) / (tau_hi - tau_lo)); 0 where a feature lies outside
    [fmin, fmax] (float32 bounds, inclusive)."""
    pred = np.asarray(pred, dtype=np.float32).astype(np.float64)
    feat = np.asarray(feat, dtype=np.float32)
    fmin = np.asarray(fmin, dtype=np.float32)
    fmax = np.asarray(fmax, dtype=np.float32)
    inside = np.all((feat >= fmin[None, :]) & (feat <= fmax[None, :]), axis=1)
    gap = np.exp(pred) - 1e-3
    w = 1.0 - f_cut((gap - tau_lo) / (tau_hi - tau_lo))
    return np.where(inside, w, 0.0)


def labels(f_precise, f_fast):
    """Training target of the learned criterion: dF = |F^precise - F^fast| per atom
    (float64, forces [3, n]) and log(dF + 1e-3) rounded to float32."""
    d = np.asarray(f_precise, dtype=np.float64) - np.asarray(f_fast, dtype=np.float64)
    dF = np.sqrt((d * d).sum(axis=0))
    return dF, np.log(dF + 1e-3).astype(np.float32)


def feature_stats(feat):
    """Per-column mean, standard deviation with n - 1 degrees of freedom, minimum and
    maximum of float32 features [n, 4], in float64: the input standardisation and the
    training range of the criterion."""
    x = np.asarray(feat, dtype=np.float32).astype(np.float64)
    mean = x.sum(axis=0) / x.shape[0]
    sd = np.sqrt(((x - mean) ** 2).sum(axis=0) / (x.shape[0] - 1))
    return dict(mean=mean, sd=sd, min=x.min(axis=0), max=x.max(axis=0))

"""Pins of the oracle's learned detection weight (Appendix B: eq. lambda_1_i with its
argument replaced by the predicted force gap; CPU only).

The network predicts y = log(|dF| + 1e-3), so exp(y) - 1e-3 is the predicted gap:
* a gap above tau_hi gives w0 = 1 exactly (f_cut = 0 beyond 1), below tau_lo w0 = 0;
* the midpoint of [tau_lo, tau_hi] gives 1 - f_cut(1/2) = 0.79296875 (f_cut(1/2) =
  0.20703125, Appendix B's polynomial);
* w0 is non-decreasing in y;
* an atom with any feature outside the training range gets 0 (the fallback to the
  centro-symmetry weight happens when the two are combined), the range being inclusive.
"""

import math

import numpy as np

from oracle import mlp

TAU_LO, TAU_HI = 5e-3, 10e-3
FMIN = np.array([0.5, 0.0, 6.0, 0.0], dtype=np.float32)
FMAX = np.array([3.0, 50.0, 14.0, 4.0], dtype=np.float32)


def _feat(n):
    return np.tile(np.array([[1.5, 0.3, 12.0, 0.2]], dtype=np.float32), (n, 1))


def test_learned_weight_values():
    pred = np.array([math.log(0.05), math.log(0.002), math.log(0.0085), math.log(0.011 + 1e-3)], dtype=np.float32)
    w = mlp.learned_w0(pred, _feat(4), FMIN, FMAX, TAU_LO, TAU_HI)
    assert w[0] == 1.0 and w[1] == 0.0 and w[3] == 1.0
    assert abs(w[2] - 0.79296875) < 1e-6


def test_learned_weight_monotone_and_bounded():
    pred = np.linspace(math.log(1e-3) + 1e-3, math.log(0.05), 2001).astype(np.float32)
    w = mlp.learned_w0(pred, _feat(pred.size), FMIN, FMAX, TAU_LO, TAU_HI)
    assert np.all(np.diff(w) >= 0.0)
    assert w.min() == 0.0 and w.max() == 1.0
    inside = (w > 0.0) & (w < 1.0)
    gap = np.exp(pred.astype(np.float64)) - 1e-3
    assert np.all((gap[inside] > TAU_LO) & (gap[inside] < TAU_HI))


def test_learned_weight_range_fallback():
    pred = np.full(6, math.log(0.05), dtype=np.float32)
    feat = _feat(6)
    feat[1, 0] = 3.5         # density above the range
    feat[2, 2] = 5.0         # coordination below
    feat[3, 3] = FMAX[3]     # on the bound: inside
    feat[4, 1] = FMIN[1]     # on the bound: inside
    feat[5, 3] = np.nextafter(FMAX[3], np.float32(10))  # just outside
    w = mlp.learned_w0(pred, feat, FMIN, FMAX, TAU_LO, TAU_HI)
    assert list(w) == [1.0, 0.0, 0.0, 1.0, 1.0, 0.0]


def test_labels_and_feature_stats():
    # a force gap of exactly 1 eV/A gives log(1.001); equal forces give log(1e-3)
    fp = np.zeros((3, 3))
    ff = np.zeros((3, 3))
    fp[:, 0] = [0.6, 0.8, 0.0]
    fp[:, 2] = [3.0, 0.0, 4.0]
    dF, lab = mlp.labels(fp, ff)
    assert list(dF) == [1.0, 0.0, 5.0]
    assert lab[1] == np.float32(math.log(1e-3)) and lab[0] == np.float32(math.log(1.001))
    # two samples per column: mean (a + b)/2, sd |a - b|/sqrt(2)
    feat = np.array([[1.0, 2.0, 12.0, 0.5], [3.0, 2.0, 10.0, 1.5]], dtype=np.float32)
    st = mlp.feature_stats(feat)
    assert list(st["mean"]) == [2.0, 2.0, 11.0, 1.0]
    assert np.allclose(st["sd"], [math.sqrt(2.0), 0.0, math.sqrt(2.0), math.sqrt(0.5)], rtol=1e-15)
    assert list(st["min"]) == [1.0, 2.0, 10.0, 0.5] and list(st["max"]) == [3.0, 2.0, 12.0, 1.5]

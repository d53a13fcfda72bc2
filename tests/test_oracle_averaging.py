"""Pins of the oracle's time-averaged switching (CPU only).

Hand-worked sequences whose every value is exact in binary fix the windows (the past
window of eqs. csp_2_i and lambda_3_i, the N samples before the current one for the CSP
mean, and the alternative current window, the newest N samples; fewer at start-up), the
order of the steps (switch on the averaged CSP, spreading of the averaged w0, mean of the
spread weights, then the minimum step) and both exceptions of the minimum-step filter.
Several sequences give different values under the two windows, so each reading is pinned
on its own.  The paper's statement that a step change takes N samples to pass through a
mean fixes the window length independently.
"""

import numpy as np
import pytest

import synth
from synth import configs
from oracle import averaging, geometry, precision


def _line(n=3):
    """n atoms on a line, 20 A apart (beyond every cutoff), in a periodic box."""
    pos = np.zeros((3, n))
    pos[0] = 20.0 * np.arange(n) + 5.0
    return synth.System(pos, np.zeros(3), np.array([20.0 * n, 30.0, 30.0]), (1, 1, 1))


def _csr(s):
    return geometry.neighbor_csr(s.pos, s.lo, s.hi, s.periodic, 5.5)


@pytest.mark.parametrize("window,want", [("past", [1.0, 1.0, 1.5, 2.0, 3.0]),
                                         ("current", [1.0, 1.5, 2.0, 3.0, 4.0])])
def test_moving_average_window_and_startup(window, want):
    s = _line(1)
    p = synth.PrecisionParams(csp_lo=0.0, csp_hi=100.0, switch_kind=0)
    tas = averaging.TimeAveragedSwitch(n_avg=3, dw_min=0.0, window=window)
    got = [tas.update(s, p, _csr(s), csp=np.array([v]))["csp_avg"][0] for v in (1.0, 2.0, 3.0, 4.0, 5.0)]
    # past: the samples before the current one (the current one alone at the first call);
    # current: the samples so far, then the newest three
    assert got == want


@pytest.mark.parametrize("window,lag", [("past", 1), ("current", 0)])
def test_step_change_takes_n_samples(window, lag):
    # a mean over N samples needs N samples to follow a step completely; the past window
    # sees a sample one call later
    s = _line(1)
    p = synth.PrecisionParams(csp_lo=0.0, csp_hi=100.0, switch_kind=0)
    n = 7
    tas = averaging.TimeAveragedSwitch(n_avg=n, dw_min=0.0, window=window)
    for _ in range(n):
        tas.update(s, p, _csr(s), csp=np.array([0.0]))
    prev = 0.0
    for k in range(1, n + lag + 1):
        v = tas.update(s, p, _csr(s), csp=np.array([10.0]))["csp_avg"][0]
        if k <= lag:
            assert v == 0.0
        elif k < n + lag:
            assert prev < v < 10.0
        else:
            assert v == 10.0
        prev = v


def test_mean_bounds_random():
    rng = np.random.default_rng(5)
    for m in range(1, 12):
        smp = [rng.uniform(-3, 7, size=50) for _ in range(m)]
        avg = averaging.moving_average(smp)
        lo, hi = np.min(smp, axis=0), np.max(smp, axis=0)
        assert np.all(avg >= lo) and np.all(avg <= hi)
    with pytest.raises(ValueError):
        averaging.moving_average([])


def test_switch_on_averaged_csp_hyb1():
    # CSP samples 3.0, 2.75, then 2.5.  Current window: mean 2.75, x = 0.5,
    # w0 = 1 - f_cut(0.5) = 1 - 0.20703125.  Past window: the mean of the two earlier
    # samples, 2.875, x = 0.75, f_cut(0.75) = 1 - 1.40625 + 0.52734375 - 0.0889892578125
    # = 0.0321044921875 (every term exact in binary), w0 = 0.9678955078125.
    s = _line(1)
    p = synth.PrecisionParams(csp_lo=2.5, csp_hi=3.0, switch_kind=1)
    got = {}
    for window in ("current", "past"):
        tas = averaging.TimeAveragedSwitch(n_avg=3, dw_min=0.0, window=window)
        for v in (3.0, 2.75):
            tas.update(s, p, _csr(s), csp=np.array([v]))
        got[window] = tas.update(s, p, _csr(s), csp=np.array([2.5]))
    assert got["current"]["csp_avg"][0] == 2.75
    assert got["current"]["w0"][0] == 0.79296875
    assert got["past"]["csp_avg"][0] == 2.875
    assert got["past"]["w0"][0] == 0.9678955078125
    # the newest sample alone would give w0 = 0
    assert precision.w0_from_csp(np.array([2.5]), 2.5, 3.0, 1)[0] == 0.0


HAND = {  # CSP sequence -> expected w0, mean of w, filtered w (linear switch on [0, 1], N = 2, step 0.3)
    "current": ([0.0, 0.5, 1.0, 0.75, 0.75, 1.0, 1.0], [0.0, 0.25, 0.75, 0.875, 0.75, 0.875, 1.0],
                [0.0, 0.0, 0.75, 0.75, 0.75, 0.75, 1.0]),
    "past": ([0.0, 0.0, 0.5, 1.0, 0.75, 0.75, 1.0], [0.0, 0.0, 0.25, 0.75, 0.875, 0.75, 0.875],
             [0.0, 0.0, 0.0, 0.75, 0.75, 0.75, 0.75]),
}


@pytest.mark.parametrize("window", ["past", "current"])
def test_hand_sequence_weight_mean_and_min_step(window):
    # linear switch on [0, 1], no spreading, N = 2, minimum step 0.3
    s = _line(1)
    p = synth.PrecisionParams(csp_lo=0.0, csp_hi=1.0, switch_kind=0)
    tas = averaging.TimeAveragedSwitch(n_avg=2, dw_min=0.3, window=window)
    seq = [0.0, 1.0, 1.0, 0.5, 1.0, 1.0, 1.0]
    want_w0, want_avg, want_w = HAND[window]
    for c, a, b, w in zip(seq, want_w0, want_avg, want_w):
        out = tas.update(s, p, _csr(s), csp=np.array([c]))
        assert (out["w0"][0], out["w_avg"][0], out["w"][0]) == (a, b, w), c
        assert out["mask"][0] == (w > 0)


def test_min_step_filter_cases():
    f = averaging.min_step_filter
    prev = None
    got = []
    for a in (0.5, 0.52, 0.56, 0.7, 0.98, 1.0, 0.99, 0.995, 0.02, 0.0):
        prev = f(np.array([a]), prev, 0.05)
        got.append(prev[0])
    assert got == [0.5, 0.5, 0.56, 0.7, 0.98, 1.0, 1.0, 1.0, 0.02, 0.0]
    # a change of exactly the minimum step is taken
    assert f(np.array([0.5]), np.array([0.25]), 0.25)[0] == 0.5
    assert f(np.array([0.375]), np.array([0.25]), 0.25)[0] == 0.25


@pytest.mark.parametrize("window,mean", [("past", 9.0), ("current", 6.0)])
def test_spreading_uses_averaged_w0(window, mean):
    # a slab whose atom k carries a large CSP in two of three samples: the mean detects it,
    # and its neighbours within r_lo get w_min = 1 although the newest sample is 0
    s = configs.slab100(4, 4, 4, seed=3, temperature=0.0, sigma=0.0, velocities=False)
    p = synth.precision_static()
    csr = _csr(s)
    mob = np.nonzero(~s.frozen.astype(bool))[0]
    k = mob[len(mob) // 2]
    tas = averaging.TimeAveragedSwitch(n_avg=3, dw_min=0.0, window=window)
    for v in (9.0, 9.0, 0.0):
        c = np.zeros(s.n)
        c[k] = v
        out = tas.update(s, p, csr, csp=c)
    assert out["csp_avg"][k] == mean and out["w0"][k] == 1.0
    box = s.hi - s.lo
    jj = np.arange(s.n)
    dx, dy, dz = geometry.displacements(s.pos, box, s.periodic, np.full(s.n, k), jj)
    r = np.sqrt(geometry.sq_dist(dx, dy, dz))
    mobile = ~s.frozen.astype(bool)
    assert np.all(out["w_min"][(r <= p.r_lo) & mobile] == 1.0)
    assert np.all(out["w_min"][r >= p.r_hi] == 0.0)
    assert np.all(out["w_min"][s.frozen.astype(bool)] == 0.0)
    # a minimum step of 0 passes every mean
    assert np.array_equal(out["w"], out["w_avg"])


def test_single_sample_reduces_to_instantaneous():
    # current window, N = 1: the instantaneous evaluation; past window, N = 1: the switch
    # acts on the previous call's CSP
    s = configs.slab100(4, 4, 5, seed=4, temperature=300.0, sigma=0.12, velocities=False)
    p = synth.precision_static()
    rng = np.random.default_rng(9)
    tas = averaging.TimeAveragedSwitch(n_avg=1, dw_min=0.0, window="current")
    past = averaging.TimeAveragedSwitch(n_avg=1, dw_min=0.0, window="past")
    prev_csp = None
    for _ in range(3):
        d = rng.normal(0.0, 0.05, size=s.pos.shape)
        d[:, s.frozen.astype(bool)] = 0.0
        s.pos = s.pos + d
        csr = _csr(s)
        out = tas.update(s, p, csr)
        ref = precision.compute_precision(s, p, csr)
        for key in ("csp", "w0", "mask", "active"):
            assert np.array_equal(out[key], ref[key]), key
        assert np.array_equal(out["w"], ref["w"])
        pout = past.update(s, p, csr)
        lagged = ref["csp"] if prev_csp is None else prev_csp
        assert np.array_equal(pout["csp_avg"], lagged)
        assert np.array_equal(pout["w0"], precision.w0_from_csp(lagged, p.csp_lo, p.csp_hi, p.switch_kind, s.frozen))
        prev_csp = ref["csp"]
    assert out["mask"].sum() > 0

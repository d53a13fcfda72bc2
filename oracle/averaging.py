"""Time-averaged switching (oracle; test infrastructure only, never called by the library).

Paper passages (Appendix B, "Construction of the switching function"; parameters in
Appendix F, "Centro-symmetry parameter" and "Switching function", Table IV):
* eq. csp_2_i: the centro-symmetry parameter entering the switch is the mean of the
  last N_CSP,avg samples of CSP_i.
* eq. lambda_1_i: the switch is applied to that mean (here in the precise-weight form
  w0 = 1 - lambda_0, as in the instantaneous evaluation).
* eq. lambda_2_i: spreading of w0 over neighbours within r_hi gives the instantaneous
  weight w_min = 1 - lambda_min.
* eq. lambda_3_i: the weight used is built from the mean of the last N_lambda,avg
  samples of w_min.
* eq. lambda_4_i: minimum step size.  The new mean replaces the previous filtered value
  only if it differs from it by at least dw_min, or if it is exactly 0 or 1; otherwise
  the previous filtered value is kept.
Two readings of the windows, selected by ``window``:
* "past" (the default; eqs. csp_2_i and lambda_3_i as printed, sums over n = 1..N of
  samples at t - n dt): the mean of CSP that forms lambda_0 at time t holds the samples
  taken before t, not the one taken at t; the weight used by the force evaluations after
  a sample is the filtered mean of the spread weights up to and including that sample.
  The force routine's order of Appendix G (fast potential, precise potential, CSP, then
  lambda) fits this reading: the forces of step t use the weight formed before t, and the
  CSP and lambda samples of step t serve the steps after it.
* "current": the newest sample enters both means (eq. vv step 2 read as forming the weight
  of step t from the positions of step t before its forces).
With "past", the first call has no earlier CSP sample and averages the current one.

Readings (the paper is silent on these):
* One call takes one sample.  A caller that updates the weights every k steps samples
  every k steps, and N then counts samples, not steps.
* Before N samples exist, a mean is over the samples available.
* The first call has no previous filtered value: the filtered weight is the mean.
* Both means use the same N (the paper sets N_lambda,avg = N_CSP,avg).
* In the precise-weight form 1 - mean(lambda) = mean(1 - lambda) and the filter's tests
  carry over unchanged (|a - b| is the same for lambda and for w = 1 - lambda; lambda in
  {0, 1} is w in {1, 0}).

Floating-point order (a definition shared with the library): a mean adds the samples
newest first, starting from 0.0, each addition rounded, then divides by the number of
samples (correctly rounded).  Every other value follows the instantaneous evaluation in
``oracle.precision``.
"""

from __future__ import annotations

import numpy as np

from . import precision


def moving_average(samples_newest_first):
    """Mean of the given samples (a list of arrays, newest first), added in that order."""
    if not samples_newest_first:
        raise ValueError("no samples")
    acc = np.zeros_like(np.asarray(samples_newest_first[0], dtype=np.float64))
    for s in samples_newest_first:
        acc = acc + np.asarray(s, dtype=np.float64)
    return acc / float(len(samples_newest_first))


def min_step_filter(w_avg, w_prev, dw_min):
    """eq. lambda_4_i: keep the previous filtered weight unless the mean moved by at least
    dw_min or reached 0 or 1.  w_prev None (first sample) returns the mean."""
    w_avg = np.asarray(w_avg, dtype=np.float64)
    if w_prev is None:
        return w_avg.copy()
    take = (np.abs(w_avg - w_prev) >= dw_min) | (w_avg == 0.0) | (w_avg == 1.0)
    return np.where(take, w_avg, w_prev)


class TimeAveragedSwitch:
    """Per-atom history of CSP and w_min samples and the filtered weight."""

    def __init__(self, n_avg: int, dw_min: float, window: str = "past"):
        if n_avg < 1:
            raise ValueError("n_avg must be at least 1")
        if window not in ("past", "current"):
            raise ValueError(window)
        self.window = window
        self.n_avg = int(n_avg)
        self.dw_min = float(dw_min)
        self.csp_hist = []  # newest first
        self.w_hist = []
        self.w = None

    def update(self, system, params, csr, w0_extra=None, csp=None):
        """One sample at the positions of ``system``; returns the pipeline's values.

        ``csp`` (optional) replaces the instantaneous CSP of the positions."""
        fz = system.frozen
        if csp is None:
            csp = precision.csp(system.pos, system.lo, system.hi, system.periodic, csr, r_cut=params.r_cut,
                                n_nn=params.n_nn, n_buffer=params.n_buffer, frozen=fz)
        csp = np.asarray(csp, dtype=np.float64)
        if self.window == "past" and self.csp_hist:
            csp_avg = moving_average(self.csp_hist)  # the samples before this one
        else:
            csp_avg = moving_average(([csp] + self.csp_hist)[:self.n_avg])
        self.csp_hist = ([csp] + self.csp_hist)[:self.n_avg]
        w0 = precision.w0_from_csp(csp_avg, params.csp_lo, params.csp_hi, params.switch_kind, fz)
        local = getattr(params, "extra_local", False)
        if w0_extra is not None and not local:
            w0 = precision.combine_extra(w0, w0_extra, fz)
        w_min = precision.spread(system.pos, system.lo, system.hi, system.periodic, w0, params.r_lo, params.r_hi, fz)
        if w0_extra is not None and local:
            w_min = precision.combine_extra(w_min, w0_extra, fz)
        self.w_hist = ([w_min] + self.w_hist)[:self.n_avg]
        w_avg = moving_average(self.w_hist)
        self.w = min_step_filter(w_avg, self.w, self.dw_min)
        mask = (self.w > 0.0).astype(np.uint8)
        return dict(csp=np.asarray(csp, dtype=np.float64), csp_avg=csp_avg, w0=w0, w_min=w_min, w_avg=w_avg,
                    w=self.w.copy(), mask=mask, active=np.nonzero(mask)[0].astype(np.int64))


__all__ = ["moving_average", "min_step_filter", "TimeAveragedSwitch"]

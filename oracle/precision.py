"""Detection and switching (oracle): CSP, w0, spreading, mask, active list.

Paper passages:
* CSP, LAMMPS definition with N + N_buffer candidates: Sec. II B (eq. csp_1_i) and
  Appendix A.  The N + N_buffer nearest neighbours (within the force cutoff) are taken
  by (squared distance, index); among all pairs of them the N/2 smallest values of
  |r_a + r_b|^2 are summed.  Fewer than N + N_buffer neighbours gives CSP = +inf.
* f_cut polynomial: Appendix B (equation below eq. lambda_1_i).
* Switch from CSP to the precise weight: Appendix B eq. lambda_1_i, read as
  w0 = 1 - f_cut((CSP - CSP_lo) / (CSP_hi - CSP_lo)) (the printed expression taken as the
  weight of the precise potential, so that CSP <= CSP_lo gives the fast potential), or
  the linear ramp clamp((CSP - lo)/(hi - lo), 0, 1) for the small plain workload.
* Spreading: Appendix B eq. lambda_2_i in the precise-weight form
  w_i = max(w0_i, max_{j : r_ij < r_hi} w0_j * f_cut((r_ij - r_lo)/(r_hi - r_lo))).
  Time averages (eqs. lambda_3_i, lambda_4_i, csp_2_i) are not part of this evaluation.
* Frozen atoms keep w = 0, get no CSP and are never sources (Appendix G, atom subgroups).

Floating-point order (shared by definition with the library): every value below is
computed with separately rounded operations in the order written.
"""

from __future__ import annotations

import numpy as np

from .geometry import displacements, sq_dist, min_image


def f_cut(x: np.ndarray) -> np.ndarray:
    """1 for x < 0; ((1 - 1.875 x) + 1.25 x^3) - 0.375 x^5 on [0, 1]; 0 for x > 1.

    x^3 = (x*x)*x and x^5 = x^3*(x*x).
    """
    x = np.asarray(x, dtype=np.float64)
    with np.errstate(invalid="ignore", over="ignore"):
        x2 = x * x
        x3 = x2 * x
        x5 = x3 * x2
        poly = ((1.0 - 1.875 * x) + 1.25 * x3) - 0.375 * x5
    return np.where(x < 0.0, 1.0, np.where(x > 1.0, 0.0, poly))


def csp(pos, lo, hi, periodic, csr, r_cut=5.0, n_nn=12, n_buffer=0, frozen=None):
    """Centro-symmetry parameter of every atom (0 for frozen atoms)."""
    n = pos.shape[1]
    box = np.asarray(hi, dtype=np.float64) - np.asarray(lo, dtype=np.float64)
    offsets, idx = csr
    m = n_nn + n_buffer
    half = n_nn // 2
    out = np.zeros(n)
    ia, ib = np.triu_indices(m, k=1)
    for i in range(n):
        if frozen is not None and frozen[i]:
            continue
        js = idx[offsets[i]:offsets[i + 1]]
        ii = np.full(js.shape, i)
        dx, dy, dz = displacements(pos, box, periodic, ii, js)
        r2 = sq_dist(dx, dy, dz)
        inside = r2 < r_cut * r_cut
        js, dx, dy, dz, r2 = js[inside], dx[inside], dy[inside], dz[inside], r2[inside]
        if js.size < m:
            out[i] = np.inf
            continue
        order = np.lexsort((js, r2))[:m]
        ax, ay, az = dx[order], dy[order], dz[order]
        sx = ax[ia] + ax[ib]
        sy = ay[ia] + ay[ib]
        sz = az[ia] + az[ib]
        v = np.sort(sq_dist(sx, sy, sz))[:half]
        s = 0.0
        for t in v:
            s = s + t
        out[i] = s
    return out


def w0_from_csp(c, csp_lo, csp_hi, switch_kind, frozen=None):
    """Initial precise weight from the CSP (eq. lambda_1_i reading, or the linear ramp)."""
    x = (np.asarray(c, dtype=np.float64) - csp_lo) / (csp_hi - csp_lo)
    if switch_kind == 0:
        w0 = np.minimum(np.maximum(x, 0.0), 1.0)
    elif switch_kind == 1:
        w0 = 1.0 - f_cut(x)
    else:
        raise ValueError(switch_kind)
    if frozen is not None:
        w0 = np.where(frozen.astype(bool), 0.0, w0)
    return w0


def spread(pos, lo, hi, periodic, w0, r_lo, r_hi, frozen=None):
    """Spreading of eq. lambda_2_i, precise-weight form, by brute force over sources.

    Candidates use the minimum-image distance; the inclusion test is r2 < r_hi^2 and
    the radius entering f_cut is sqrt(r2) (correctly rounded).
    """
    w = np.array(w0, dtype=np.float64, copy=True)
    n = pos.shape[1]
    fz = np.zeros(n, bool) if frozen is None else frozen.astype(bool)
    if r_hi <= 0.0:
        w[fz] = 0.0
        return w
    box = np.asarray(hi, dtype=np.float64) - np.asarray(lo, dtype=np.float64)
    sources = np.nonzero((w0 > 0.0) & ~fz)[0]
    targets = np.arange(n)
    for j in sources:
        jj = np.full(n, j)
        dx, dy, dz = displacements(pos, box, periodic, jj, targets)
        r2 = sq_dist(dx, dy, dz)
        sel = r2 < r_hi * r_hi
        r = np.sqrt(r2[sel])
        val = w0[j] * f_cut((r - r_lo) / (r_hi - r_lo))
        w[sel] = np.maximum(w[sel], val)
    w[fz] = 0.0
    return w


def combine_extra(w, w0_extra, frozen=None):
    """max(w, w0_extra) with frozen atoms kept at 0: an additional detection weight (the
    learned criterion's) joined to a CSP-based weight."""
    out = np.maximum(np.asarray(w, dtype=np.float64), np.asarray(w0_extra, dtype=np.float64))
    if frozen is not None:
        out = np.where(frozen.astype(bool), 0.0, out)
    return out


def compute_precision(system, params, csr, w0_extra=None, csp_given=None):
    """Returns dict(csp, w0, w, mask, active) for ``system`` under ``params``.

    ``w0_extra`` joins the CSP-based w0 before the spreading, or the spread weight after it
    when ``params.extra_local`` is set (its detections are then not spread); ``csp_given``
    replaces the CSP of the positions."""
    frozen = system.frozen
    if csp_given is None:
        c = csp(system.pos, system.lo, system.hi, system.periodic, csr, r_cut=params.r_cut,
                n_nn=params.n_nn, n_buffer=params.n_buffer, frozen=frozen)
    else:
        c = np.asarray(csp_given, dtype=np.float64)
    w0 = w0_from_csp(c, params.csp_lo, params.csp_hi, params.switch_kind, frozen)
    local = getattr(params, "extra_local", False)
    if w0_extra is not None and not local:
        w0 = combine_extra(w0, w0_extra, frozen)
    w = spread(system.pos, system.lo, system.hi, system.periodic, w0, params.r_lo,
               params.r_hi, frozen)
    if w0_extra is not None and local:
        w = combine_extra(w, w0_extra, frozen)
    mask = (w > 0.0).astype(np.uint8)
    active = np.nonzero(mask)[0].astype(np.int64)
    return dict(csp=c, w0=w0, w=w, mask=mask, active=active)


__all__ = ["f_cut", "csp", "w0_from_csp", "spread", "combine_extra", "compute_precision", "min_image"]

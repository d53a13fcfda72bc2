"""Pins of the oracle's geometry, CSP, switching and spreading (CPU only).

Each check ties the oracle to something other than itself: values printed in the
paper, exact lattice geometry, or brute force.
"""

import numpy as np
import pytest

import synth
from synth import configs
from oracle import geometry, precision

A = synth.A_CU


def _perfect(cells=4):
    pos = synth.fcc_positions(cells, cells, cells)
    hi = np.full(3, cells * A)
    return synth.System(pos, np.zeros(3), hi, (1, 1, 1))


def test_fcut_printed_polynomial():
    # Appendix B: f(x) = 1 - 1.875x + 1.25x^3 - 0.375x^5 on [0, 1], 1 below, 0 above
    x = np.array([-1.0, 0.0, 0.5, 1.0, 2.0])
    f = precision.f_cut(x)
    assert f[0] == 1.0 and f[1] == 1.0 and f[3] == 0.0 and f[4] == 0.0
    assert f[2] == 0.20703125  # exact in binary: 1 - 0.9375 + 0.15625 - 0.01171875
    # first and second derivative vanish at x = 1 (the paper's smoothness claim there)
    h = 1e-4
    d1 = (precision.f_cut(1 - h) - precision.f_cut(1 - 2 * h)) / h
    assert abs(d1) < 1e-6
    # the printed form is not C1 at x = 0: slope -1.875 just above 0
    assert abs((precision.f_cut(h) - 1.0) / h + 1.875) < 1e-3


def test_neighbor_counts_perfect_fcc():
    s = _perfect(4)
    off, idx = geometry.neighbor_csr(s.pos, s.lo, s.hi, s.periodic, 5.5)
    # shells at a/sqrt2 (12), a (6), a*sqrt(3/2) (24), a*sqrt2 = 5.112 (12): 54 within 5.5 A
    assert np.all(np.diff(off) == 54)
    for i in (0, 7, 100):
        row = idx[off[i]:off[i + 1]]
        assert np.all(np.diff(row) > 0) and i not in row


def test_neighbor_kdtree_matches_brute_force():
    s = configs.bulk(11, seed=3, temperature=600.0)  # 5324 atoms: KD-tree path
    assert s.n > 4000
    off, idx = geometry.neighbor_csr(s.pos, s.lo, s.hi, s.periodic, 5.5)
    rng = np.random.default_rng(0)
    box = s.box
    for i in rng.choice(s.n, 25, replace=False):
        d = s.pos - s.pos[:, [i]]
        d -= box[:, None] * np.round(d / box[:, None])
        r2 = (d * d).sum(0)
        expect = np.nonzero((r2 < 5.5 ** 2) & (np.arange(s.n) != i))[0]
        assert np.array_equal(idx[off[i]:off[i + 1]], expect)


def test_csp_perfect_lattice_is_zero():
    s = _perfect(4)
    csr = geometry.neighbor_csr(s.pos, s.lo, s.hi, s.periodic, 5.5)
    c = precision.csp(s.pos, s.lo, s.hi, s.periodic, csr)
    assert np.max(np.abs(c)) <= 1e-20


def test_csp_single_vacancy_exact():
    s = _perfect(4)
    vac = 37
    keep = np.arange(s.n) != vac
    centre = s.pos[:, vac]
    s.pos = np.ascontiguousarray(s.pos[:, keep])
    csr = geometry.neighbor_csr(s.pos, s.lo, s.hi, s.periodic, 5.5)
    c = precision.csp(s.pos, s.lo, s.hi, s.periodic, csr)
    d = s.pos - centre[:, None]
    d -= s.box[:, None] * np.round(d / s.box[:, None])
    nn = np.sqrt((d * d).sum(0)) < 0.8 * A
    assert nn.sum() == 12
    # a missing nearest neighbour leaves its opposite unpaired: the best partner is a
    # second-shell site, giving |r_a + r_b|^2 = a^2/2 for every tie choice
    assert np.allclose(c[nn], A * A / 2.0, rtol=0, atol=1e-12)
    assert np.max(np.abs(c[~nn])) < 1e-20


def test_csp_surface_top_layer():
    s = configs.slab100(4, 4, 4, seed=1, temperature=0.0, frozen_planes=0, velocities=False)
    csr = geometry.neighbor_csr(s.pos, s.lo, s.hi, s.periodic, 5.5)
    c = precision.csp(s.pos, s.lo, s.hi, s.periodic, csr)
    z = s.pos[2]
    top = np.isclose(z, z.max())
    second = np.isclose(z, z.max() - A / 2)
    inner = (z < z.max() - A) & (z > z.min() + A)
    # 4 of the 12 neighbours are missing; the tie among second-shell candidates decides
    # between a^2 and 1.5 a^2 (tie broken by atom index)
    assert np.all(np.isclose(c[top], A * A) | np.isclose(c[top], 1.5 * A * A))
    assert np.max(np.abs(c[second])) < 1e-20
    assert np.max(np.abs(c[inner])) < 1e-20


def test_csp_too_few_neighbours_is_infinite():
    pos = np.array([[0.0, 2.5, 0.0], [0.0, 0.0, 2.5], [0.0, 0.0, 0.0]])
    s = synth.System(pos, np.full(3, -50.0), np.full(3, 50.0), (0, 0, 0))
    csr = geometry.neighbor_csr(s.pos, s.lo, s.hi, s.periodic, 5.5)
    c = precision.csp(s.pos, s.lo, s.hi, s.periodic, csr)
    assert np.all(np.isinf(c))
    w0 = precision.w0_from_csp(c, 2.5, 3.0, 1)
    assert np.all(w0 == 1.0)


@pytest.mark.parametrize("kind", [0, 1])
def test_switch_limits(kind):
    c = np.array([0.0, 2.5, 2.75, 3.0, 10.0, np.inf])
    w0 = precision.w0_from_csp(c, 2.5, 3.0, kind)
    assert w0[0] == 0.0 and w0[1] == 0.0 and w0[3] == 1.0 and w0[4] == 1.0 and w0[5] == 1.0
    if kind == 0:
        assert w0[2] == 0.5
    else:
        assert w0[2] == 1.0 - 0.20703125


def test_spreading_single_source_closed_form():
    s = _perfect(10)  # L = 36.15 A > 2 * 12 A
    w0 = np.zeros(s.n)
    src = int(np.argmin(np.abs(s.pos - 18.075).sum(0)))
    w0[src] = 1.0
    w = precision.spread(s.pos, s.lo, s.hi, s.periodic, w0, 4.0, 12.0)
    d = s.pos - s.pos[:, [src]]
    r = np.sqrt((d * d).sum(0))
    x = (r - 4.0) / 8.0
    expect = np.where(r < 12.0, np.where(x < 0, 1.0, np.where(x > 1, 0.0,
                      1 - 1.875 * x + 1.25 * x ** 3 - 0.375 * x ** 5)), 0.0)
    assert np.allclose(w, expect, rtol=0, atol=1e-15)
    # the paper counts 626 atoms within r_hi = 12 A of an atom at 0 K; with the source
    # itself 627 atoms receive a non-zero weight
    assert int((w > 0).sum()) == 627
    assert np.all(w[r <= 4.0] == 1.0)


def test_spreading_takes_maximum_and_respects_frozen():
    s = _perfect(8)
    w0 = np.zeros(s.n)
    w0[[0, 500]] = [0.3, 0.8]
    frozen = np.zeros(s.n, np.uint8)
    frozen[1] = 1
    w = precision.spread(s.pos, s.lo, s.hi, s.periodic, w0, 4.0, 12.0, frozen)
    assert w[1] == 0.0
    assert w[0] >= 0.3 and w[500] == 0.8
    # brute force of the definition for a few atoms
    box = s.box
    for i in (2, 77, 1200):
        vals = [w0[i]]
        for j in (0, 500):
            d = s.pos[:, i] - s.pos[:, j]
            d -= box * np.round(d / box)
            r = np.sqrt((d * d).sum())
            if r < 12.0:
                vals.append(w0[j] * precision.f_cut((r - 4.0) / 8.0))
        assert w[i] == pytest.approx(max(vals), abs=1e-15)


def test_precision_cfg0_statistics():
    s = configs.cfg0()
    csr = geometry.neighbor_csr(s.pos, s.lo, s.hi, s.periodic, 5.5)
    pr = precision.compute_precision(s, synth.precision_cfg0(), csr)
    assert s.n == 860
    assert np.array_equal(pr["mask"], (pr["w"] > 0).astype(np.uint8))
    assert np.array_equal(pr["active"], np.nonzero(pr["w"] > 0)[0])
    # no spreading for the plain workload: w == w0
    assert np.array_equal(pr["w"], pr["w0"])


def test_extra_weight_before_or_after_spreading():
    """An additional detection weight joins the CSP weight before the spreading (its
    detections spread like CSP ones) or, with extra_local, after it (only the atom itself)."""
    import dataclasses
    s = configs.cfg0_static()
    p = synth.precision_static()
    csr = geometry.neighbor_csr(s.pos, s.lo, s.hi, s.periodic, 5.5)
    base = precision.compute_precision(s, p, csr)
    k = int(np.nonzero(base["w"] == 0.0)[0][0])  # an atom far from every vacancy
    extra = np.zeros(s.n)
    extra[k] = 1.0
    spread_in = precision.compute_precision(s, p, csr, w0_extra=extra)
    local = precision.compute_precision(s, dataclasses.replace(p, extra_local=True), csr, w0_extra=extra)
    assert spread_in["w"][k] == 1.0 and local["w"][k] == 1.0
    grown = np.nonzero((spread_in["w"] > 0) & (base["w"] == 0))[0]
    assert grown.size > 20 and k in grown  # k and its undetected neighbours within r_hi
    assert np.array_equal(np.nonzero((local["w"] > 0) & (base["w"] == 0))[0], [k])
    assert np.array_equal(local["w0"], base["w0"])
    # both keep everything the CSP criterion detects
    assert np.all(spread_in["w"] >= base["w"]) and np.all(local["w"] >= base["w"])

"""Parameters of the synthetic potentials and of the precision criterion (inputs only).

The EAM amplitudes below are chosen so that the perfect FCC lattice at
``a = 3.615`` Angstrom is stress-free; that property is checked by the oracle tests,
not computed here.  The random ACE parameters are plain normal draws in a fixed order
(radial mixing ``W``, then ``c1``, then ``c2``).
"""

from __future__ import annotations

import dataclasses

import numpy as np

from .systems import A_CU


@dataclasses.dataclass(frozen=True)
class EamParams:
    """Closed-form EAM: phi(r)=A exp(-alpha(r-r0)) psi((r-rc)/h),
    rho(r)=exp(-beta(r-r0)) psi((r-rc)/h), F(rho)=-sqrt(rho)."""

    A: float
    alpha: float
    beta: float
    r0: float
    rc: float = 5.0
    h: float = 0.5


@dataclasses.dataclass(frozen=True)
class Eam2Params:
    """The paper's EAM2 copper potential (Appendix E): pair potential Phi of two Morse-like
    terms, a constant delta and three short-range repulsions S_n; density zeta of a
    Gaussian and an exponential term; embedding xi piecewise around xi(1) = xi0, shifted
    by f0 (the fit's energy offset, Sec. III B); taper psi((r - rc)/h)."""

    E1: float
    E2: float
    delta: float
    alpha1: float
    alpha2: float
    r01: float
    r02: float
    S: tuple
    rs: tuple
    a: float
    beta1: float
    beta2: float
    r03: float
    r04: float
    xi0: float
    xi2: float
    q: tuple
    Q1: float
    Q2: float
    f0: float
    rc: float
    h: float


def eam2_original() -> Eam2Params:
    """Appendix E, Table III, column 'Value original' (EAM2 of Mishin et al.)."""
    return Eam2Params(E1=2.01458e+02, E2=6.59288e-03, delta=8.62250e-03, alpha1=2.97758e+00, alpha2=1.54927e+00,
                      r01=8.35910e-01, r02=4.46867e+00, S=(4.0, 40.0, 1150.0), rs=(2.24, 1.80, 1.20),
                      a=3.80362e+00, beta1=1.73940e-01, beta2=5.35661e+02, r03=-2.19885e+00, r04=-2.61984e+02,
                      xi0=-2.30000e+00, xi2=1.40000e+00, q=(-1.30000e+00, -9.00000e-01, 1.80000e+00, 3.00000e+00),
                      Q1=4.00000e-01, Q2=3.00000e-01, f0=0.0, rc=5.50679e+00, h=5.00370e-01)


def eam2_fit300k() -> Eam2Params:
    """Appendix E, Table III, column 'Value fit 300K' (the paper's refit, F_0^Fit included)."""
    return Eam2Params(E1=2.01486e+02, E2=6.44057e-03, delta=2.18016e-02, alpha1=2.96972e+00, alpha2=1.55510e+00,
                      r01=8.36347e-01, r02=4.46690e+00, S=(4.0, 40.0, 1150.0), rs=(2.24, 1.80, 1.20),
                      a=3.80541e+00, beta1=1.66589e-01, beta2=5.35661e+02, r03=-2.19834e+00, r04=-2.61984e+02,
                      xi0=-2.30089e+00, xi2=1.39912e+00, q=(-1.29894e+00, -8.99672e-01, 1.79940e+00, 2.99944e+00),
                      Q1=3.99178e-01, Q2=3.00455e-01, f0=-1.50036e-01, rc=5.50679e+00, h=5.00370e-01)


@dataclasses.dataclass(frozen=True)
class AceParams:
    """Synthetic ACE: Chebyshev radial basis of ``n_max`` functions mixed by ``W``
    (shape ``[l_max+1, n_max, n_max]``), real spherical harmonics up to ``l_max``,
    coefficient vectors ``c1``/``c2`` over the product basis, optional EAM anchor."""

    n_max: int
    l_max: int
    W: np.ndarray
    c1: np.ndarray
    c2: np.ndarray
    rc: float = 5.0
    h: float = 0.5
    s_a: float = 6.0
    eps: float = 0.1
    anchor: EamParams | None = None


@dataclasses.dataclass(frozen=True)
class PrecisionParams:
    """Detection and switching parameters.

    ``switch_kind`` 0: w0 = clamp((CSP-lo)/(hi-lo), 0, 1); 1: w0 = 1 - f_cut((CSP-lo)/(hi-lo)).
    ``r_hi`` = 0 disables spreading.  ``n_nn`` nearest neighbours (``+ n_buffer``) enter
    the centro-symmetry parameter; neighbours are taken within ``r_cut``.  ``extra_local``:
    an additional detection weight (the learned criterion's) joins after the spreading.
    """

    csp_lo: float
    csp_hi: float
    switch_kind: int
    r_lo: float = 0.0
    r_hi: float = 0.0
    n_nn: int = 12
    n_buffer: int = 0
    r_cut: float = 5.0
    extra_local: bool = False


def eam_cu_like(a: float = A_CU) -> EamParams:
    """The fast potential: alpha 4.3/A, beta 1.8/A, r0 = a/sqrt(2), stress-free at ``a``."""
    return EamParams(A=0.1464436514321396, alpha=4.3, beta=1.8, r0=a / np.sqrt(2.0))


def eam_anchor(a: float = A_CU) -> EamParams:
    """The EAM-like part folded into the anchored ACE (alpha 4.4, beta 1.75, stress-free)."""
    return EamParams(A=0.14169266975963063, alpha=4.4, beta=1.75, r0=a / np.sqrt(2.0))


def eam_label_anchor(a: float = A_CU) -> EamParams:
    """EAM part of the label potential: one tenth of the way from the fast potential to
    ``eam_anchor`` (alpha 4.31, beta 1.795), amplitude again chosen stress-free."""
    return EamParams(A=0.14595440108128369, alpha=4.31, beta=1.795, r0=a / np.sqrt(2.0))


def ace_random(n_max: int, l_max: int, n_basis: int, seed: int,
               anchored: bool = False, coef_std: float = 0.01, anchor: EamParams | None = None) -> AceParams:
    """Random-initialised ACE parameters.

    Draw order from ``default_rng(seed)``: W ~ N(0, 1/n_max) of shape
    ``[l_max+1, n_max, n_max]`` (index ``[l, n, k]``), then ``c1`` and ``c2`` ~ N(0, coef_std)
    of length ``n_basis`` (the size of the product basis, supplied by the caller).
    """
    rng = np.random.default_rng(seed)
    W = rng.normal(0.0, 1.0 / np.sqrt(n_max), size=(l_max + 1, n_max, n_max))
    c1 = rng.normal(0.0, coef_std, size=n_basis)
    c2 = rng.normal(0.0, coef_std, size=n_basis)
    if anchored and anchor is None:
        anchor = eam_anchor()
    return AceParams(n_max=n_max, l_max=l_max, W=W, c1=c1, c2=c2, anchor=anchor if anchored else None)


def ace_label_model(n_basis: int, seed: int = 4242, coef_std: float = 1e-4) -> AceParams:
    """Precise potential of the learned-indicator workload (n_max 10, l_max 4): an EAM part
    whose force constants differ slightly from the fast potential's (``eam_label_anchor``)
    plus a small random many-body part.  Both potentials hold the perfect lattice at the
    same spacing, so their forces agree on the lattice and part the more, the further an
    atom's surroundings are displaced, compressed or cut by a surface."""
    return ace_random(10, 4, n_basis, seed, anchored=True, coef_std=coef_std, anchor=eam_label_anchor())


def precision_cfg0() -> PrecisionParams:
    """Linear switch 0.2-0.5 A^2, no spreading."""
    return PrecisionParams(csp_lo=0.2, csp_hi=0.5, switch_kind=0)


def precision_hyb1() -> PrecisionParams:
    """The paper's Hyb1 set (Table IV): CSP 2.5/3.0 A^2, f_cut switch, spreading radii 4/12 A.
    Its time averages (N = 110 samples, minimum step 1/N) are integrator settings."""
    return PrecisionParams(csp_lo=2.5, csp_hi=3.0, switch_kind=1, r_lo=4.0, r_hi=12.0)


def precision_hyb2() -> PrecisionParams:
    """The paper's Hyb2 set (Appendix K): Hyb1 with spreading radii 8/20 A."""
    return PrecisionParams(csp_lo=2.5, csp_hi=3.0, switch_kind=1, r_lo=8.0, r_hi=20.0)


def precision_static() -> PrecisionParams:
    """Hyb1 thresholds with shorter spreading radii 4/8 A (for small periodic boxes)."""
    return PrecisionParams(csp_lo=2.5, csp_hi=3.0, switch_kind=1, r_lo=4.0, r_hi=8.0)

"""Atomic cluster expansion energy (oracle), Sec. III A.

The paper fixes only the outer form E_i = phi_i^(1) + sqrt(phi_i^(2)) with
phi_i^(p) = sum_v c_v^(p) B_iv.  The synthetic basis behind it is defined here:

* radial functions   g_k(r) = T_k(2 r / r_c - 1) psi((r - r_c)/h),  k = 0..n_max-1
  (Chebyshev polynomials of the first kind, the same taper psi as the EAM),
  mixed per l:        R_nl(r) = sum_k W[l, n, k] g_k(r)
* real orthonormal spherical harmonics Y_lm (index l*l + l + m)
      m = 0 : N_l0 Q_l0(z)
      m > 0 : sqrt(2) N_lm Q_lm(z) Re((x + i y)^m)
      m < 0 : sqrt(2) N_l|m| Q_l|m|(z) Im((x + i y)^|m|)
  with Q_lm = d^m P_l / dz^m, N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!), unit vector (x,y,z)
* atomic base          A_nlm = (1/s_A) sum_j R_nl(r_ij) Y_lm(r_ij / r_ij)
* product basis, in this order:
      B1_n        = A_n00
      B2_(n1n2l)  = sum_m A_n1lm A_n2lm                       n1 <= n2, l = 0..l_max
      B3_(p1p2p3) = sum_m1m2m3 G(l1 l2 l3; m1 m2 m3) A_p1m1 A_p2m2 A_p3m3
  over (n, l) labels p = n (l_max + 1) + l with p1 <= p2 <= p3, l1 + l2 + l3 even and
  |l1 - l2| <= l3 <= l1 + l2; G is the real Gaunt coefficient (integral of three Y).
* the square root is replaced by F_eps(x) = sign(x) (sqrt(|x| + eps^2) - eps), which
  tends to sqrt for x > 0 as eps -> 0 and is defined for negative arguments.
* optional anchor: E_i^ACE = E_i^rand + E_i^EAM(theta') (an EAM of the same form with
  other parameters), making the synthetic precise potential physical.
"""

from __future__ import annotations

import functools
import math

import numpy as np
import torch

from . import eam as _eam


# ---------------------------------------------------------------- spherical harmonics
@functools.lru_cache(maxsize=None)
def _legendre_derivative_coeffs(l: int, m: int):
    """Power-series coefficients (ascending) of d^m P_l / dz^m."""
    c = np.polynomial.legendre.leg2poly([0.0] * l + [1.0])
    for _ in range(m):
        c = np.polynomial.polynomial.polyder(c)
    return tuple(float(v) for v in np.atleast_1d(c))


def _horner(coeffs, z):
    out = torch.zeros_like(z) + coeffs[-1]
    for c in reversed(coeffs[:-1]):
        out = out * z + c
    return out


def real_sph_harm(u: torch.Tensor, l_max: int) -> torch.Tensor:
    """Y_lm of unit vectors ``u`` [P, 3] -> [P, (l_max+1)^2] (index l*l + l + m)."""
    x, y, z = u[:, 0], u[:, 1], u[:, 2]
    # (x + i y)^m by repeated complex multiplication
    re = [torch.ones_like(x)]
    im = [torch.zeros_like(x)]
    for m in range(1, l_max + 1):
        re.append(re[-1] * x - im[-1] * y)
        im.append(re[-2] * y + im[-1] * x)
    cols = []
    for l in range(l_max + 1):
        for m in range(-l, l + 1):
            am = abs(m)
            norm = math.sqrt((2 * l + 1) / (4.0 * math.pi)
                             * math.factorial(l - am) / math.factorial(l + am))
            q = _horner(_legendre_derivative_coeffs(l, am), z)
            if m == 0:
                cols.append(norm * q)
            elif m > 0:
                cols.append(math.sqrt(2.0) * norm * q * re[am])
            else:
                cols.append(math.sqrt(2.0) * norm * q * im[am])
    return torch.stack(cols, dim=1)


# ------------------------------------------------------------------- Gaunt tensors
@functools.lru_cache(maxsize=None)
def gaunt(l_max: int):
    """Real Gaunt tensors G[(l1,l2,l3)] of shape (2l1+1, 2l2+1, 2l3+1).

    Integral over the sphere of Y_l1m1 Y_l2m2 Y_l3m3 by a product rule that is exact for
    the degree involved: Gauss-Legendre in cos(theta) with ``3 l_max / 2 + 2`` nodes and a
    uniform rule with ``3 l_max + 2`` points in the azimuth.
    """
    nq = 3 * l_max // 2 + 2
    nph = 3 * l_max + 2
    xs, ws = np.polynomial.legendre.leggauss(nq)
    ph = np.arange(nph) * (2.0 * np.pi / nph)
    ct = np.repeat(xs, nph)
    st = np.sqrt(1.0 - ct * ct)
    phv = np.tile(ph, nq)
    wt = np.repeat(ws, nph) * (2.0 * np.pi / nph)
    u = torch.as_tensor(np.stack([st * np.cos(phv), st * np.sin(phv), ct], axis=1))
    Y = real_sph_harm(u, l_max).numpy()
    out = {}
    for l1 in range(l_max + 1):
        for l2 in range(l_max + 1):
            for l3 in range(l_max + 1):
                if (l1 + l2 + l3) % 2 or l3 < abs(l1 - l2) or l3 > l1 + l2:
                    continue
                Y1 = Y[:, l1 * l1:(l1 + 1) ** 2]
                Y2 = Y[:, l2 * l2:(l2 + 1) ** 2]
                Y3 = Y[:, l3 * l3:(l3 + 1) ** 2]
                g = np.einsum("q,qa,qb,qc->abc", wt, Y1, Y2, Y3)
                g[np.abs(g) < 1e-14] = 0.0
                out[(l1, l2, l3)] = g
    return out


# ------------------------------------------------------------------ basis catalogue
@functools.lru_cache(maxsize=None)
def basis_spec(n_max: int, l_max: int):
    """Enumeration of the product basis: list of ("1", n), ("2", n1, n2, l),
    ("3", p1, p2, p3) in the documented order."""
    spec = [("1", n) for n in range(n_max)]
    for n1 in range(n_max):
        for n2 in range(n1, n_max):
            for l in range(l_max + 1):
                spec.append(("2", n1, n2, l))
    P = n_max * (l_max + 1)
    for p1 in range(P):
        for p2 in range(p1, P):
            for p3 in range(p2, P):
                l1, l2, l3 = p1 % (l_max + 1), p2 % (l_max + 1), p3 % (l_max + 1)
                if (l1 + l2 + l3) % 2 or l3 < abs(l1 - l2) or l3 > l1 + l2:
                    continue
                spec.append(("3", p1, p2, p3))
    return tuple(spec)


def num_basis(n_max: int, l_max: int) -> int:
    return len(basis_spec(n_max, l_max))


@functools.lru_cache(maxsize=None)
def _b3_groups(n_max: int, l_max: int):
    """Triples grouped by (l1, l2, l3): {(l1,l2,l3): (columns, n1s, n2s, n3s)}."""
    groups = {}
    for col, s in enumerate(basis_spec(n_max, l_max)):
        if s[0] != "3":
            continue
        p1, p2, p3 = s[1:]
        L = l_max + 1
        key = (p1 % L, p2 % L, p3 % L)
        groups.setdefault(key, ([], [], [], []))
        g = groups[key]
        g[0].append(col)
        g[1].append(p1 // L)
        g[2].append(p2 // L)
        g[3].append(p3 // L)
    return {k: tuple(np.array(v, dtype=np.int64) for v in g) for k, g in groups.items()}


# ------------------------------------------------------------------------- radial
def chebyshev_radial(r: torch.Tensor, n_max: int, rc: float, h: float) -> torch.Tensor:
    """g_k(r) = T_k(2r/r_c - 1) psi((r - r_c)/h), k = 0..n_max-1 -> [P, n_max]."""
    x = 2.0 * r / rc - 1.0
    T = [torch.ones_like(x), x]
    for _ in range(2, n_max):
        T.append(2.0 * x * T[-1] - T[-2])
    taper = _eam.psi((r - rc) / h)
    return torch.stack(T[:n_max], dim=1) * taper[:, None]


def f_eps(x: torch.Tensor, eps: float) -> torch.Tensor:
    e2 = eps * eps
    pos = torch.sqrt(torch.clamp(x, min=0.0) + e2) - eps
    neg = -(torch.sqrt(torch.clamp(-x, min=0.0) + e2) - eps)
    return torch.where(x >= 0.0, pos, neg)


# ------------------------------------------------------------------------- energy
def atomic_base(pos_t, box, periodic, i, j, prm, sites):
    """A_l tensors [n_sites, n_max, 2l+1] for the atoms in ``sites`` (ascending)."""
    sites = np.asarray(sites, dtype=np.int64)
    row = np.full(pos_t.shape[1], -1, dtype=np.int64)
    row[sites] = np.arange(sites.size)
    sel = row[i] >= 0
    i, j = i[sel], j[sel]
    d = _eam.pair_vectors(pos_t, box, periodic, i, j)
    r = torch.sqrt((d * d).sum(dim=0))
    u = (d / r).T
    g = chebyshev_radial(r, prm.n_max, prm.rc, prm.h)  # [P, K]
    Y = real_sph_harm(u, prm.l_max)  # [P, (L+1)^2]
    W = torch.as_tensor(prm.W)
    rows = torch.as_tensor(row[i])
    A = []
    for l in range(prm.l_max + 1):
        R = g @ W[l].T  # [P, n_max]: R_nl = sum_k W[l,n,k] g_k
        Yl = Y[:, l * l:(l + 1) ** 2]
        contrib = (R[:, :, None] * Yl[:, None, :]) / prm.s_a
        A.append(torch.zeros(sites.size, prm.n_max, 2 * l + 1, dtype=torch.float64)
                 .index_add(0, rows, contrib))
    return A


def product_basis(A, n_max: int, l_max: int) -> torch.Tensor:
    """B [n_sites, n_basis] in the documented order."""
    cols = [A[0][:, n, 0] for n in range(n_max)]
    for n1 in range(n_max):
        for n2 in range(n1, n_max):
            for l in range(l_max + 1):
                cols.append((A[l][:, n1, :] * A[l][:, n2, :]).sum(dim=1))
    B12 = torch.stack(cols, dim=1)
    nb = num_basis(n_max, l_max)
    B3 = torch.zeros(B12.shape[0], nb, dtype=torch.float64)
    G = gaunt(l_max)
    parts = []
    for (l1, l2, l3), (colsg, n1s, n2s, n3s) in _b3_groups(n_max, l_max).items():
        g = torch.as_tensor(G[(l1, l2, l3)])
        X1 = A[l1][:, n1s, :]
        X2 = A[l2][:, n2s, :]
        X3 = A[l3][:, n3s, :]
        val = torch.einsum("abc,ita,itb,itc->it", g, X1, X2, X3)
        parts.append((torch.as_tensor(colsg), val))
    idx = torch.cat([c for c, _ in parts])
    vals = torch.cat([v for _, v in parts], dim=1)
    B3 = B3.index_copy(1, idx, vals)
    nb12 = B12.shape[1]
    return torch.cat([B12, B3[:, nb12:]], dim=1)


def site_energies(pos_t, box, periodic, i, j, prm, n: int, sites, c1=None, c2=None,
                  return_parts=False):
    """E_i^ACE for atoms in ``sites``; a length-``n`` tensor (0 outside ``sites``).

    ``c1``/``c2`` may be given as tensors (e.g. with requires_grad) to differentiate
    with respect to the coefficients.
    """
    sites = np.asarray(sites, dtype=np.int64)
    if sites.size == 0:
        e = torch.zeros(n, dtype=torch.float64) + 0.0 * pos_t.sum()
        return (e, None) if return_parts else e
    A = atomic_base(pos_t, box, periodic, i, j, prm, sites)
    B = product_basis(A, prm.n_max, prm.l_max)
    c1 = torch.as_tensor(prm.c1) if c1 is None else c1
    c2 = torch.as_tensor(prm.c2) if c2 is None else c2
    phi1 = B @ c1
    phi2 = B @ c2
    e_s = phi1 + f_eps(phi2, prm.eps)
    e = torch.zeros(n, dtype=torch.float64).index_copy(0, torch.as_tensor(sites), e_s)
    if prm.anchor is not None:
        e = e + _eam.site_energies(pos_t, box, periodic, i, j, prm.anchor, n, sites=sites)
    if return_parts:
        return e, dict(A=A, B=B, phi1=phi1, phi2=phi2)
    return e

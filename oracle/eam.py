"""Embedded-atom model (oracle), eq. energy_eam of Sec. III B.

E_i = F(rho_i) + 1/2 sum_j phi(r_ij),  rho_i = sum_j rho(r_ij), over j != i with r_ij < r_c.

Functional form of the synthetic fast potential (closed form; the taper psi is the one
the paper uses for its EAM2 pair and density functions, Appendix E):
    psi(x)   = x^4 / (1 + x^4) for x < 0, else 0
    phi(r)   = A exp(-alpha (r - r0)) psi((r - r_c)/h)
    rho(r)   = exp(-beta (r - r0)) psi((r - r_c)/h)
    F(rho)   = -sqrt(rho)   (F = 0 at rho = 0)

The paper's own EAM2 copper potential (Appendix E; parameter objects with the field
``xi0``) is the second form:
    Phi(r)  = (E1 M(r, r01, alpha1) + E2 M(r, r02, alpha2) + delta) psi((r - rc)/h)
              - sum_n Theta(rs_n - r) S_n (rs_n - r)^4,
    M(r, r0, alpha) = exp(-2 alpha (r - r0)) - 2 exp(-alpha (r - r0)),
    zeta(r) = (a exp(-beta1 (r - r03)^2) + exp(-beta2 (r - r04))) psi((r - rc)/h),
    xi(x)   = xi0 + xi2 (x-1)^2 / 2 + sum_n q_n (x-1)^(n+2)                        for x <= 1,
              (xi0 + xi2 (x-1)^2 / 2 + q1 (x-1)^3 + Q1 (x-1)^4) / (1 + Q2 (x-1)^3)   otherwise,
    plus the energy offset f0 of the paper's refit (Sec. III B); Theta(0) = 1.

Written with float64 torch tensors so that forces can be taken as the negative
gradient of the weighted energy by autograd.
"""

from __future__ import annotations

import numpy as np
import torch


def psi(x: torch.Tensor) -> torch.Tensor:
    x4 = x ** 4
    return torch.where(x < 0.0, x4 / (1.0 + x4), torch.zeros_like(x))


def _is_eam2(p) -> bool:
    return hasattr(p, "xi0")


def _morse(r, r0, alpha):
    """M(r, r0, alpha) of Appendix E: exp(-2 alpha (r - r0)) - 2 exp(-alpha (r - r0))."""
    return torch.exp(-2.0 * alpha * (r - r0)) - 2.0 * torch.exp(-alpha * (r - r0))


def pair_phi(r: torch.Tensor, p) -> torch.Tensor:
    if _is_eam2(p):
        # Appendix E: (E1 M(r, r01, a1) + E2 M(r, r02, a2) + delta) psi((r - rc)/h)
        #             - sum_n Theta(rs_n - r) S_n (rs_n - r)^4
        v = (p.E1 * _morse(r, p.r01, p.alpha1) + p.E2 * _morse(r, p.r02, p.alpha2) + p.delta) * psi((r - p.rc) / p.h)
        for S, rs in zip(p.S, p.rs):
            v = v - torch.where(rs - r >= 0.0, S * (rs - r) ** 4, torch.zeros_like(r))
        return v
    return p.A * torch.exp(-p.alpha * (r - p.r0)) * psi((r - p.rc) / p.h)


def pair_rho(r: torch.Tensor, p) -> torch.Tensor:
    if _is_eam2(p):
        # Appendix E: (a exp(-beta1 (r - r03)^2) + exp(-beta2 (r - r04))) psi((r - rc)/h)
        return (p.a * torch.exp(-p.beta1 * (r - p.r03) ** 2) + torch.exp(-p.beta2 * (r - p.r04))) * psi((r - p.rc) / p.h)
    return torch.exp(-p.beta * (r - p.r0)) * psi((r - p.rc) / p.h)


def embed(rho: torch.Tensor, p=None) -> torch.Tensor:
    if p is not None and _is_eam2(p):
        # Appendix E eq. mishin_embedding_function, plus the fit's offset (Sec. III B)
        x = rho - 1.0
        low = p.xi0 + 0.5 * p.xi2 * x ** 2
        for k, qn in enumerate(p.q):
            low = low + qn * x ** (k + 3)
        high = (p.xi0 + 0.5 * p.xi2 * x ** 2 + p.q[0] * x ** 3 + p.Q1 * x ** 4) / (1.0 + p.Q2 * x ** 3)
        return torch.where(rho <= 1.0, low, high) + p.f0
    safe = torch.where(rho > 0.0, rho, torch.ones_like(rho))
    return torch.where(rho > 0.0, -torch.sqrt(safe), torch.zeros_like(rho))


def pair_vectors(pos_t: torch.Tensor, box, periodic, i: np.ndarray, j: np.ndarray):
    """Differentiable minimum-image vectors x_j - x_i (image shifts taken as constants)."""
    d = pos_t[:, j] - pos_t[:, i]
    with torch.no_grad():
        shift = torch.zeros_like(d)
        for k in range(3):
            if periodic[k]:
                L = float(box[k])
                dk = d[k]
                shift[k] = torch.where(dk >= 0.5 * L, torch.full_like(dk, L),
                                       torch.where(dk < -0.5 * L, torch.full_like(dk, -L),
                                                   torch.zeros_like(dk)))
    return d - shift


def site_energies(pos_t, box, periodic, i, j, p, n: int, sites=None) -> torch.Tensor:
    """E_i of eq. energy_eam for all ``n`` atoms (pairs (i, j) already inside r_c).

    ``sites`` (optional index array) restricts the pairs to centres in that set; the
    returned vector still has length ``n`` (zeros elsewhere).
    """
    if sites is not None:
        sel = np.isin(i, sites)
        i, j = i[sel], j[sel]
    d = pair_vectors(pos_t, box, periodic, i, j)
    r = torch.sqrt((d * d).sum(dim=0))
    it = torch.as_tensor(i)
    rho = torch.zeros(n, dtype=torch.float64).index_add(0, it, pair_rho(r, p))
    pair = torch.zeros(n, dtype=torch.float64).index_add(0, it, pair_phi(r, p))
    e = embed(rho, p) + 0.5 * pair
    if sites is not None:
        m = torch.zeros(n, dtype=torch.bool)
        m[torch.as_tensor(sites)] = True
        e = torch.where(m, e, torch.zeros_like(e))
    return e


def density(pos, box, periodic, i, j, p, n: int) -> np.ndarray:
    """rho_i = sum_j rho(r_ij) (float64 numpy)."""
    with torch.no_grad():
        d = pair_vectors(torch.as_tensor(pos), box, periodic, i, j)
        r = torch.sqrt((d * d).sum(dim=0))
        rho = torch.zeros(n, dtype=torch.float64).index_add(0, torch.as_tensor(i), pair_rho(r, p))
    return rho.numpy()

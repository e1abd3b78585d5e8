"""Nondimensional compressible Navier-Stokes fluxes (paper, Appendix B).

State q = (rho, rho u, rho v, rho w, rho E) on the last axis.  Every function
accepts float64 or complex128 tensors so that pointwise flux Jacobians can be
taken by complex-step differentiation (exact to rounding); |.| and max() are
written so that they propagate the imaginary part of the branch they select.

Readings of the appendix used here (each a correction of a printing slip):
  * thermal conductivity kappa = mu / ((gamma-1) Pr Ma^2) with p_inf = 1/(gamma Ma^2)
    and T = gamma Ma^2 p / rho, so that kappa grad T = (mu gamma / Pr) grad e;
  * Stokes stress tau = mu (grad v + grad v^T) - (2/3) mu (div v) I;
  * Sutherland's law with T_suth / T_inf = 110.4 / 288.15.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

GAMMA = 1.4
PRANDTL = 0.72
SUTHERLAND_RATIO = 110.4 / 288.15


@dataclass(frozen=True)
class FlowParams:
    mach: float
    reynolds: float
    gamma: float = GAMMA
    prandtl: float = PRANDTL
    suth: float = SUTHERLAND_RATIO


def _cabs(z: torch.Tensor) -> torch.Tensor:
    """|z| that keeps the complex-step derivative: z * sign(Re z)."""
    if z.is_complex():
        return z * torch.sign(z.real)
    return torch.abs(z)


def _cmax(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """max(a, b) comparing real parts; ties go to a."""
    if a.is_complex():
        return torch.where(a.real >= b.real, a, b)
    return torch.where(a >= b, a, b)


def primitives(q: torch.Tensor, prm: FlowParams):
    rho = q[..., 0]
    u = q[..., 1] / rho
    v = q[..., 2] / rho
    w = q[..., 3] / rho
    p = (prm.gamma - 1.0) * (q[..., 4] - 0.5 * rho * (u * u + v * v + w * w))
    return rho, u, v, w, p


def flux_adv(q: torch.Tensor, d: int, prm: FlowParams) -> torch.Tensor:
    """Advective flux f^a_d(q) in Cartesian direction d (0, 1, 2)."""
    rho, u, v, w, p = primitives(q, prm)
    vel = (u, v, w)[d]
    out = [q[..., 0] * vel, q[..., 1] * vel, q[..., 2] * vel, q[..., 3] * vel,
           vel * (q[..., 4] + p)]
    out[1 + d] = out[1 + d] + p
    return torch.stack(out, dim=-1)


def viscosity(t: torch.Tensor, prm: FlowParams) -> torch.Tensor:
    """Sutherland's law in nondimensional form (T_inf = 1)."""
    return (1.0 + prm.suth) / (t + prm.suth) * t * torch.sqrt(t)


def viscous_stress(q: torch.Tensor, g: tuple[torch.Tensor, torch.Tensor, torch.Tensor], prm: FlowParams):
    """Velocities, the viscous stress tensor tau[i][k] and the heat flux
    (mu gamma / Pr) de/dx_k at every node; g[k] holds d q / d x_k (conserved
    variables).  Shared by the viscous fluxes of all three directions."""
    rho, u, v, w, p = primitives(q, prm)
    vel = (u, v, w)
    temp = prm.gamma * prm.mach ** 2 * p / rho
    mu = viscosity(temp, prm)
    # velocity gradients dv_i/dx_k = (d(rho v_i)/dx_k - v_i d rho/dx_k) / rho
    dv = [[(g[k][..., 1 + i] - vel[i] * g[k][..., 0]) / rho for k in range(3)] for i in range(3)]
    # specific internal energy gradient: e = E - |v|^2 / 2 with E = rho E / rho
    ee = q[..., 4] / rho
    de = [(g[k][..., 4] - ee * g[k][..., 0]) / rho
          - (vel[0] * dv[0][k] + vel[1] * dv[1][k] + vel[2] * dv[2][k]) for k in range(3)]
    div = dv[0][0] + dv[1][1] + dv[2][2]
    tau = [[None] * 3 for _ in range(3)]
    for d in range(3):
        for i in range(3):
            t = mu * (dv[i][d] + dv[d][i])
            if i == d:
                t = t - (2.0 / 3.0) * mu * div
            tau[i][d] = t
    heat = [mu * prm.gamma / prm.prandtl * de[d] for d in range(3)]
    return vel, tau, heat, rho


def viscous_flux_of(stress, d: int, prm: FlowParams) -> torch.Tensor:
    """f^nu_d from the output of viscous_stress."""
    vel, tau, heat, rho = stress
    tau_d = [tau[i][d] for i in range(3)]
    energy = vel[0] * tau_d[0] + vel[1] * tau_d[1] + vel[2] * tau_d[2] + heat[d]
    inv_re = 1.0 / prm.reynolds
    zero = torch.zeros_like(rho)
    return torch.stack([zero, tau_d[0] * inv_re, tau_d[1] * inv_re, tau_d[2] * inv_re,
                        energy * inv_re], dim=-1)


def flux_visc(q: torch.Tensor, g: tuple[torch.Tensor, torch.Tensor, torch.Tensor],
              d: int, prm: FlowParams) -> torch.Tensor:
    """Viscous flux f^nu_d(q, grad q); g[k] holds d q / d x_k (conserved variables)."""
    return viscous_flux_of(viscous_stress(q, g, prm), d, prm)


def wave_speed(q: torch.Tensor, d: int, prm: FlowParams) -> torch.Tensor:
    """|v_d| + c at a node."""
    rho, u, v, w, p = primitives(q, prm)
    c = torch.sqrt(prm.gamma * p / rho)
    return _cabs((u, v, w)[d]) + c


def llf_flux(ql: torch.Tensor, qr: torch.Tensor, d: int, prm: FlowParams) -> torch.Tensor:
    """Local Lax-Friedrichs (Rusanov) flux through a face with normal +e_d.

    ql is the state on the side the normal points away from, qr the other side;
    lambda = max(|v_d| + c) over the two states at this face node.
    """
    lam = _cmax(wave_speed(ql, d, prm), wave_speed(qr, d, prm))
    return 0.5 * (flux_adv(ql, d, prm) + flux_adv(qr, d, prm)) - 0.5 * lam[..., None] * (qr - ql)

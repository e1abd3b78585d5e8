"""GL-DGSEM residual H(Q) for the compressible Navier-Stokes equations on a
periodic Cartesian hexahedral mesh (paper, Section 2.1 and Appendix C).

Discretization (paper, eq. DGSEMsystem / DGSEMsystem2):
  J_j w_j dq_j/dt - int^N f . grad(phi_j) + oint^N f_hat phi_j = 0
  J_j w_j g_j     = -int^N q grad(phi_j) + oint^N phi_j q_hat n
with f = f^a(q) - f^nu(q, g), the local Lax-Friedrichs advective flux and the
Bassi-Rebay 1 viscous flux f_hat^nu = {{f^nu(q, g)}}.n, q_hat = {{q}}.

Array layout: a field on the mesh is a tensor of shape
  [Kz, Ky, Kx, P, P, P, 5]   (element z, y, x; node k, j, i; variable)
with P = N + 1.  Flattening gives the natural order used everywhere in this
project: element e = ex + K ey + K^2 ez, node n = i + P j + P^2 k, variable v,
DOF = (e P^3 + n) * 5 + v.

Direction d (0 = x, 1 = y, 2 = z) runs along element axis 2 - d and node axis
5 - d.  The mapping is x = x_e + (h/2)(xi + 1), so J = (h/2)^3 and
d xi / d x = 2 / h.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from . import gl
from .physics import FlowParams, flux_adv, flux_visc, llf_flux


@dataclass(frozen=True)
class Mesh:
    k_elem: int          # elements per direction
    order: int           # polynomial order N
    length: float = 2.0 * math.pi

    @property
    def p(self) -> int:
        return self.order + 1

    @property
    def h(self) -> float:
        return self.length / self.k_elem

    @property
    def jac(self) -> float:
        return (self.h / 2.0) ** 3

    @property
    def scale(self) -> float:
        return 2.0 / self.h

    @property
    def n_elem(self) -> int:
        return self.k_elem ** 3

    @property
    def n_dof(self) -> int:
        return self.n_elem * self.p ** 3 * 5

    def shape(self) -> tuple[int, ...]:
        k, p = self.k_elem, self.p
        return (k, k, k, p, p, p, 5)


def elem_axis(d: int) -> int:
    return 2 - d


def node_axis(d: int) -> int:
    return 5 - d


def operators(mesh: Mesh, device, dtype=torch.float64):
    x, w = gl.gl_nodes_weights(mesh.order)
    d = gl.derivative_matrix(mesh.order)
    t = lambda a: torch.tensor(a, dtype=dtype, device=device)
    return t(x), t(w), t(d)


def node_coordinates(mesh: Mesh) -> np.ndarray:
    """Physical coordinates [Kz, Ky, Kx, P, P, P, 3] (x, y, z) of every node."""
    xi, _ = gl.gl_nodes_weights(mesh.order)
    k, p, h = mesh.k_elem, mesh.p, mesh.h
    e = np.arange(k)
    line = e[:, None] * h + 0.5 * h * (xi[None, :] + 1.0)          # [K, P]
    xs = line[None, None, :, None, None, :]                          # ex, i
    ys = line[None, :, None, None, :, None]                          # ey, j
    zs = line[:, None, None, :, None, None]                          # ez, k
    full = np.broadcast_shapes(xs.shape, ys.shape, zs.shape)
    return np.stack([np.broadcast_to(xs, full), np.broadcast_to(ys, full),
                     np.broadcast_to(zs, full)], axis=-1)


def curved_node_coordinates(mesh: Mesh, amplitude: float = 0.05, kind: str = "sine") -> np.ndarray:
    """Nodes of a smoothly perturbed periodic mesh, [Kz, Ky, Kx, P, P, P, 3].

    kind "sine": every coordinate of the Cartesian node position xi (in
    [0, L)^3) is shifted by amplitude * L * sin(t xi_x) sin(t xi_y) sin(t xi_z),
    t = 2 pi / L (the same shift for x, y and z).  kind "skew": coordinate d is
    shifted by amplitude * L * sin(t xi_x + a_d) sin(t xi_y + 2 a_d)
    sin(t xi_z + 3 a_d), a_d = 0.7 (d + 1), a different shift per coordinate.
    Both shifts are L-periodic, so the mesh stays periodic."""
    xi = node_coordinates(mesh)
    t = 2.0 * np.pi / mesh.length
    if kind == "sine":
        s = np.sin(t * xi[..., 0]) * np.sin(t * xi[..., 1]) * np.sin(t * xi[..., 2])
        return xi + (amplitude * mesh.length * s)[..., None]
    if kind != "skew":
        raise ValueError(kind)
    out = xi.copy()
    for d in range(3):
        a = 0.7 * (d + 1)
        out[..., d] += amplitude * mesh.length * (np.sin(t * xi[..., 0] + a) * np.sin(t * xi[..., 1] + 2 * a)
                                                  * np.sin(t * xi[..., 2] + 3 * a))
    return out


def mass_diagonal(mesh: Mesh) -> np.ndarray:
    """Diagonal of M per node, J w_i w_j w_k, shape [Kz, Ky, Kx, P, P, P]."""
    _, w = gl.gl_nodes_weights(mesh.order)
    k = mesh.k_elem
    m = mesh.jac * w[:, None, None] * w[None, :, None] * w[None, None, :]
    return np.broadcast_to(m, (k, k, k) + m.shape).copy()


def taylor_green_state(mesh: Mesh, prm: FlowParams, seed: int, amplitude: float = 1e-3,
                       coords: np.ndarray | None = None) -> np.ndarray:
    """Taylor-Green-like conserved state with a seeded perturbation.

    Velocity in units of the reference speed: u = sin x cos y cos z,
    v = -cos x sin y cos z, w = 0, rho = 1,
    p = 1/(gamma Ma^2) + (cos 2x + cos 2y)(cos 2z + 2)/16.
    Perturbation: rho *= 1 + a xi_1, u_k += a xi_{k+1}, p *= 1 + a xi_5 with
    xi ~ U(-1, 1) i.i.d. per node from numpy's PCG64 seeded generator.
    coords: the node positions to evaluate at (default: the Cartesian nodes).
    """
    xyz = node_coordinates(mesh) if coords is None else coords
    x, y, z = xyz[..., 0], xyz[..., 1], xyz[..., 2]
    rho = np.ones_like(x)
    u = np.sin(x) * np.cos(y) * np.cos(z)
    v = -np.cos(x) * np.sin(y) * np.cos(z)
    w = np.zeros_like(x)
    p = 1.0 / (prm.gamma * prm.mach ** 2) + (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0) / 16.0
    rng = np.random.default_rng(seed)
    xi = rng.uniform(-1.0, 1.0, size=x.shape + (5,))
    rho = rho * (1.0 + amplitude * xi[..., 0])
    u = u + amplitude * xi[..., 1]
    v = v + amplitude * xi[..., 2]
    w = w + amplitude * xi[..., 3]
    p = p * (1.0 + amplitude * xi[..., 4])
    e_tot = p / (prm.gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return np.stack([rho, rho * u, rho * v, rho * w, e_tot], axis=-1)


def uniform_state(mesh: Mesh, prm: FlowParams, velocity=(0.3, -0.2, 0.1)) -> np.ndarray:
    rho = 1.0
    u, v, w = velocity
    p = 1.0 / (prm.gamma * prm.mach ** 2)
    e_tot = p / (prm.gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    q = np.array([rho, rho * u, rho * v, rho * w, e_tot])
    return np.broadcast_to(q, mesh.shape()).copy()


def _along(a: torch.Tensor, d: int) -> torch.Tensor:
    """Move the node axis of direction d next to the variable axis: [..., P, 5]."""
    return a.movedim(node_axis(d), -2)


def _back(a: torch.Tensor, d: int) -> torch.Tensor:
    return a.movedim(-2, node_axis(d))


def lifted_gradient(q: torch.Tensor, mesh: Mesh):
    """BR1 lifted gradient g_d, d = x, y, z (strong form of eq. DGSEMsystem2:2).

    g_d = s [ D q + (1/w_N) delta_{l,N} (q_hat_R - q_N) - (1/w_0) delta_{l,0} (q_hat_L - q_0) ]
    with q_hat = (q+ + q-)/2 and s = 2/h.
    """
    _, w, dm = operators(mesh, q.device, torch.float64)
    dm = dm.to(q.dtype)
    n = mesh.order
    s = mesh.scale
    out = []
    for d in range(3):
        qm = _along(q, d)
        g = dm @ qm
        q_first, q_last = qm[..., 0, :], qm[..., n, :]
        q_right = torch.roll(qm, -1, dims=elem_axis(d))[..., 0, :]
        q_left = torch.roll(qm, 1, dims=elem_axis(d))[..., n, :]
        g = g.clone()
        g[..., n, :] += (0.5 / float(w[n])) * (q_right - q_last)
        g[..., 0, :] -= (0.5 / float(w[0])) * (q_left - q_first)
        out.append(_back(s * g, d))
    return tuple(out)


def lifted_gradient_weak(q: torch.Tensor, mesh: Mesh):
    """Weak form of the same lifting: g = s (1/w_l)[-sum_a w_a D[a,l] q_a + delta_{lN} q_hat_R - delta_{l0} q_hat_L]."""
    _, w, dm = operators(mesh, q.device, torch.float64)
    n = mesh.order
    s = mesh.scale
    vw = (-(dm.T) * w[None, :]).to(q.dtype)
    winv = (1.0 / w).to(q.dtype)
    out = []
    for d in range(3):
        qm = _along(q, d)
        g = vw @ qm
        q_right = torch.roll(qm, -1, dims=elem_axis(d))[..., 0, :]
        q_left = torch.roll(qm, 1, dims=elem_axis(d))[..., n, :]
        g = g.clone()
        g[..., n, :] += 0.5 * (qm[..., n, :] + q_right)
        g[..., 0, :] -= 0.5 * (qm[..., 0, :] + q_left)
        out.append(_back(s * winv[:, None] * g, d))
    return tuple(out)


def face_flux(ql, qr, gl_, gr_, d: int, prm: FlowParams):
    """Total numerical flux through a +e_d face: LLF advective minus BR1 viscous."""
    return (llf_flux(ql, qr, d, prm)
            - 0.5 * (flux_visc(ql, gl_, d, prm) + flux_visc(qr, gr_, d, prm)))


def residual(q: torch.Tensor, mesh: Mesh, prm: FlowParams, form: str = "weak") -> torch.Tensor:
    """H(Q) of eq. DiscretNS (mass-weighted), same layout as q.

    Weak form per direction d, with l the line index along d:
      H_d = J s w_t1 w_t2 [ -sum_a w_a D[a,l] F_d(a) + delta_{lN} Fhat_R - delta_{l0} Fhat_L ]
    Strong form (identical by summation-by-parts):
      H_d = J s w_t1 w_t2 w_l [ sum_a D[l,a] F_d(a) + (1/w_l)(delta_{lN}(Fhat_R - F_N) - delta_{l0}(Fhat_L - F_0)) ]
    """
    _, w, dm = operators(mesh, q.device, torch.float64)
    n = mesh.order
    g = lifted_gradient(q, mesh)
    m_diag = torch.tensor(mass_diagonal(mesh), device=q.device, dtype=torch.float64)
    total = torch.zeros_like(q)
    winv = (1.0 / w).to(q.dtype)
    for d in range(3):
        f = flux_adv(q, d, prm) - flux_visc(q, g, d, prm)
        fm = _along(f, d)
        qm = _along(q, d)
        gm = tuple(_along(gk, d) for gk in g)
        roll_r = lambda a: torch.roll(a, -1, dims=elem_axis(d))
        ql = qm[..., n, :]
        qr = roll_r(qm)[..., 0, :]
        gl_ = tuple(gk[..., n, :] for gk in gm)
        gr_ = tuple(roll_r(gk)[..., 0, :] for gk in gm)
        fhat_r = face_flux(ql, qr, gl_, gr_, d, prm)
        fhat_l = torch.roll(fhat_r, 1, dims=elem_axis(d))
        if form == "weak":
            vw = (-(dm.T) * w[None, :]).to(q.dtype)
            r = vw @ fm
            r = r.clone()
            r[..., n, :] += fhat_r
            r[..., 0, :] -= fhat_l
            r = winv[:, None] * r
        elif form == "strong":
            r = (dm.to(q.dtype)) @ fm
            r = r.clone()
            r[..., n, :] += winv[n] * (fhat_r - fm[..., n, :])
            r[..., 0, :] -= winv[0] * (fhat_l - fm[..., 0, :])
        else:
            raise ValueError(form)
        total = total + _back(r, d)
    return mesh.scale * m_diag[..., None].to(q.dtype) * total

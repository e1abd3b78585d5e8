"""Plain FP64 GL-DGSEM residual of the implicit step (test oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

What it computes, with the paper's notation:
  * R(Q) = M (Q - Q_s) / dt + H(Q)    (eq. ImplicitDisc with backward Euler,
    eq. DiscretNS), the nonlinear residual whose negative is the right-hand
    side B of the Newton system (eq. NewtonLinSys1);
  * H_j = - int f . grad(phi_j) + oint f_hat phi_j   per node j (eq. DGSEMsystem:1),
    with f = f^a(q) - f^nu(q, g), every integral evaluated with the
    Gauss-Lobatto rule on the element's own nodes;
  * g_j = ( - int q grad(phi_j) + oint phi_j q_hat n ) / (J w_j)   (eq. DGSEMsystem:2);
  * f_hat = local Lax-Friedrichs advective flux minus the Bassi-Rebay 1
    viscous flux {{f^nu(q, g)}}; q_hat = {{q}} (Section 2.1);
  * the nondimensional Navier-Stokes fluxes of Appendix B.

The weak forms above are written as quadrature sums; nothing here uses the
strong (summation-by-parts) rewrite, so a test that compares against a
strong-form evaluation checks both.

Mesh: K^3 cubes of side h = length / K, periodic; x = x_e + (h/2)(xi + 1),
so J = (h/2)^3, the face Jacobian is (h/2)^2 and d xi / dx = 2 / h.
Arrays have shape [K, K, K, P, P, P, 5] = (ez, ey, ex, k, j, i, v): Cartesian
direction d (0 = x, 1 = y, 2 = z) runs along element axis 2 - d and node axis
5 - d.  Flattening gives the DOF order 5 (e P^3 + n) + v with
e = ex + K ey + K^2 ez and n = i + P j + P^2 k.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from numpy.polynomial import legendre as npleg

NVAR = 5


@dataclass(frozen=True)
class Flow:
    """Reference numbers of the nondimensional equations (Appendix B)."""
    mach: float
    reynolds: float
    gamma: float = 1.4
    prandtl: float = 0.72
    sutherland: float = 110.4 / 288.15


@dataclass(frozen=True)
class Grid:
    k_elem: int
    order: int
    length: float = 2.0 * math.pi

    @property
    def p(self) -> int:
        return self.order + 1

    @property
    def h(self) -> float:
        return self.length / self.k_elem


# --------------------------------------------------------------------------
# Gauss-Lobatto rule and Lagrange basis (Section 2.1)
# --------------------------------------------------------------------------

def gl_rule(order: int):
    """Nodes: -1, 1 and the roots of L_N'; weights 2 / (N (N+1) L_N(x)^2)."""
    coef = np.zeros(order + 1)
    coef[order] = 1.0
    inner = np.sort(npleg.legroots(npleg.legder(coef)).real)
    x = np.concatenate([[-1.0], inner, [1.0]])
    # one Newton polish of the interior roots on L_N' (roots of a companion
    # matrix carry a few ulps of error)
    d1 = npleg.legder(coef)
    d2 = npleg.legder(coef, 2)
    x[1:-1] -= npleg.legval(x[1:-1], d1) / npleg.legval(x[1:-1], d2)
    w = 2.0 / (order * (order + 1) * npleg.legval(x, coef) ** 2)
    return x, w


def lagrange_derivative(x: np.ndarray) -> np.ndarray:
    """D[l, a] = phi_a'(x_l) for the Lagrange basis on nodes x (product rule)."""
    p = len(x)
    dm = np.zeros((p, p))
    for a in range(p):
        denom = np.prod([x[a] - x[m] for m in range(p) if m != a])
        for l in range(p):
            if l == a:
                dm[l, a] = sum(1.0 / (x[a] - x[m]) for m in range(p) if m != a)
            else:
                num = np.prod([x[l] - x[m] for m in range(p) if m not in (a, l)])
                dm[l, a] = num / denom
    return dm


def mass(grid: Grid) -> np.ndarray:
    """Diagonal mass matrix J w_i w_j w_k per node, shape [K, K, K, P, P, P]."""
    _, w = gl_rule(grid.order)
    jac = (grid.h / 2.0) ** 3
    m = jac * np.einsum("k,j,i->kji", w, w, w)
    k = grid.k_elem
    return np.broadcast_to(m, (k, k, k) + m.shape).copy()


# --------------------------------------------------------------------------
# Fluxes (Appendix B)
# --------------------------------------------------------------------------

def primitive(q: np.ndarray, flow: Flow):
    """rho, velocity [..., 3], pressure, specific internal energy, temperature."""
    rho = q[..., 0]
    vel = q[..., 1:4] / rho[..., None]
    e_int = q[..., 4] / rho - 0.5 * np.sum(vel * vel, axis=-1)
    p = (flow.gamma - 1.0) * rho * e_int
    temp = flow.gamma * flow.mach ** 2 * p / rho
    return rho, vel, p, e_int, temp


def euler_flux(q: np.ndarray, d: int, flow: Flow) -> np.ndarray:
    """f^a_d = (rho u_d, rho u u_d + p e_d, (rho E + p) u_d)."""
    rho, vel, p, _, _ = primitive(q, flow)
    ud = vel[..., d]
    f = np.empty_like(q)
    f[..., 0] = rho * ud
    for i in range(3):
        f[..., 1 + i] = q[..., 1 + i] * ud + (p if i == d else 0.0)
    f[..., 4] = (q[..., 4] + p) * ud
    return f


def sutherland(temp: np.ndarray, flow: Flow) -> np.ndarray:
    s = flow.sutherland
    return temp ** 1.5 * (1.0 + s) / (temp + s)


def viscous_flux(q: np.ndarray, grad: np.ndarray, d: int, flow: Flow) -> np.ndarray:
    """f^nu_d = (0, tau[:, d], v . tau[:, d] + kappa dT/dx_d) / Re.

    grad[..., k, v] = d q_v / d x_k.  Velocity and internal-energy gradients
    follow from the conserved ones by the quotient rule; kappa grad T =
    (mu gamma / Pr) grad e in these units.
    """
    rho, vel, _, _, temp = primitive(q, flow)
    mu = sutherland(temp, flow)
    grho = grad[..., :, 0]                                      # [..., 3]
    # grad_v[..., i, k] = d v_i / d x_k
    grad_v = (np.swapaxes(grad[..., :, 1:4], -1, -2) - vel[..., :, None] * grho[..., None, :]) \
        / rho[..., None, None]
    energy = q[..., 4] / rho
    grad_e = (grad[..., :, 4] - energy[..., None] * grho) / rho[..., None] \
        - np.einsum("...i,...ik->...k", vel, grad_v)
    div = np.trace(grad_v, axis1=-2, axis2=-1)
    tau_d = mu[..., None] * (grad_v[..., :, d] + grad_v[..., d, :])
    tau_d[..., d] -= (2.0 / 3.0) * mu * div
    heat = mu * flow.gamma / flow.prandtl * grad_e[..., d]
    f = np.zeros_like(q)
    f[..., 1:4] = tau_d / flow.reynolds
    f[..., 4] = (np.sum(vel * tau_d, axis=-1) + heat) / flow.reynolds
    return f


def lax_friedrichs(q_minus: np.ndarray, q_plus: np.ndarray, d: int, flow: Flow) -> np.ndarray:
    """Rusanov flux through a face of normal +e_d, q_minus on the side the normal leaves."""
    speeds = []
    for q in (q_minus, q_plus):
        rho, vel, p, _, _ = primitive(q, flow)
        speeds.append(np.abs(vel[..., d]) + np.sqrt(flow.gamma * p / rho))
    lam = np.maximum(speeds[0], speeds[1])
    return 0.5 * (euler_flux(q_minus, d, flow) + euler_flux(q_plus, d, flow)) \
        - 0.5 * lam[..., None] * (q_plus - q_minus)


# --------------------------------------------------------------------------
# Weak-form operators (eq. DGSEMsystem)
# --------------------------------------------------------------------------

def _line_last(a: np.ndarray, d: int) -> np.ndarray:
    """Put the node axis of direction d just before the variable axis."""
    return np.moveaxis(a, 5 - d, -2)


def _line_back(a: np.ndarray, d: int) -> np.ndarray:
    return np.moveaxis(a, -2, 5 - d)


def _transverse_weights(w: np.ndarray) -> np.ndarray:
    """w_a w_b of the two transverse directions, [P, P].

    Moving one node axis next to the variable axis keeps the other two in
    order, so in line-last layout the product is the same for every direction."""
    return np.outer(w, w)


def _neighbour(a: np.ndarray, d: int, step: int) -> np.ndarray:
    """Field of the element at +step along direction d (periodic)."""
    return np.roll(a, -step, axis=2 - d)


def lifted_gradient(q: np.ndarray, grid: Grid) -> np.ndarray:
    """BR1 gradient of eq. DGSEMsystem:2 in weak form; returns [..., 3, 5]."""
    x, w = gl_rule(grid.order)
    dm = lagrange_derivative(x)
    n = grid.order
    jac = (grid.h / 2.0) ** 3
    jac_face = (grid.h / 2.0) ** 2
    scale = 2.0 / grid.h
    mw = mass(grid)
    g = np.zeros(q.shape[:-1] + (3, NVAR))
    for d in range(3):
        ql = _line_last(q, d)                                   # [..., P, 5]
        wt = _transverse_weights(w)
        # - int q d(phi_j)/dx_d: sum over nodes a on the line through j
        vol = -jac * scale * np.einsum("a,al,...av->...lv", w, dm, ql)
        vol = vol * wt[:, :, None, None]
        # + oint phi_j q_hat n_d: right face (n = +e_d) at l = N, left face at l = 0
        surf = np.zeros_like(vol)
        right = _line_last(_neighbour(q, d, +1), d)[..., 0, :]
        left = _line_last(_neighbour(q, d, -1), d)[..., n, :]
        surf[..., n, :] += jac_face * wt[:, :, None] * 0.5 * (ql[..., n, :] + right)
        surf[..., 0, :] -= jac_face * wt[:, :, None] * 0.5 * (ql[..., 0, :] + left)
        g[..., d, :] = _line_back(vol + surf, d) / mw[..., None]
    return g


def operator_h(q: np.ndarray, grid: Grid, flow: Flow) -> np.ndarray:
    """H(Q) of eq. DiscretNS from eq. DGSEMsystem:1 (mass-weighted, same layout as q)."""
    x, w = gl_rule(grid.order)
    dm = lagrange_derivative(x)
    n = grid.order
    jac = (grid.h / 2.0) ** 3
    jac_face = (grid.h / 2.0) ** 2
    scale = 2.0 / grid.h
    g = lifted_gradient(q, grid)
    h = np.zeros_like(q)
    for d in range(3):
        f = euler_flux(q, d, flow) - viscous_flux(q, g, d, flow)
        fl = _line_last(f, d)
        wt = _transverse_weights(w)
        vol = -jac * scale * np.einsum("a,al,...av->...lv", w, dm, fl) * wt[:, :, None, None]
        # numerical flux on every +e_d face: own node l = N against the right neighbour's l = 0
        q_in = _line_last(q, d)[..., n, :]
        q_out = _line_last(_neighbour(q, d, +1), d)[..., 0, :]
        g_in = np.moveaxis(g, 5 - d, -3)[..., n, :, :]
        g_out = np.moveaxis(_neighbour(g, d, +1), 5 - d, -3)[..., 0, :, :]
        f_hat = lax_friedrichs(q_in, q_out, d, flow) \
            - 0.5 * (viscous_flux(q_in, g_in, d, flow) + viscous_flux(q_out, g_out, d, flow))
        f_hat_left = _neighbour(f_hat, d, -1)       # each element's -e_d face is its left neighbour's +e_d face
        surf = np.zeros_like(vol)
        surf[..., n, :] += jac_face * wt[:, :, None] * f_hat
        surf[..., 0, :] -= jac_face * wt[:, :, None] * f_hat_left
        h += _line_back(vol + surf, d)
    return h


def residual(q: np.ndarray, grid: Grid, flow: Flow, q_s: np.ndarray | None = None,
             dt: float | None = None) -> np.ndarray:
    """R(Q) = M (Q - Q_s) / dt + H(Q); without q_s, H(Q)."""
    h = operator_h(q, grid, flow)
    if q_s is None:
        return h
    return mass(grid)[..., None] * (q - q_s) / dt + h

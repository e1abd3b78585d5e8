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
  * the nondimensional Navier-Stokes fluxes of Appendix B;
  * A v = (M / dt + dH/dQ) v, the Newton matrix of eq. NewtonLinSys1 applied to
    a vector, by complex-step differentiation of R (jacobian_apply*): |x| and
    max are written so that a complex argument carries their derivative
    (x sign(Re x), comparison of real parts), with the same values as np.abs
    and np.maximum on real input.

  * optionally (viscous="sipg") the symmetric interior penalty viscous flux,
    the paper's choice for its example (Section 4): the volume term keeps the
    lifted gradient (whose surface value {{q}} carries the symmetric term),
    and the face flux is compact,
        f_hat^nu = {{f^nu(q, grad q)}} + sigma f^nu({{q}}, [[q]] n),
    the average of each side's viscous flux with its own (broken) gradient
    of the nodal interpolant, plus a penalty: the viscous flux of the mean
    state applied to the jump q^- - q^+ taken as a gradient along the face
    normal, scaled by sigma = eta (N + 1)^2 / h;
  * optional isothermal no-slip walls (Walls) on the two domain faces normal
    to one direction, the mesh staying periodic in the other two: the outer
    state of a wall face is the function q^-(q^+) of Section 2.1.1 (the
    Dirichlet condition; see wall_ghost), the BR1 surface value of the lifting
    is 1/2 (q^+ + q^-(q^+)), the advective flux is the Lax-Friedrichs flux
    between q^+ and q^-(q^+), and the viscous flux is that of the wall state
    1/2 (q^+ + q^-) with the inner gradient (the Neumann part of the
    condition, Section 2.1.2).

The weak forms above are written as quadrature sums; nothing here uses the
strong (summation-by-parts) rewrite, so a test that compares against a
strong-form evaluation checks both.

Mesh: K^3 cubes of side h = length / K, periodic; x = x_e + (h/2)(xi + 1),
so J = (h/2)^3, the face Jacobian is (h/2)^2 and d xi / dx = 2 / h.  The
*_curved functions take any periodic mesh of curved hexahedra given by its
node positions (high-order mapping sampled at the GL nodes): metric terms in
the conservative curl form, contravariant fluxes, face fluxes along J a^i.
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


@dataclass(frozen=True)
class Walls:
    """Isothermal no-slip walls on the domain faces x_d = 0 and x_d = length
    (elements 0 and K-1 along d); periodic in the other two directions."""
    d: int = 2
    t_wall: float = 1.0


def wall_ghost(q: np.ndarray, flow: Flow, t_wall: float) -> np.ndarray:
    """Outer state q^-(q^+) of an isothermal no-slip wall: the same density, the
    momentum reversed, and rho E^- = 2 rho e_w - rho E^+ with e_w the specific
    internal energy at the wall temperature, so that the average
    1/2 (q^+ + q^-) is exactly the wall state (zero velocity, temperature
    t_wall) for every q^+.  Linear in q^+ (the Jacobian q^-_{q^+} of
    Section 2.1.1 is a constant matrix)."""
    e_w = t_wall / (flow.gamma * (flow.gamma - 1.0) * flow.mach ** 2)
    out = np.empty_like(q)
    out[..., 0] = q[..., 0]
    out[..., 1:4] = -q[..., 1:4]
    out[..., 4] = 2.0 * q[..., 0] * e_w - q[..., 4]
    return out


def _layer(a: np.ndarray, d: int, index: int) -> tuple:
    """Index tuple selecting the elements at position `index` along direction d."""
    sl = [slice(None)] * 3          # element axes lead every array
    sl[2 - d] = index
    return tuple(sl)


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


def _abs(x: np.ndarray) -> np.ndarray:
    """|x| written as x sign(Re x): the same value for real x, and on a
    complex-step argument its imaginary part carries sign(x) x' (zero at 0)."""
    return x * np.sign(x.real)


def _larger(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """max(a, b) by the real parts, a at a tie (the same value for real input)."""
    return np.where(a.real >= b.real, a, b)


def lax_friedrichs(q_minus: np.ndarray, q_plus: np.ndarray, d: int, flow: Flow) -> np.ndarray:
    """Rusanov flux through a face of normal +e_d, q_minus on the side the normal leaves."""
    speeds = []
    for q in (q_minus, q_plus):
        rho, vel, p, _, _ = primitive(q, flow)
        speeds.append(_abs(vel[..., d]) + np.sqrt(flow.gamma * p / rho))
    lam = _larger(speeds[0], speeds[1])
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


def lifted_gradient(q: np.ndarray, grid: Grid, walls: Walls | None = None,
                    flow: Flow | None = None) -> np.ndarray:
    """BR1 gradient of eq. DGSEMsystem:2 in weak form; returns [..., 3, 5].
    With walls (flow needed for the wall state), the outer value at a wall face
    is q^-(q^+) (wall_ghost)."""
    x, w = gl_rule(grid.order)
    dm = lagrange_derivative(x)
    n = grid.order
    jac = (grid.h / 2.0) ** 3
    jac_face = (grid.h / 2.0) ** 2
    scale = 2.0 / grid.h
    mw = mass(grid)
    g = np.zeros(q.shape[:-1] + (3, NVAR), dtype=q.dtype)
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
        if walls is not None and walls.d == d:
            right, left = right.copy(), left.copy()
            hi, lo = _layer(right, d, -1), _layer(left, d, 0)
            right[hi] = wall_ghost(ql[..., n, :][hi], flow, walls.t_wall)
            left[lo] = wall_ghost(ql[..., 0, :][lo], flow, walls.t_wall)
        surf[..., n, :] += jac_face * wt[:, :, None] * 0.5 * (ql[..., n, :] + right)
        surf[..., 0, :] -= jac_face * wt[:, :, None] * 0.5 * (ql[..., 0, :] + left)
        g[..., d, :] = _line_back(vol + surf, d) / mw[..., None]
    return g


def wall_fluxes(q: np.ndarray, g: np.ndarray, d: int, flow: Flow, walls: Walls):
    """Numerical fluxes along +e_d through the two wall faces of the elements
    next to them: (through the +d face of the last layer, through the -d face
    of the first layer), each [.., P, P, 5] on those elements' face nodes.
    Lax-Friedrichs between the inner state and q^-(q^+) (the normal +e_d leaves
    the inner side at the upper wall and enters it at the lower one), minus the
    viscous flux of the wall state 1/2 (q^+ + q^-) with the inner gradient."""
    n = q.shape[3] - 1
    out = []
    for side, l in ((-1, n), (0, 0)):
        sel = _layer(q, d, side)
        q_in = _line_last(q, d)[..., l, :][sel]
        g_in = np.moveaxis(g, 5 - d, -3)[..., l, :, :][sel]
        q_gh = wall_ghost(q_in, flow, walls.t_wall)
        q_w = 0.5 * (q_in + q_gh)
        adv = lax_friedrichs(q_in, q_gh, d, flow) if side == -1 else lax_friedrichs(q_gh, q_in, d, flow)
        out.append(adv - viscous_flux(q_w, g_in, d, flow))
    return out[0], out[1]


def broken_gradient(q: np.ndarray, grid: Grid) -> np.ndarray:
    """Element-local gradient of the nodal interpolant at the nodes (no surface
    term): along each direction d, (2/h) sum_a D[l][a] q_a on the d-line; [..., 3, 5]."""
    x, _ = gl_rule(grid.order)
    dm = lagrange_derivative(x)
    scale = 2.0 / grid.h
    g = np.zeros(q.shape[:-1] + (3, NVAR), dtype=q.dtype)
    for d in range(3):
        g[..., d, :] = _line_back(scale * np.einsum("la,...av->...lv", dm, _line_last(q, d)), d)
    return g


SIPG_ETA = 1.0


def sipg_penalty(grid: Grid, eta: float | None = None) -> float:
    """sigma = eta (N + 1)^2 / h (eta: SIPG_ETA unless given)."""
    return (SIPG_ETA if eta is None else eta) * (grid.order + 1) ** 2 / grid.h


def sipg_viscous_flux(q_in, gb_in, q_out, gb_out, d: int, flow: Flow, sigma: float) -> np.ndarray:
    """Compact viscous flux through a +e_d face (q_in on the side the normal leaves):
    {{f^nu_d(q, grad q)}} + sigma f^nu_d({{q}}, [[q]] e_d), [[q]] = q_out - q_in."""
    jump = np.zeros(q_in.shape[:-1] + (3, NVAR), dtype=np.result_type(q_in, q_out))
    jump[..., d, :] = q_out - q_in
    return 0.5 * (viscous_flux(q_in, gb_in, d, flow) + viscous_flux(q_out, gb_out, d, flow)) \
        + sigma * viscous_flux(0.5 * (q_in + q_out), jump, d, flow)


def operator_h(q: np.ndarray, grid: Grid, flow: Flow, walls: Walls | None = None,
               viscous: str = "br1") -> np.ndarray:
    """H(Q) of eq. DiscretNS from eq. DGSEMsystem:1 (mass-weighted, same layout as q);
    optional isothermal no-slip walls (wall_fluxes on their faces); viscous face
    flux "br1" (Bassi-Rebay 1) or "sipg" (symmetric interior penalty)."""
    if viscous not in ("br1", "sipg"):
        raise ValueError(viscous)
    if viscous == "sipg" and walls is not None:
        raise NotImplementedError("walls with the interior-penalty flux")
    x, w = gl_rule(grid.order)
    dm = lagrange_derivative(x)
    n = grid.order
    jac = (grid.h / 2.0) ** 3
    jac_face = (grid.h / 2.0) ** 2
    scale = 2.0 / grid.h
    g = lifted_gradient(q, grid, walls, flow)
    gb = broken_gradient(q, grid) if viscous == "sipg" else None
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
        if viscous == "sipg":
            gb_in = np.moveaxis(gb, 5 - d, -3)[..., n, :, :]
            gb_out = np.moveaxis(_neighbour(gb, d, +1), 5 - d, -3)[..., 0, :, :]
            f_hat = lax_friedrichs(q_in, q_out, d, flow) \
                - sipg_viscous_flux(q_in, gb_in, q_out, gb_out, d, flow, sipg_penalty(grid))
        else:
            f_hat = lax_friedrichs(q_in, q_out, d, flow) \
                - 0.5 * (viscous_flux(q_in, g_in, d, flow) + viscous_flux(q_out, g_out, d, flow))
        f_hat_left = _neighbour(f_hat, d, -1)       # each element's -e_d face is its left neighbour's +e_d face
        if walls is not None and walls.d == d:
            f_hi, f_lo = wall_fluxes(q, g, d, flow, walls)
            f_hat, f_hat_left = f_hat.copy(), f_hat_left.copy()
            f_hat[_layer(f_hat, d, -1)] = f_hi
            f_hat_left[_layer(f_hat_left, d, 0)] = f_lo
        surf = np.zeros_like(vol)
        surf[..., n, :] += jac_face * wt[:, :, None] * f_hat
        surf[..., 0, :] -= jac_face * wt[:, :, None] * f_hat_left
        h += _line_back(vol + surf, d)
    return h


def residual(q: np.ndarray, grid: Grid, flow: Flow, q_s: np.ndarray | None = None,
             dt: float | None = None, walls: Walls | None = None, viscous: str = "br1") -> np.ndarray:
    """R(Q) = M (Q - Q_s) / dt + H(Q); without q_s, H(Q)."""
    h = operator_h(q, grid, flow, walls, viscous)
    if q_s is None:
        return h
    return mass(grid)[..., None] * (q - q_s) / dt + h


CS_STEP = 1e-30


def jacobian_apply(q: np.ndarray, v: np.ndarray, grid: Grid, flow: Flow, dt: float | None = None,
                   walls: Walls | None = None, viscous: str = "br1") -> np.ndarray:
    """A v = (M / dt + dH/dQ(q)) v, the Newton matrix of eq. NewtonLinSys1 at q
    applied to v (without dt: dH/dQ(q) v), by complex-step differentiation of
    the residual: Im R(q + i h v) / h with h = 1e-30, exact to rounding (no
    subtraction of nearby values)."""
    qc = q.astype(np.complex128) + 1j * CS_STEP * v
    if dt is None:
        return operator_h(qc, grid, flow, walls, viscous).imag / CS_STEP
    return residual(qc, grid, flow, q_s=q, dt=dt, walls=walls, viscous=viscous).imag / CS_STEP


def wall_face_mask(k_elem: int, walls: Walls | None) -> np.ndarray:
    """Physical faces of every element (natural element order e = ex + K ey + K^2 ez):
    bit 2 d' + s is set when the face of direction d' on side s (0: the -d'
    face, node index 0; 1: the +d' face, node index N) lies on a wall."""
    mask = np.zeros((k_elem, k_elem, k_elem), dtype=np.uint8)
    if walls is not None:
        d = walls.d
        mask[_layer(mask, d, 0)] |= np.uint8(1 << (2 * d))
        mask[_layer(mask, d, -1)] |= np.uint8(1 << (2 * d + 1))
    return mask.reshape(-1)


# --------------------------------------------------------------------------
# Curvilinear elements: high-order mapping x(xi) sampled at the GL nodes and
# its metric terms.  H keeps the weak form of eq. DGSEMsystem, with the
# contravariant fluxes F^i = sum_n (J a^i)_n f_n in reference space and the
# face normal J a^i (its length is the face area element).
# --------------------------------------------------------------------------

def _d_along(a: np.ndarray, axis: int, dm: np.ndarray) -> np.ndarray:
    """out[.., l, ..] = sum_a D[l, a] a[.., a, ..] along the given node axis."""
    out = np.moveaxis(a, axis, -1) @ dm.T
    return np.moveaxis(out, -1, axis)


def metric_terms(xyz: np.ndarray, grid: Grid):
    """(J a^i)_n in the conservative curl form and J, from node positions.

    xyz [K, K, K, P, P, P, 3].  With X the element's node coordinates and
    (n, m, l) cyclic, (J a^i)_n = - e_i . curl_xi( X_l grad_xi X_m ), every
    derivative taken with the GL derivative matrix on the element's nodes
    (Kopriva 2006).  The discrete divergence sum_i d/dxi_i (J a^i)_n then
    vanishes identically, which is what keeps a uniform state steady.  J is
    the determinant of the discrete d x / d xi.  Returns ja [..., 3 (i), 3 (n)]
    and jac [...].  Each element is shifted to its first node first, which
    leaves the curl form unchanged (the curl of a discrete gradient is zero)."""
    x, _ = gl_rule(grid.order)
    dm = lagrange_derivative(x)
    X = xyz - xyz[:, :, :, :1, :1, :1, :]
    # dX[..., j, m] = d X_m / d xi_j   (xi_j runs along node axis 5 - j)
    dX = np.stack([_d_along(X, 5 - j, dm) for j in range(3)], axis=-2)
    ja = np.zeros(X.shape[:-1] + (3, 3))
    for n in range(3):
        m, l = (n + 1) % 3, (n + 2) % 3
        v = X[..., l][..., None] * dX[..., :, m]                 # v_j = X_l d X_m / d xi_j
        for i in range(3):
            j, k = (i + 1) % 3, (i + 2) % 3
            curl_i = _d_along(v[..., k], 5 - j, dm) - _d_along(v[..., j], 5 - k, dm)
            ja[..., i, n] = -curl_i
    return ja, np.linalg.det(dX)


def curved_mass(grid: Grid, jac: np.ndarray) -> np.ndarray:
    """Diagonal mass J_j w_i w_j w_k per node."""
    _, w = gl_rule(grid.order)
    return jac * np.einsum("k,j,i->kji", w, w, w)


def lax_friedrichs_normal(q_minus, q_plus, nvec, flow: Flow):
    """Rusanov flux along the (unnormalized) normal nvec [..., 3], scaled by |nvec|."""
    s = np.linalg.norm(nvec, axis=-1)
    nh = nvec / s[..., None]
    speeds = []
    for q in (q_minus, q_plus):
        rho, vel, p, _, _ = primitive(q, flow)
        speeds.append(_abs(np.sum(vel * nh, axis=-1)) + np.sqrt(flow.gamma * p / rho))
    lam = _larger(speeds[0], speeds[1])
    f = sum(nvec[..., d, None] * (euler_flux(q_minus, d, flow) + euler_flux(q_plus, d, flow)) for d in range(3))
    return 0.5 * f - 0.5 * (lam * s)[..., None] * (q_plus - q_minus)


def _face_metric(ja: np.ndarray, i: int, l: int) -> np.ndarray:
    """(J a^i) at the nodes l of the line along xi_i: [K, K, K, P, P, 3]."""
    return np.moveaxis(ja[..., i, :], 5 - i, -2)[..., l, :]


def lifted_gradient_curved(q: np.ndarray, grid: Grid, ja: np.ndarray, jac: np.ndarray) -> np.ndarray:
    """BR1 gradient of eq. DGSEMsystem:2 on curved elements:
    J_j w_j g_{n,j} = sum_i [ - int (J a^i)_n q d(phi_j)/d xi_i + oint phi_j q_hat (J a^i)_n ]."""
    x, w = gl_rule(grid.order)
    dm = lagrange_derivative(x)
    n = grid.order
    wt = _transverse_weights(w)
    g = np.zeros(q.shape[:-1] + (3, NVAR), dtype=q.dtype)
    for i in range(3):
        ql = _line_last(q, i)
        right = _line_last(_neighbour(q, i, +1), i)[..., 0, :]
        left = _line_last(_neighbour(q, i, -1), i)[..., n, :]
        for c in range(3):
            jl = _line_last(ja[..., i, c][..., None], i)              # [..., P, 1]
            vol = -np.einsum("a,al,...av->...lv", w, dm, jl * ql) * wt[:, :, None, None]
            surf = np.zeros_like(vol)
            surf[..., n, :] += wt[:, :, None] * jl[..., n, :] * 0.5 * (ql[..., n, :] + right)
            surf[..., 0, :] -= wt[:, :, None] * jl[..., 0, :] * 0.5 * (ql[..., 0, :] + left)
            g[..., c, :] += _line_back(vol + surf, i)
    return g / curved_mass(grid, jac)[..., None, None]


def operator_h_curved(q: np.ndarray, grid: Grid, flow: Flow, ja: np.ndarray, jac: np.ndarray) -> np.ndarray:
    """H(Q) on curved elements: per reference direction i, the weak form of
    eq. DGSEMsystem:1 with F^i = sum_n (J a^i)_n f_n and the face flux along
    J a^i of the element that owns the +xi_i face."""
    x, w = gl_rule(grid.order)
    dm = lagrange_derivative(x)
    n = grid.order
    wt = _transverse_weights(w)
    g = lifted_gradient_curved(q, grid, ja, jac)
    f = [euler_flux(q, c, flow) - viscous_flux(q, g, c, flow) for c in range(3)]
    h = np.zeros_like(q)
    for i in range(3):
        ft = sum(ja[..., i, c][..., None] * f[c] for c in range(3))
        fl = _line_last(ft, i)
        vol = -np.einsum("a,al,...av->...lv", w, dm, fl) * wt[:, :, None, None]
        q_in = _line_last(q, i)[..., n, :]
        q_out = _line_last(_neighbour(q, i, +1), i)[..., 0, :]
        g_in = np.moveaxis(g, 5 - i, -3)[..., n, :, :]
        g_out = np.moveaxis(_neighbour(g, i, +1), 5 - i, -3)[..., 0, :, :]
        nvec = _face_metric(ja, i, n)
        visc = sum(nvec[..., c, None] * (viscous_flux(q_in, g_in, c, flow) + viscous_flux(q_out, g_out, c, flow))
                   for c in range(3))
        f_hat = lax_friedrichs_normal(q_in, q_out, nvec, flow) - 0.5 * visc
        f_hat_left = _neighbour(f_hat, i, -1)
        surf = np.zeros_like(vol)
        surf[..., n, :] += wt[:, :, None] * f_hat
        surf[..., 0, :] -= wt[:, :, None] * f_hat_left
        h += _line_back(vol + surf, i)
    return h


def residual_curved(q: np.ndarray, grid: Grid, flow: Flow, ja: np.ndarray, jac: np.ndarray,
                    q_s: np.ndarray | None = None, dt: float | None = None) -> np.ndarray:
    """R(Q) = M (Q - Q_s) / dt + H(Q) on curved elements; without q_s, H(Q)."""
    h = operator_h_curved(q, grid, flow, ja, jac)
    if q_s is None:
        return h
    return curved_mass(grid, jac)[..., None] * (q - q_s) / dt + h


def jacobian_apply_curved(q: np.ndarray, v: np.ndarray, grid: Grid, flow: Flow, ja: np.ndarray,
                          jac: np.ndarray, dt: float | None = None) -> np.ndarray:
    """A v on curved elements, by the same complex step as jacobian_apply."""
    qc = q.astype(np.complex128) + 1j * CS_STEP * v
    if dt is None:
        return operator_h_curved(qc, grid, flow, ja, jac).imag / CS_STEP
    return residual_curved(qc, grid, flow, ja, jac, q_s=q, dt=dt).imag / CS_STEP

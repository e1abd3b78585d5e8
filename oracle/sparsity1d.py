"""Jacobian sparsity of the 1D scalar DGSEM on Gauss and Gauss-Lobatto nodes
(test oracle; TEST INFRASTRUCTURE ONLY, see the package header).

The paper explains why static condensation applies to the GL-DGSEM by the
sparsity of the implicit Jacobian (Section 3.1, "Jacobian Sparsity
Patterns", with the off-diagonal terms of eq. AdvOffDiag and eq. DiffOffDiag)
and illustrates it on a periodic 1D mesh of seven elements of order 9 and a
scalar equation.  This module builds that Jacobian for the linear
advection-diffusion equation  d_t q + d_x (a q - nu d_x q) = 0:

  * nodes "gl" (Gauss-Lobatto, boundary nodes at +-1) or "gauss"
    (Gauss-Legendre, no node on the boundary), collocated quadrature, weak
    form per element as in eq. DGSEMsystem:
        H_j = - sum_m w_m D_mj F_m + l_j(1) Fhat_R - l_j(-1) Fhat_L,
    with l_j(+-1) the Lagrange basis at the element ends;
  * gradient lifted with the face average (eq. DGSEMsystem:2):
        J w_j g_j = - sum_m w_m D_mj q_m + l_j(1) qhat_R - l_j(-1) qhat_L;
  * advective face flux a {q} - (lam / 2) [q] (Lax-Friedrichs with lam > |a|
    couples both neighbours);
  * viscous face flux "br1": nu {g} of the lifted gradients of both sides
    (the scheme of the Navier-Stokes residual here), or "compact": nu {d_x q}
    of each side's own derivative plus a jump penalty, a compact flux of the
    kind the paper restricts its analysis to.

The 3D operator (operator_h3) applies the same 1D operator along the x-, y-
and z-lines of a periodic mesh of cubes, weighted by the transverse
quadrature weights: with constant coefficients on Cartesian cubes the weak
form splits by direction.  It serves the paper's 3D claims on its 2x2x2,
order-3 style mesh (here 3^3 so that opposite neighbours differ).

Because the equation is linear, the Jacobian is the matrix of H, formed
column by column by applying H to unit vectors (brute force).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg

from .dgsem import gl_rule, lagrange_derivative


def nodes_weights(kind: str, order: int):
    """Nodes (ascending) and weights of the collocation rule with order + 1 nodes."""
    if kind == "gl":
        return gl_rule(order)
    if kind == "gauss":
        x, w = npleg.leggauss(order + 1)
        return x, w
    raise ValueError(kind)


def lagrange_at(x: np.ndarray, xi: float) -> np.ndarray:
    """l_j(xi) for the Lagrange basis on nodes x (product formula)."""
    p = len(x)
    out = np.ones(p)
    for j in range(p):
        for k in range(p):
            if k != j:
                out[j] *= (xi - x[k]) / (x[j] - x[k])
    return out


def operator_h(q: np.ndarray, kind: str, order: int, length: float = 2.0, a: float = 1.0,
               lam: float = 2.0, nu: float = 0.0, viscous: str = "br1", sigma: float = 10.0) -> np.ndarray:
    """H(q) for q of shape [..., K, P] (leading axes: independent lines) on a
    periodic mesh of K equal elements."""
    k_elem = q.shape[-2]
    x, w = nodes_weights(kind, order)
    dm = lagrange_derivative(x)
    l_lo, l_hi = lagrange_at(x, -1.0), lagrange_at(x, 1.0)
    jac = length / k_elem / 2.0
    # values at the face to the right of each element: minus side (this
    # element), plus side (the next element)
    q_m = q @ l_hi
    q_p = np.roll(q @ l_lo, -1, axis=-1)
    q_hat = 0.5 * (q_m + q_p)
    q_hat_left = np.roll(q_hat, 1, axis=-1)
    # lifted gradient, weak form
    g = np.zeros_like(q)
    for j in range(len(x)):
        vol = -sum(w[m] * dm[m, j] * q[..., m] for m in range(len(x)))
        g[..., j] = (vol + l_hi[j] * q_hat - l_lo[j] * q_hat_left) / (jac * w[j])
    flux = a * q - nu * g
    f_hat = a * 0.5 * (q_m + q_p) - 0.5 * lam * (q_p - q_m)
    if nu != 0.0:
        if viscous == "br1":
            g_m, g_p = g @ l_hi, np.roll(g @ l_lo, -1, axis=-1)
            f_hat = f_hat - nu * 0.5 * (g_m + g_p)
        elif viscous == "compact":
            d = (q @ dm.T) / jac                      # each element's own derivative at its nodes
            d_m, d_p = d @ l_hi, np.roll(d @ l_lo, -1, axis=-1)
            f_hat = f_hat - nu * 0.5 * (d_m + d_p) + nu * sigma / (2.0 * jac) * (q_p - q_m)
        else:
            raise ValueError(viscous)
    f_hat_left = np.roll(f_hat, 1, axis=-1)
    h = np.zeros_like(q)
    for j in range(len(x)):
        vol = -sum(w[m] * dm[m, j] * flux[..., m] for m in range(len(x)))
        h[..., j] = vol + l_hi[j] * f_hat - l_lo[j] * f_hat_left
    return h


def jacobian(k_elem: int, order: int, kind: str, **kw) -> np.ndarray:
    """dH/dq as a dense [K P, K P] matrix (element-major DOF order)."""
    p = order + 1
    n = k_elem * p
    a = np.zeros((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        a[:, c] = operator_h(e.reshape(k_elem, p), kind, order, **kw).reshape(-1)
    return a


def block(a: np.ndarray, p: int, e_row: int, e_col: int) -> np.ndarray:
    """The (e_row, e_col) block of a matrix in element-major DOF order."""
    return a[e_row * p:(e_row + 1) * p, e_col * p:(e_col + 1) * p]


def operator_h3(q: np.ndarray, kind: str, order: int, length: float = 2.0, **kw) -> np.ndarray:
    """H(q) of the same equation on a periodic K^3 mesh of cubes, q of shape
    [Kz, Ky, Kx, P, P, P] (element z, y, x; node k, j, i).  With constant
    coefficients on Cartesian cubes the weak form splits by direction: the
    term of direction d is the 1D operator along the d-lines, times the
    quadrature weights and face Jacobian of the two transverse directions."""
    x, w = nodes_weights(kind, order)
    jt = (length / q.shape[0] / 2.0) ** 2             # transverse face Jacobian (h/2)^2
    h = np.zeros_like(q)
    for d in range(3):
        ea, na = 2 - d, 5 - d                            # element and node axis of direction d
        lines = np.moveaxis(np.moveaxis(q, ea, -1), na if na < ea else na - 1, -1)
        # lines: [..transverse elements, transverse nodes.., K, P]
        hl = operator_h(lines, kind, order, length=length, **kw)
        hd = np.moveaxis(np.moveaxis(hl, -1, na if na < ea else na - 1), -1, ea)
        wt = np.ones(q.shape[3:])
        for t in range(3):
            if t != d:
                shape = [1, 1, 1]
                shape[2 - t] = len(w)
                wt = wt * w.reshape(shape)
        h += jt * wt[None, None, None] * hd
    return h


def jacobian3(k_elem: int, order: int, kind: str, **kw) -> np.ndarray:
    """dH/dq of the 3D operator as a dense matrix, element-major
    (e = ex + K ey + K^2 ez, node n = i + P j + P^2 k)."""
    p = order + 1
    shape = (k_elem, k_elem, k_elem, p, p, p)
    n = int(np.prod(shape))
    a = np.zeros((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        a[:, c] = operator_h3(e.reshape(shape), kind, order, **kw).reshape(-1)
    return a

"""Legendre-Gauss-Lobatto (GL) nodes, weights and the nodal derivative matrix.

These are the one-dimensional building blocks of the tensor-product GL-DGSEM
(paper, Appendix C: the quadrature rule and the Lagrange basis on the
quadrature nodes).  On GL nodes the rule is exact for polynomials of degree
up to 2N-1 (paper, Introduction), and because the end points are nodes, only
one Lagrange polynomial is nonzero on each end of the interval (Appendix C,
discrete orthogonality) -- the property that makes A_ii block-diagonal.

All values are computed in float64 with numpy.  Nothing here belongs to the
static-condensation arithmetic; this module only builds the synthetic
discretization whose Jacobian is handed to the solver.
"""
from __future__ import annotations

import functools
import math

import numpy as np


def legendre(n: int, x: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Legendre polynomial L_n(x) and its derivative by the three-term recurrence."""
    x = np.asarray(x, dtype=np.float64)
    if n == 0:
        return np.ones_like(x), np.zeros_like(x)
    if n == 1:
        return x.copy(), np.ones_like(x)
    l_prev2, l_prev1 = np.ones_like(x), x.copy()
    d_prev2, d_prev1 = np.zeros_like(x), np.ones_like(x)
    for k in range(2, n + 1):
        l_k = ((2 * k - 1) * x * l_prev1 - (k - 1) * l_prev2) / k
        d_k = d_prev2 + (2 * k - 1) * l_prev1
        l_prev2, l_prev1 = l_prev1, l_k
        d_prev2, d_prev1 = d_prev1, d_k
    return l_prev1, d_prev1


@functools.lru_cache(maxsize=None)
def gl_nodes_weights(n_order: int) -> tuple[np.ndarray, np.ndarray]:
    """N+1 Gauss-Lobatto nodes on [-1, 1] (ascending) and their weights.

    Interior nodes are the roots of L_N'(x); they are found by Newton's method on
    q(x) = L_{N+1}(x) - L_{N-1}(x), which vanishes exactly at all N+1 GL nodes,
    started from the Chebyshev-Gauss-Lobatto points.  Weights are
    w_j = 2 / (N (N+1) L_N(x_j)^2).
    """
    if n_order < 1:
        raise ValueError("polynomial order must be >= 1")
    n = n_order
    x = -np.cos(np.pi * np.arange(n + 1) / n)
    x[0], x[-1] = -1.0, 1.0
    for _ in range(100):
        lp1, _ = legendre(n + 1, x[1:-1])
        lm1, _ = legendre(n - 1, x[1:-1])
        ln, _ = legendre(n, x[1:-1])
        q = lp1 - lm1
        dq = (2 * n + 1) * ln
        step = q / dq
        x[1:-1] -= step
        if np.max(np.abs(step), initial=0.0) < 1e-16:
            break
    # enforce exact symmetry of the node set
    x = 0.5 * (x - x[::-1])
    if n % 2 == 0:
        x[n // 2] = 0.0
    ln, _ = legendre(n, x)
    w = 2.0 / (n * (n + 1) * ln * ln)
    return x, w


def barycentric_weights(x: np.ndarray) -> np.ndarray:
    lam = np.empty_like(x)
    for j in range(len(x)):
        lam[j] = 1.0 / np.prod([x[j] - x[i] for i in range(len(x)) if i != j])
    return lam


@functools.lru_cache(maxsize=None)
def derivative_matrix(n_order: int) -> np.ndarray:
    """D[i, j] = l_j'(x_i) for the Lagrange basis on the GL nodes.

    Off-diagonal entries come from the barycentric form; each diagonal entry is
    minus the sum of its row, so that D annihilates constants exactly.
    """
    x, _ = gl_nodes_weights(n_order)
    lam = barycentric_weights(x)
    p = len(x)
    d = np.zeros((p, p))
    for i in range(p):
        for j in range(p):
            if i != j:
                d[i, j] = (lam[j] / lam[i]) / (x[i] - x[j])
        d[i, i] = -np.sum(d[i, :])
    return d


def lagrange_eval(n_order: int, xi: np.ndarray) -> np.ndarray:
    """Matrix V[m, j] = l_j(xi_m) of the GL Lagrange basis at arbitrary points."""
    x, _ = gl_nodes_weights(n_order)
    xi = np.atleast_1d(np.asarray(xi, dtype=np.float64))
    v = np.ones((len(xi), len(x)))
    for j in range(len(x)):
        for i in range(len(x)):
            if i != j:
                v[:, j] *= (xi - x[i]) / (x[j] - x[i])
    return v


def sbp_boundary(n_order: int) -> np.ndarray:
    """B = diag(-1, 0, ..., 0, 1): the boundary matrix of the SBP identity W D + (W D)^T = B."""
    b = np.zeros((n_order + 1, n_order + 1))
    b[0, 0], b[-1, -1] = -1.0, 1.0
    return b


def closed_form_nodes(n_order: int) -> tuple[np.ndarray, np.ndarray] | None:
    """Textbook closed forms for small N (used only as test pins)."""
    if n_order == 1:
        return np.array([-1.0, 1.0]), np.array([1.0, 1.0])
    if n_order == 2:
        return np.array([-1.0, 0.0, 1.0]), np.array([1 / 3, 4 / 3, 1 / 3])
    if n_order == 3:
        a = 1 / math.sqrt(5)
        return np.array([-1.0, -a, a, 1.0]), np.array([1 / 6, 5 / 6, 5 / 6, 1 / 6])
    if n_order == 4:
        a = math.sqrt(3 / 7)
        return (np.array([-1.0, -a, 0.0, a, 1.0]),
                np.array([1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10]))
    return None

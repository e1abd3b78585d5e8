"""Mixed-order GL-DGSEM residual with mortars on non-affine hexahedra (test oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

The uneven-order configuration: every element e of a periodic K^3 mesh carries
its own polynomial order N_e (p-adaptation, which the paper motivates in its
introduction but does not discretize).  Per element the residual is the one of
module `oracle.dgsem` (eq. DGSEMsystem: weak form as Gauss-Lobatto sums on the
element's own nodes, Bassi-Rebay 1 lifting, local Lax-Friedrichs advective and
BR1 viscous face fluxes, Appendix B fluxes, curl-form metric terms).  What is
new is the face between two elements:

  * mortar (the usual DGSEM treatment of p-nonconforming faces; the paper is
    silent): both face traces are interpolated to the Gauss-Lobatto nodes of
    order M = max(N_L, N_R) of the face; q_hat = 1/2 (q_L + q_R) and the face
    flux f_hat(q_L, q_R, g_L, g_R, n) are evaluated there;
  * each side receives the mortar integral of the face quantity against its
    own face basis, computed with the mortar's quadrature:
        S_ab = sum_mn w_m w_n F_mn l_a(x_m) l_b(x_n) = (I^T (W F) I)_ab,
    I the interpolation matrix from the side's face nodes to the mortar's;
    this is the discrete projection W_N^-1 I^T W_M followed by the side's own
    quadrature, so on a conforming face (I = identity) it is w_a w_b F_ab,
    the conforming scheme of `oracle.dgsem`, and the sum over a face's
    nodes is the same on both sides (conservation);
  * the face normal J a^i on the mortar is that of the element owning the
    face (the one whose +xi_i face it is), interpolated to the mortar.

Geometry: the vertices of the K^3 grid on [0, L)^3 are displaced by
x_d = X_d + a L sin(X_1 + t) sin(X_2 + t) sin(X_3 + t) (every d; periodic in
each X_k with period L = 2 pi; the phase t = pi/4 keeps the vertices of a
2-element-per-direction grid off the zeros of the sines, where t = 0 would
leave that mesh Cartesian) and every element is the trilinear map of its 8
vertices sampled at its own GL nodes.  A trilinear map makes every metric term an exact
polynomial of degree <= 2 per direction, so both sides of a p-nonconforming
face see the same normal polynomial and a uniform state stays exactly steady
(free-stream preservation); a map of higher degree would need the face metric
treatment of Kopriva et al. (2019) on mixed-order faces.

Element e = ex + K ey + K^2 ez; element arrays are [..., P, P, P, 5] =
(k, j, i, v) with P = N_e + 1 and any leading batch axes; the global vector
concatenates the elements, each flattened as 5 (i + P j + P^2 k) + v.
Cartesian direction d runs along node axis -2 - d of a state array.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from .dgsem import (CS_STEP, NVAR, Flow, Grid, euler_flux, gl_rule, lagrange_derivative,
                    lax_friedrichs_normal, metric_terms, viscous_flux)


@dataclass(frozen=True)
class MortarMesh:
    k_elem: int
    orders: tuple
    amplitude: float = 0.05
    length: float = 2.0 * math.pi
    phase: float = 0.25 * math.pi

    @property
    def n_elem(self) -> int:
        return self.k_elem ** 3

    def neighbour(self, e: int, d: int, step: int) -> int:
        k = self.k_elem
        c = [e % k, (e // k) % k, e // (k * k)]
        c[d] = (c[d] + step) % k
        return c[0] + k * c[1] + k * k * c[2]

    def dof_offsets(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum([NVAR * (n + 1) ** 3 for n in self.orders])]).astype(np.int64)

    @property
    def n_dof(self) -> int:
        return int(self.dof_offsets()[-1])


def vertex_position(mesh: MortarMesh, ix: int, iy: int, iz: int) -> np.ndarray:
    """Displaced grid vertex (unwrapped: index K lies at L, not 0)."""
    h = mesh.length / mesh.k_elem
    x = np.array([ix, iy, iz], dtype=float) * h
    s = np.sin(x + mesh.phase)
    return x + mesh.amplitude * mesh.length * s[0] * s[1] * s[2]


def element_nodes(mesh: MortarMesh, e: int) -> np.ndarray:
    """Node positions [P, P, P, 3] of the trilinear element at its GL nodes."""
    k = mesh.k_elem
    ex, ey, ez = e % k, (e // k) % k, e // (k * k)
    x, _ = gl_rule(mesh.orders[e])
    t = 0.5 * (x + 1.0)
    lin = [1.0 - t, t]                                # weight of vertex a = 0 / 1 along a line
    xyz = np.zeros((len(x),) * 3 + (3,))
    for a in (0, 1):
        for b in (0, 1):
            for c in (0, 1):
                wgt = np.einsum("k,j,i->kji", lin[c], lin[b], lin[a])
                xyz += wgt[..., None] * vertex_position(mesh, ex + a, ey + b, ez + c)
    return xyz


def interpolation_matrix(x_from: np.ndarray, x_to: np.ndarray) -> np.ndarray:
    """I[m, a] = l_a(x_to[m]) for the Lagrange basis on x_from."""
    if len(x_from) == len(x_to) and np.array_equal(x_from, x_to):
        return np.eye(len(x_from))
    out = np.ones((len(x_to), len(x_from)))
    for a in range(len(x_from)):
        for b in range(len(x_from)):
            if b != a:
                out[:, a] *= (x_to - x_from[b]) / (x_from[a] - x_from[b])
    return out


@dataclass
class _Element:
    order: int
    w: np.ndarray
    dm: np.ndarray
    ja: np.ndarray          # [P, P, P, 3 (i), 3 (n)]
    jac: np.ndarray         # [P, P, P]
    mass: np.ndarray        # J w_i w_j w_k
    wt: list                # per direction: product of the two transverse weights, [P, P, P]


@dataclass
class _Face:
    left: int               # owner: the face is its +xi_d face (node index N_L)
    right: int              # neighbour: its -xi_d face (node index 0)
    d: int
    wm: np.ndarray          # mortar weights
    il: np.ndarray          # interpolation left face nodes -> mortar
    ir: np.ndarray
    nvec: np.ndarray        # owner's J a^d on the mortar nodes, [M+1, M+1, 3]


@dataclass
class MortarGeometry:
    mesh: MortarMesh
    elems: list = field(default_factory=list)
    faces: list = field(default_factory=list)


def _along(a: np.ndarray, ax: int, index: int) -> tuple:
    """Index tuple fixing node axis `ax` (negative) of array a at `index`."""
    idx = [slice(None)] * a.ndim
    idx[a.ndim + ax] = index
    return tuple(idx)


def build_geometry(mesh: MortarMesh) -> MortarGeometry:
    if len(mesh.orders) != mesh.n_elem or min(mesh.orders) < 1:
        raise ValueError("one order >= 1 per element")
    geo = MortarGeometry(mesh)
    for e in range(mesh.n_elem):
        n = mesh.orders[e]
        x, w = gl_rule(n)
        ja, jac = metric_terms(element_nodes(mesh, e)[None, None, None], Grid(1, n))
        ja, jac = ja[0, 0, 0], jac[0, 0, 0]
        if np.any(jac <= 0.0):
            raise ValueError("folded element")
        w3 = np.einsum("k,j,i->kji", w, w, w)
        wk, wj, wi = w[:, None, None], w[None, :, None], w[None, None, :]
        wt = [np.broadcast_to(wk * wj, w3.shape), np.broadcast_to(wk * wi, w3.shape),
              np.broadcast_to(wj * wi, w3.shape)]
        geo.elems.append(_Element(n, w, lagrange_derivative(x), ja, jac, jac * w3, wt))
    for e in range(mesh.n_elem):
        for d in range(3):
            r = mesh.neighbour(e, d, +1)
            nl, nr = mesh.orders[e], mesh.orders[r]
            m = max(nl, nr)
            xm, wm = gl_rule(m)
            il = interpolation_matrix(gl_rule(nl)[0], xm)
            ir = interpolation_matrix(gl_rule(nr)[0], xm)
            ja_d = geo.elems[e].ja[..., d, :]                   # [P, P, P, 3]
            n_face = ja_d[_along(ja_d, -2 - d, nl)]              # [P, P, 3]
            geo.faces.append(_Face(e, r, d, wm, il, ir, _face_map(n_face, il, il, 1)))
    return geo


def _face_map(f: np.ndarray, left: np.ndarray, right: np.ndarray, tail: int) -> np.ndarray:
    """left @ F @ right^T over the two face node axes of f = [..., a, b, tail...]."""
    src = (f.ndim - 2 - tail, f.ndim - 1 - tail)
    g = np.moveaxis(f, src, (-2, -1))
    return np.moveaxis(left @ g @ right.T, (-2, -1), src)


def _to_side(fm: np.ndarray, im: np.ndarray, wm: np.ndarray, tail: int) -> np.ndarray:
    """Mortar integral against the side's face basis: I^T (w_m w_n F_mn) I."""
    src = (fm.ndim - 2 - tail, fm.ndim - 1 - tail)
    g = np.moveaxis(fm, src, (-2, -1)) * np.outer(wm, wm)
    return np.moveaxis(im.T @ g @ im, (-2, -1), src)


def _weak_line(f: np.ndarray, ax: int, w: np.ndarray, dm: np.ndarray) -> np.ndarray:
    """out_l = sum_a w_a D[a, l] f_a along node axis ax (the GL sum of f dphi_l/dxi)."""
    g = np.moveaxis(f, ax, -1) @ (w[:, None] * dm)
    return np.moveaxis(g, -1, ax)


def split(vec: np.ndarray, geo: MortarGeometry) -> list:
    """Global vector [..., n_dof] -> element arrays [..., P, P, P, 5]."""
    off = geo.mesh.dof_offsets()
    lead = vec.shape[:-1]
    return [vec[..., off[e]:off[e + 1]].reshape(lead + (el.order + 1,) * 3 + (NVAR,))
            for e, el in enumerate(geo.elems)]


def join(parts: list) -> np.ndarray:
    lead = parts[0].shape[:-4]
    return np.concatenate([p.reshape(lead + (-1,)) for p in parts], axis=-1)


def lifted_gradient(qs: list, geo: MortarGeometry) -> list:
    """BR1 gradient (eq. DGSEMsystem:2): J_j w_j g_{c,j} = sum_i [ - int (J a^i)_c q dphi_j/dxi_i
    + oint phi_j q_hat (J a^i)_c ], the face integrals on the mortars."""
    gs = []
    for q, el in zip(qs, geo.elems):
        g = np.zeros(q.shape[:-1] + (3, NVAR), dtype=q.dtype)
        for i in range(3):
            for c in range(3):
                g[..., c, :] -= _weak_line(el.ja[..., i, c][..., None] * q, -2 - i, el.w, el.dm) \
                    * el.wt[i][..., None]
        gs.append(g)
    for f in geo.faces:
        ql = qs[f.left][_along(qs[f.left], -2 - f.d, geo.elems[f.left].order)]
        qr = qs[f.right][_along(qs[f.right], -2 - f.d, 0)]
        q_hat = 0.5 * (_face_map(ql, f.il, f.il, 1) + _face_map(qr, f.ir, f.ir, 1))
        gl = gs[f.left][_along(gs[f.left], -3 - f.d, geo.elems[f.left].order)]
        gr = gs[f.right][_along(gs[f.right], -3 - f.d, 0)]
        for c in range(3):
            fm = q_hat * f.nvec[..., c, None]
            gl[..., c, :] += _to_side(fm, f.il, f.wm, 1)
            gr[..., c, :] -= _to_side(fm, f.ir, f.wm, 1)
    return [g / el.mass[..., None, None] for g, el in zip(gs, geo.elems)]


def operator_h(qs: list, geo: MortarGeometry, flow: Flow) -> list:
    """H(Q) per element (eq. DGSEMsystem:1): - int F^i dphi/dxi_i with
    F^i = sum_c (J a^i)_c (f^a_c - f^nu_c), plus the mortar integral of the face
    flux f_hat = LLF(q_L, q_R, n) - 1/2 (f^nu(q_L, g_L) + f^nu(q_R, g_R)) . n."""
    gs = lifted_gradient(qs, geo)
    hs = []
    for q, g, el in zip(qs, gs, geo.elems):
        fl = [euler_flux(q, c, flow) - viscous_flux(q, g, c, flow) for c in range(3)]
        h = np.zeros_like(q)
        for i in range(3):
            ft = sum(el.ja[..., i, c][..., None] * fl[c] for c in range(3))
            h -= _weak_line(ft, -2 - i, el.w, el.dm) * el.wt[i][..., None]
        hs.append(h)
    for f in geo.faces:
        nl = geo.elems[f.left].order
        ql = _face_map(qs[f.left][_along(qs[f.left], -2 - f.d, nl)], f.il, f.il, 1)
        qr = _face_map(qs[f.right][_along(qs[f.right], -2 - f.d, 0)], f.ir, f.ir, 1)
        gl = _face_map(gs[f.left][_along(gs[f.left], -3 - f.d, nl)], f.il, f.il, 2)
        gr = _face_map(gs[f.right][_along(gs[f.right], -3 - f.d, 0)], f.ir, f.ir, 2)
        visc = sum(f.nvec[..., c, None] * (viscous_flux(ql, gl, c, flow) + viscous_flux(qr, gr, c, flow))
                   for c in range(3))
        f_hat = lax_friedrichs_normal(ql, qr, f.nvec, flow) - 0.5 * visc
        hs[f.left][_along(hs[f.left], -2 - f.d, nl)] += _to_side(f_hat, f.il, f.wm, 1)
        hs[f.right][_along(hs[f.right], -2 - f.d, 0)] -= _to_side(f_hat, f.ir, f.wm, 1)
    return hs


def mass(geo: MortarGeometry) -> np.ndarray:
    """Diagonal of M in the global order (J w_i w_j w_k repeated over the 5 variables)."""
    return np.concatenate([np.repeat(el.mass.reshape(-1), NVAR) for el in geo.elems])


def residual(q: np.ndarray, geo: MortarGeometry, flow: Flow, q_s: np.ndarray | None = None,
             dt: float | None = None) -> np.ndarray:
    """R(Q) = M (Q - Q_s)/dt + H(Q) on global vectors [..., n_dof]; without q_s, H(Q)."""
    h = join(operator_h(split(q, geo), geo, flow))
    if q_s is None:
        return h
    return mass(geo) * (q - q_s) / dt + h


def jacobian_apply(q: np.ndarray, v: np.ndarray, geo: MortarGeometry, flow: Flow,
                   dt: float | None = None) -> np.ndarray:
    """A v = (M/dt + dH/dQ) v by complex step (v may carry leading batch axes)."""
    qc = q.astype(np.complex128) + 1j * CS_STEP * v
    if dt is None:
        return residual(qc, geo, flow).imag / CS_STEP
    return residual(qc, geo, flow, q_s=q, dt=dt).imag / CS_STEP


_WORKER_ARGS = None


def _worker_init(*args):
    global _WORKER_ARGS
    _WORKER_ARGS = args


def _unit_columns(c0: int, nb: int, args=None):
    """Columns c0 .. c0 + nb - 1 of A (as rows of a sparse matrix)."""
    q, geo, flow, dt = _WORKER_ARGS if args is None else args
    v = np.zeros((nb, q.shape[-1]))
    v[np.arange(nb), c0 + np.arange(nb)] = 1.0
    return sp.csr_matrix(jacobian_apply(q, v, geo, flow, dt))


def _unit_columns_star(c):
    return _unit_columns(*c)


def jacobian_matrix(q: np.ndarray, geo: MortarGeometry, flow: Flow, dt: float | None = None,
                    batch: int = 64, workers: int = 1) -> sp.csr_matrix:
    """The Newton matrix A of eq. NewtonLinSys1, column by column (complex step on
    batches of unit vectors); exact to rounding.  With workers > 1 the batches
    are shared out to that many spawned processes (the same arithmetic per
    column; the batches only decide which columns are evaluated together)."""
    n = q.shape[-1]
    chunks = [(c0, min(batch, n - c0)) for c0 in range(0, n, batch)]
    if workers > 1:
        import multiprocessing
        from concurrent.futures import ProcessPoolExecutor
        ctx = multiprocessing.get_context("spawn")
        with ProcessPoolExecutor(workers, mp_context=ctx, initializer=_worker_init,
                                 initargs=(q, geo, flow, dt)) as ex:
            cols = list(ex.map(_unit_columns_star, chunks, chunksize=max(1, len(chunks) // (4 * workers))))
    else:
        cols = [_unit_columns(c0, nb, (q, geo, flow, dt)) for c0, nb in chunks]
    a = sp.vstack(cols).T.tocsr()                      # rows of the stack are columns of A
    a.eliminate_zeros()
    return a

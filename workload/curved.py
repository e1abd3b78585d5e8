"""Implicit-step inputs on curved periodic hexahedra: H(Q) of the GL-DGSEM with
metric terms, and the backward-Euler Jacobian A = M/dt + dH/dQ as per-element
blocks for the static condensation.

Discretization (paper, Section 2.1 and Appendix C, with the curvilinear
mapping x(xi) of the element and its metric terms): per reference direction
xi_i the contravariant flux F^i = sum_n (J a^i)_n f_n enters the weak volume
term, the face flux is taken along the (unnormalized) vector J a^i of the
element that owns the +xi_i face, and the BR1 gradient carries the same
metric terms,
    J_j w_j g_{n,j} = sum_i [ - int (J a^i)_n q d(phi_j)/d xi_i + oint phi_j q_hat (J a^i)_n ].
(J a^i)_n is the conservative curl form of the metric identities, evaluated
with the GL derivative matrix on the element's own nodes, and J the
determinant of the discrete dx/dxi; the mass is J w_i w_j w_k per node.

Every function here takes fields of shape [..., Kz, Ky, Kx, P, P, P, 5] with
any number of leading batch axes, and real or complex values: the Jacobian is
built by complex-step differentiation of H (exact to rounding), many
directions at once.  The sparsity of A is the same as on Cartesian cubes (the
gradient still acts along xi-lines through a node, and the fluxes are
pointwise), so the same partition into A_ii, A_ib, A_bi and A_bb applies.

Columns are probed in colour classes: elements whose (ix, iy, iz) agree
modulo m, with m >= 3 a divisor of K (or m = K).  A column of element c
reaches rows in c and in its face and edge neighbours only, so two elements
of one class, at least three elements apart along some axis, never write to
the same row and one evaluation of H per local DOF serves the whole class.
"""
from __future__ import annotations

import numpy as np
import torch

from . import gl
from .dgsem import Mesh
from .physics import FlowParams, flux_adv, primitives, viscous_flux_of, viscous_stress

CS_STEP = 1e-30

# axes counted from the right, so that leading batch axes pass through
_NODE = {0: -2, 1: -3, 2: -4}     # node axis of direction d (x, y, z) in [..., P, P, P, 5]
_ELEM = {0: -5, 1: -6, 2: -7}     # element axis of direction d


def _along(a: torch.Tensor, d: int) -> torch.Tensor:
    """Node axis of direction d next to the last axis: [..., P, last]."""
    return a.movedim(_NODE[d], -2)


def _back(a: torch.Tensor, d: int) -> torch.Tensor:
    return a.movedim(-2, _NODE[d])


def _shift(a: torch.Tensor, d: int, step: int) -> torch.Tensor:
    """Field of the element step elements further along d (periodic)."""
    return torch.roll(a, -step, dims=_ELEM[d])


def _d_along(a: torch.Tensor, axis: int, dm: torch.Tensor) -> torch.Tensor:
    """GL derivative of a [..., P, P, P] node field along one node axis."""
    return (dm @ a.movedim(axis, -1).unsqueeze(-1)).squeeze(-1).movedim(-1, axis)


def metric_terms(xyz: torch.Tensor, order: int):
    """(J a^i)_n in curl form and J from node positions xyz [K, K, K, P, P, P, 3].

    With X the element's nodes, shifted to its first node, and (n, m, l) cyclic:
    (J a^i)_n = -e_i . curl_xi(X_l grad_xi X_m).  Returns ja [..., 3 (i), 3 (n)]
    and jac [...]; raises if J <= 0 anywhere."""
    x, _ = gl.gl_nodes_weights(order)
    dm = torch.tensor(gl.derivative_matrix(order), dtype=torch.float64, device=xyz.device)
    X = xyz - xyz[:, :, :, :1, :1, :1, :]
    node_ax = {0: 5, 1: 4, 2: 3}              # xi_j along node axis 5 - j of a [K,K,K,P,P,P] field
    dX = torch.stack([torch.stack([_d_along(X[..., m], node_ax[j], dm) for m in range(3)], dim=-1)
                      for j in range(3)], dim=-2)                       # [..., j, m] = dX_m / dxi_j
    ja = torch.zeros(X.shape[:-1] + (3, 3), dtype=torch.float64, device=xyz.device)
    for n in range(3):
        m, l = (n + 1) % 3, (n + 2) % 3
        v = X[..., l][..., None] * dX[..., :, m]                         # v_j = X_l dX_m / dxi_j
        for i in range(3):
            j, k = (i + 1) % 3, (i + 2) % 3
            ja[..., i, n] = -(_d_along(v[..., k], node_ax[j], dm) - _d_along(v[..., j], node_ax[k], dm))
    jac = torch.linalg.det(dX)
    if bool((jac <= 0).any()):
        raise ValueError("mapping is not invertible: J <= 0 at some node")
    return ja, jac


class CurvedGeometry:
    """Metric terms, Jacobian determinant and nodal mass of a curved mesh."""

    def __init__(self, mesh: Mesh, xyz, device="cpu"):
        xyz = torch.as_tensor(np.asarray(xyz), dtype=torch.float64, device=device)
        if tuple(xyz.shape) != mesh.shape()[:-1] + (3,):
            raise ValueError(f"xyz: expected shape {mesh.shape()[:-1] + (3,)}")
        self.mesh = mesh
        self.xyz = xyz
        self.ja, self.jac = metric_terms(xyz, mesh.order)
        _, w = gl.gl_nodes_weights(mesh.order)
        w = torch.tensor(w, dtype=torch.float64, device=device)
        self.w = w
        self.mass = self.jac * (w[:, None, None] * w[None, :, None] * w[None, None, :])
        dm = torch.tensor(gl.derivative_matrix(mesh.order), dtype=torch.float64, device=device)
        self.vw = -(dm.T) * w[None, :]                                   # vw[l, a] = -w_a D[a, l]
        self.wt = w[:, None] * w[None, :]                                # transverse weights


def wall_ghost(q: torch.Tensor, prm: FlowParams, t_wall: float) -> torch.Tensor:
    """Outer state of an isothermal no-slip wall (the Dirichlet condition
    q^-(q^+) of Section 2.1.1): density kept, momentum reversed,
    rho E^- = 2 rho e_w - rho E^+ (e_w: internal energy at t_wall), so that
    1/2 (q^+ + q^-) is the wall state (at rest, temperature t_wall)."""
    e_w = t_wall / (prm.gamma * (prm.gamma - 1.0) * prm.mach ** 2)
    return torch.stack([q[..., 0], -q[..., 1], -q[..., 2], -q[..., 3], 2.0 * e_w * q[..., 0] - q[..., 4]],
                       dim=-1)


def _with_walls(face: torch.Tensor, d: int, wall_lo, wall_hi) -> torch.Tensor:
    """Replace the face values [..., Kz, Ky, Kx, P, P, 5] of the first (wall_lo)
    and last (wall_hi) element layers along d; None leaves a layer unchanged."""
    ax = _ELEM[d] + 1                       # face arrays lack the node axis of d
    parts = list(torch.unbind(face, dim=ax))
    if wall_lo is not None:
        parts[0] = wall_lo
    if wall_hi is not None:
        parts[-1] = wall_hi
    return torch.stack(parts, dim=ax)


def _layer(a: torch.Tensor, d: int, index: int, face: bool = True) -> torch.Tensor:
    """Elements at position `index` along d of a face array (face=True) or node field."""
    return a.select(_ELEM[d] + (1 if face else 0), index)


def _normal_speed(q: torch.Tensor, nh: torch.Tensor, prm: FlowParams) -> torch.Tensor:
    """|v . n_hat| + c, with |.| and its complex-step derivative through Re."""
    rho, u, v, w, p = primitives(q, prm)
    vn = u * nh[..., 0] + v * nh[..., 1] + w * nh[..., 2]
    avn = vn * torch.sign(vn.real) if vn.is_complex() else vn.abs()
    return avn + torch.sqrt(prm.gamma * p / rho)


def llf_normal(q_in: torch.Tensor, q_out: torch.Tensor, nvec: torch.Tensor, prm: FlowParams) -> torch.Tensor:
    """Rusanov flux along the unnormalized face vector nvec [..., 3], scaled by |nvec|."""
    s = torch.linalg.norm(nvec, dim=-1)
    nh = nvec / s[..., None]
    a, b = _normal_speed(q_in, nh, prm), _normal_speed(q_out, nh, prm)
    lam = torch.where(a.real >= b.real, a, b)
    f = sum(nvec[..., c, None] * (flux_adv(q_in, c, prm) + flux_adv(q_out, c, prm)) for c in range(3))
    return 0.5 * f - 0.5 * (lam * s)[..., None] * (q_out - q_in)


def lifted_gradient(q: torch.Tensor, geo: CurvedGeometry, walls=None, prm: FlowParams | None = None,
                    broken: bool = False):
    """BR1 gradient on curved elements: (dq/dx, dq/dy, dq/dz), each shaped like q.
    walls = (d, t_wall): isothermal no-slip walls on the domain faces normal to
    d, whose outer value is wall_ghost of the inner one (prm needed).
    broken=True: the element's own face values in place of the surface value
    {{q}}, which by summation by parts is the gradient of the element's own
    interpolant (no lifting)."""
    n = geo.mesh.order
    vw = geo.vw.to(q.dtype)
    wt = geo.wt[:, :, None, None]
    g = [torch.zeros_like(q) for _ in range(3)]
    for i in range(3):
        ql = _along(q, i)
        right = _along(_shift(q, i, +1), i)[..., 0, :]
        left = _along(_shift(q, i, -1), i)[..., n, :]
        if broken:
            right, left = ql[..., n, :], ql[..., 0, :]
        if walls is not None and walls[0] == i:
            right = _with_walls(right, i, None, wall_ghost(_layer(ql[..., n, :], i, -1), prm, walls[1]))
            left = _with_walls(left, i, wall_ghost(_layer(ql[..., 0, :], i, 0), prm, walls[1]), None)
        for c in range(3):
            jl = _along(geo.ja[..., i, c][..., None], i)                 # [K,K,K,P,P,P(l),1]
            t = (vw @ (jl * ql)) * wt
            t = t.clone()
            t[..., n, :] += geo.wt[:, :, None] * jl[..., n, :] * 0.5 * (ql[..., n, :] + right)
            t[..., 0, :] -= geo.wt[:, :, None] * jl[..., 0, :] * 0.5 * (ql[..., 0, :] + left)
            g[c] = g[c] + _back(t, i)
    m = geo.mass[..., None]
    return tuple(gc / m for gc in g)


SIPG_ETA = 1.0


def operator_h(q: torch.Tensor, geo: CurvedGeometry, prm: FlowParams, walls=None,
               viscous: str = "br1") -> torch.Tensor:
    """H(Q) on curved elements (mass-weighted, same shape as q).  walls = (d,
    t_wall): on the two wall faces normal to d the face flux is the
    Lax-Friedrichs flux between the inner state and its wall_ghost minus the
    viscous flux of the wall state 1/2 (q^+ + q^-) with the inner gradient,
    along the face vector J a^d of the element itself.  viscous="sipg": the face viscous flux is
    the symmetric interior penalty flux of a Cartesian mesh, the average of each
    side's viscous flux with its own broken gradient plus sigma times the
    viscous flux of the mean state applied to the jump taken as a gradient
    along the face normal, sigma = eta (N + 1)^2 / h (walls not supported)."""
    if viscous not in ("br1", "sipg") or (viscous == "sipg" and walls is not None):
        raise ValueError(f"viscous flux {viscous} with walls={walls}")
    n = geo.mesh.order
    vw = geo.vw.to(q.dtype)
    wt = geo.wt[:, :, None, None]
    g = lifted_gradient(q, geo, walls, prm)
    gb = lifted_gradient(q, geo, broken=True) if viscous == "sipg" else None
    sigma = SIPG_ETA * (n + 1) ** 2 / geo.mesh.h
    st = viscous_stress(q, g, prm)
    f = [flux_adv(q, c, prm) - viscous_flux_of(st, c, prm) for c in range(3)]
    h = torch.zeros_like(q)
    for i in range(3):
        ft = sum(geo.ja[..., i, c][..., None] * f[c] for c in range(3))
        t = (vw @ _along(ft, i)) * wt
        q_in = _along(q, i)[..., n, :]
        q_out = _along(_shift(q, i, +1), i)[..., 0, :]
        g_in = tuple(_along(gc, i)[..., n, :] for gc in g)
        g_out = tuple(_along(_shift(gc, i, +1), i)[..., 0, :] for gc in g)
        nvec = _along(geo.ja[..., i, :], i)[..., n, :]                   # (J a^i) at the +xi_i face nodes
        if viscous == "sipg":
            g_in = tuple(_along(gc, i)[..., n, :] for gc in gb)
            g_out = tuple(_along(_shift(gc, i, +1), i)[..., 0, :] for gc in gb)
        st_in, st_out = viscous_stress(q_in, g_in, prm), viscous_stress(q_out, g_out, prm)
        visc = sum(nvec[..., c, None] * (viscous_flux_of(st_in, c, prm) + viscous_flux_of(st_out, c, prm))
                   for c in range(3))
        if viscous == "sipg":
            nh = nvec / torch.linalg.norm(nvec, dim=-1)[..., None]
            jump = q_out - q_in
            st_p = viscous_stress(0.5 * (q_in + q_out), tuple(nh[..., c, None] * jump for c in range(3)), prm)
            visc = visc + 2.0 * sigma * sum(nvec[..., c, None] * viscous_flux_of(st_p, c, prm) for c in range(3))
        f_hat = llf_normal(q_in, q_out, nvec, prm) - 0.5 * visc
        f_left = torch.roll(f_hat, 1, dims=_ELEM[i] + 1)                 # face arrays lack the d node axis
        if walls is not None and walls[0] == i:
            fw = []
            for l, idx in ((n, -1), (0, 0)):
                qi = _layer(_along(q, i)[..., l, :], i, idx)
                gi = tuple(_layer(_along(gc, i)[..., l, :], i, idx) for gc in g)
                nv = _layer(_along(geo.ja[..., i, :], i)[..., l, :], i, idx)
                qg = wall_ghost(qi, prm, walls[1])
                adv = llf_normal(qi, qg, nv, prm) if l == n else llf_normal(qg, qi, nv, prm)
                stw = viscous_stress(0.5 * (qi + qg), gi, prm)
                fw.append(adv - sum(nv[..., c, None] * viscous_flux_of(stw, c, prm) for c in range(3)))
            f_hat = _with_walls(f_hat, i, None, fw[0])
            f_left = _with_walls(f_left, i, fw[1], None)
        t = t.clone()
        t[..., n, :] += geo.wt[:, :, None] * f_hat
        t[..., 0, :] -= geo.wt[:, :, None] * f_left
        h = h + _back(t, i)
    return h


def _colour_modulus(k: int) -> int:
    for m in range(3, k + 1):
        if k % m == 0:
            return m
    return k


class CurvedJacobianParts:
    """A = M/dt + dH/dQ on a curved mesh as dense own blocks plus node-block
    couplings to other elements (the input format of the block partition)."""

    def __init__(self, q: torch.Tensor, geo: CurvedGeometry, prm: FlowParams, dt: float,
                 max_batch: int | None = None, walls=None, progress=None, viscous: str = "br1"):
        mesh = geo.mesh
        self.mesh, self.prm, self.dt, self.device = mesh, prm, dt, q.device
        k, p = mesh.k_elem, mesh.p
        p3, ne = p ** 3, mesh.n_elem
        nloc = 5 * p3
        q = q.reshape(mesh.shape()).to(torch.float64)
        # colour moduli per direction (x, y, z): a divisor >= 3 of K where the mesh
        # wraps around, any m >= 3 across walls (elements there do not wrap)
        mods = [3 if (walls is not None and walls[0] == d and k >= 3) else _colour_modulus(k) for d in range(3)]
        dev = q.device
        idx = torch.arange(k, device=dev)
        iz, iy, ix = torch.meshgrid(idx, idx, idx, indexing="ij")
        colour = ((iz % mods[2]) * mods[1] + (iy % mods[1])) * mods[0] + (ix % mods[0])
        colour = colour.reshape(-1)
        n_colours = mods[0] * mods[1] * mods[2]
        # distinct neighbour offsets after the periodic wrap
        offs, seen = [], set()
        for oz in (-1, 0, 1):
            for oy in (-1, 0, 1):
                for ox in (-1, 0, 1):
                    key = (oz % k, oy % k, ox % k)
                    if key == (0, 0, 0) or key in seen:
                        continue
                    seen.add(key)
                    offs.append((oz, oy, ox))
        ez, ey, ex = (t.reshape(-1) for t in (iz, iy, ix))
        nbr = [((ez + oz) % k * k + (ey + oy) % k) * k + (ex + ox) % k for oz, oy, ox in offs]
        if max_batch is None:
            max_batch = max(1, int(4e8 // (16 * mesh.n_dof * 24)))
        self.own = torch.zeros((ne, nloc, nloc), dtype=torch.float64, device=dev)
        rows, cols, vals = [], [], []
        nid = torch.arange(ne * p3, device=dev).reshape(ne, p3)
        qc = q.to(torch.complex128)
        for col in range(n_colours):
            elems = torch.nonzero(colour == col).reshape(-1)
            if progress is not None:
                progress(col, n_colours)
            if elems.numel() == 0:
                continue
            for j0 in range(0, nloc, max_batch):
                j1 = min(nloc, j0 + max_batch)
                b = j1 - j0
                x = qc.expand((b,) + tuple(qc.shape)).clone().reshape(b, ne, p3 * 5)
                jj = torch.arange(j0, j1, device=dev)
                x[jj[:, None] - j0, elems[None, :], jj[:, None]] += 1j * CS_STEP
                hd = operator_h(x.reshape((b,) + mesh.shape()), geo, prm, walls, viscous).imag / CS_STEP
                hd = hd.reshape(b, ne, p3 * 5)                           # [cols j, row elem, row (n, v)]
                self.own[elems, :, j0:j1] = hd[:, elems, :].permute(1, 2, 0)
                for nb in nbr:
                    blk = hd[:, nb[elems], :]                            # [b, |C|, p3 * 5]
                    blk = blk.reshape(b, elems.numel(), p3, 5)
                    cn, cv = jj // 5, jj % 5
                    # [|C|, row node, col local j] -> node blocks
                    nzr = torch.nonzero(blk.abs().amax(-1) != 0, as_tuple=False)   # (j, c, row node)
                    if nzr.numel() == 0:
                        continue
                    rows.append(nid[nb[elems][nzr[:, 1]], nzr[:, 2]])
                    cols.append(nid[elems[nzr[:, 1]], cn[nzr[:, 0]]])
                    v = torch.zeros((nzr.shape[0], 5, 5), dtype=torch.float64, device=dev)
                    v[torch.arange(nzr.shape[0], device=dev), :, cv[nzr[:, 0]]] = \
                        blk[nzr[:, 0], nzr[:, 1], nzr[:, 2], :]
                    vals.append(v)
        mass = (geo.mass / dt).reshape(ne, p3)
        diag = torch.arange(nloc, device=dev)
        self.own[:, diag, diag] += mass.repeat_interleave(5, dim=1)
        r, c, v = torch.cat(rows), torch.cat(cols), torch.cat(vals)
        nn = ne * p3
        uk, inv = torch.unique(r * nn + c, sorted=True, return_inverse=True)
        out = torch.zeros((uk.numel(), 5, 5), dtype=torch.float64, device=dev)
        out.index_add_(0, inv, v)
        self._coupl = (uk // nn, uk % nn, out)

    def own_blocks(self, e0: int, e1: int) -> torch.Tensor:
        return self.own[e0:e1]

    def couplings(self):
        return self._coupl

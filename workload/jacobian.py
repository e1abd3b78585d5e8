"""Analytic Jacobian dH/dQ of the BR1 / local-Lax-Friedrichs GL-DGSEM residual.

The paper builds the implicit-step Jacobian analytically from pointwise flux
Jacobians and the linear DGSEM operators (Sections 2.1.1 and 2.1.2: advective
and diffusive linearizations; the lifted gradient enters through eq. GradDGImp).
This module does the same by the chain rule, with two choices of its own:

  * the pointwise Jacobians  Ja_d = df^a_d/dq,  Jv_d = df^nu_d/dq (g fixed),
    G_dd' = df^nu_d/dg_d'  and the LLF face Jacobians are taken by complex-step
    differentiation of the flux functions (exact to rounding, and independent
    of the printed Appendix B matrices, which carry typos);
  * the result is produced per element: a dense "own" block (all columns in
    the element itself) plus a list of node-block couplings to other elements.

Notation (direction d, line index l along d, transverse nodes t = (t1, t2)):
  c_t       = J s w_t1 w_t2            (s = 2/h)
  Vw[l, a]  = -w_a D[a, l]             (weak volume operator)
  bhat[l,a] = Vw[l,a] + (1/2) delta_{lN} delta_{aN} - (1/2) delta_{l0} delta_{a0}
  Lloc[b,b']= s (D[b,b'] - delta_{bN}delta_{b'N}/(2 w_N) + delta_{b0}delta_{b'0}/(2 w_0))
The BR1 viscous part of row r is  -sum_m beta_rm f^nu_d(q_m, g_m)  with
beta = c_t bhat on the element's own d-line and beta = +-c_t/2 at the neighbour
face node; g_d'(m) = sum_n L_d'[m, n] q_n is the lifting operator (Lloc along
the d'-line plus +-s/(2w) to the node across a d'-face).
"""
from __future__ import annotations

import numpy as np
import torch

from . import gl
from .dgsem import Mesh, elem_axis, node_axis, lifted_gradient
from .physics import FlowParams, flux_adv, flux_visc, llf_flux

CS_STEP = 1e-30


def _cs_jacobian(fun, x: torch.Tensor, nin: int) -> torch.Tensor:
    """Complex-step Jacobian of fun w.r.t. the last axis of x: [..., nout, nin]."""
    cols = []
    xc = x.to(torch.complex128)
    for k in range(nin):
        xp = xc.clone()
        xp[..., k] = xp[..., k] + 1j * CS_STEP
        cols.append(fun(xp).imag / CS_STEP)
    return torch.stack(cols, dim=-1)


def pointwise_jacobians(q: torch.Tensor, mesh: Mesh, prm: FlowParams):
    """Ja[d], Jv[d], G[d][d'] at every node and LLF PL[d], PR[d] at every +e_d face.

    Node tensors have shape [Kz, Ky, Kx, P, P, P, 5, 5]; face tensors
    [Kz, Ky, Kx, P, P, 5, 5] indexed by the two transverse node indices in
    their natural order (the d axis removed).
    """
    g = lifted_gradient(q, mesh)
    gcat = torch.cat(g, dim=-1)                                       # [..., 15]
    ja, jv, gg, pl, pr = [], [], [], [], []
    n = mesh.order
    for d in range(3):
        ja.append(_cs_jacobian(lambda z: flux_adv(z, d, prm), q, 5))
        jv.append(_cs_jacobian(lambda z: flux_visc(z, g, d, prm), q, 5))
        full = _cs_jacobian(lambda z: flux_visc(q.to(z.dtype), (z[..., 0:5], z[..., 5:10], z[..., 10:15]), d, prm),
                            gcat, 15)
        gg.append([full[..., 5 * dp:5 * dp + 5] for dp in range(3)])
        qm = q.movedim(node_axis(d), -2)
        ql = qm[..., n, :]
        qr = torch.roll(qm, -1, dims=elem_axis(d))[..., 0, :]
        pl.append(_cs_jacobian(lambda z: llf_flux(z, qr.to(z.dtype), d, prm), ql, 5))
        pr.append(_cs_jacobian(lambda z: llf_flux(ql.to(z.dtype), z, d, prm), qr, 5))
    return ja, jv, gg, pl, pr


class _Ops:
    def __init__(self, mesh: Mesh, device):
        x, w = gl.gl_nodes_weights(mesh.order)
        dm = gl.derivative_matrix(mesh.order)
        n = mesh.order
        s = mesh.scale
        vw = -(dm.T) * w[None, :]
        bhat = vw.copy()
        bhat[n, n] += 0.5
        bhat[0, 0] -= 0.5
        lloc = s * dm.copy()
        lloc[n, n] -= s / (2 * w[n])
        lloc[0, 0] += s / (2 * w[0])
        t = lambda a: torch.tensor(a, dtype=torch.float64, device=device)
        self.w, self.vw, self.bhat, self.lloc = t(w), t(vw), t(bhat), t(lloc)
        self.n = n
        self.s = s
        self.jac = mesh.jac
        self.lnbr_hi = s / (2 * w[n])       # coefficient to (E+, 0) from b = N
        self.lnbr_lo = -s / (2 * w[0])      # coefficient to (E-, N) from b = 0


def _canon(x: torch.Tensor, d: int, dp: int | None = None) -> torch.Tensor:
    """Reorder node axes of a node tensor [Kz,Ky,Kx,P,P,P,...] to [..., t1, t2, l, ...].

    With dp given, t1 is the node axis of direction dp and t2 the remaining one.
    """
    la = node_axis(d)
    if dp is None:
        others = [a for a in (3, 4, 5) if a != la]
    else:
        others = [node_axis(dp)] + [a for a in (3, 4, 5) if a not in (la, node_axis(dp))]
    rest = list(range(6, x.dim()))
    return x.permute(0, 1, 2, others[0], others[1], la, *rest)


def _canon_flat(x: torch.Tensor, d: int, dp: int | None = None) -> torch.Tensor:
    """Same as _canon for element-flattened node tensors [E, P, P, P, ...]."""
    la = 3 - d
    if dp is None:
        others = [a for a in (1, 2, 3) if a != la]
    else:
        others = [3 - dp] + [a for a in (1, 2, 3) if a not in (la, 3 - dp)]
    rest = list(range(4, x.dim()))
    return x.permute(0, others[0], others[1], la, *rest)


def _face_canon(f: torch.Tensor, d: int, dp: int | None = None) -> torch.Tensor:
    """Face tensor [Kz,Ky,Kx,Pa,Pb,...] (transverse axes in natural order) to [..., t1, t2, ...]."""
    la = node_axis(d)
    nat = [a for a in (3, 4, 5) if a != la]           # natural transverse node axes
    if dp is None or nat[0] == node_axis(dp):
        return f
    return f.transpose(3, 4)


class JacobianParts:
    """Own dense blocks (per element chunk) and inter-element node-block couplings."""

    def __init__(self, q: torch.Tensor, mesh: Mesh, prm: FlowParams, dt: float):
        self.mesh, self.prm, self.dt = mesh, prm, dt
        self.device = q.device
        self.ops = _Ops(mesh, q.device)
        self.ja, self.jv, self.gg, self.pl, self.pr = pointwise_jacobians(q, mesh, prm)
        from .dgsem import mass_diagonal
        self.mass = torch.tensor(mass_diagonal(mesh), device=q.device)

    # ---------------------------------------------------------------- own
    def own_blocks(self, e0: int, e1: int) -> torch.Tensor:
        """Dense d H_e / d q_e (+ M/dt) for flattened elements [e0, e1): [E', P^3*5, P^3*5]."""
        mesh, o = self.mesh, self.ops
        k, p, n = mesh.k_elem, mesh.p, mesh.order
        ne = e1 - e0
        dev = self.device
        a_own = torch.zeros((ne, p, p, p, 5, p, p, p, 5), dtype=torch.float64, device=dev)
        def flat(x, dd, dp=None):
            x = x.reshape((k ** 3,) + tuple(x.shape[3:]))[e0:e1]
            return _canon_flat(x, dd, dp)

        def flat_face(x, dd, dp=None):
            x = _face_canon(x, dd, dp)
            return x.reshape((k ** 3,) + tuple(x.shape[3:]))[e0:e1]
        w = o.w
        for d in range(3):
            ea = elem_axis(d)
            # ---- same-line terms: rows (t1,t2,l), cols (t1,t2,a')
            ct = o.jac * o.s * (w[:, None] * w[None, :])                  # [t1, t2]
            ja = flat(self.ja[d], d)                               # [E, t1, t2, a, 5, 5]
            jv = flat(self.jv[d], d)
            gdd = flat(self.gg[d][d], d)
            t_same = torch.einsum('la,etuavw->etulavw', o.vw, ja)
            t_same -= torch.einsum('la,etuavw->etulavw', o.bhat, jv)
            t_same -= torch.einsum('lb,etubvw,ba->etulavw', o.bhat, gdd, o.lloc)
            t_same *= ct[None, :, :, None, None, None, None]
            # own face advective terms and the back-coupling through the neighbour's gradient
            pl_r = flat_face(self.pl[d], d)                        # [E, t1, t2, 5, 5]
            pr_l = flat_face(torch.roll(self.pr[d], 1, dims=ea), d)
            g_nb_r = flat(torch.roll(self.gg[d][d], -1, dims=ea), d)[:, :, :, 0]
            g_nb_l = flat(torch.roll(self.gg[d][d], 1, dims=ea), d)[:, :, :, n]
            ctv = ct[None, :, :, None, None]
            t_same[:, :, :, n, n] += ctv * (pl_r + (o.s / (4 * float(w[0]))) * g_nb_r)
            t_same[:, :, :, 0, 0] += ctv * (-pr_l + (o.s / (4 * float(w[n]))) * g_nb_l)
            la = 3 - d                 # node axis of d within a_own rows (1 = k, 2 = j, 3 = i)
            others = [a for a in (1, 2, 3) if a != la]
            view = a_own.permute(0, others[0], others[1], la, 4, others[0] + 4, others[1] + 4, la + 4, 8)
            d1 = torch.diagonal(view, 0, 1, 5)                             # [E, t2, l, v, t2', a', v', t1]
            d2 = torch.diagonal(d1, 0, 1, 4)                               # [E, l, v, a', v', t1, t2]
            d2 += t_same.permute(0, 3, 5, 4, 6, 1, 2)
            del t_same, ja, jv
            # ---- plane terms d' != d: rows (b, c, l), cols (b', c, a)
            for dp in range(3):
                if dp == d:
                    continue
                g = flat(self.gg[d][dp], d, dp)                            # [E, b, c, a, 5, 5]
                ctp = o.jac * o.s * (w[:, None] * w[None, :])              # [b, c]
                t_pl = torch.einsum('la,bq,ebcavw->ebclaqvw', o.bhat, o.lloc, g)
                t_pl *= -ctp[None, :, :, None, None, None, None, None]
                lb = 3 - dp
                lc = [a for a in (1, 2, 3) if a not in (la, lb)][0]
                view = a_own.permute(0, lb, lc, la, 4, lb + 4, lc + 4, la + 4, 8)   # [E,b,c,l,v,b',c',a,v']
                dg = torch.diagonal(view, 0, 2, 6)                                  # [E,b,l,v,b',a,v',c]
                dg += t_pl.permute(0, 1, 3, 6, 5, 4, 7, 2)
                del t_pl
        # mass / dt on the diagonal
        m = self.mass.reshape(k ** 3, p, p, p)[e0:e1]                        # [E, k, j, i]
        diag = torch.diagonal(a_own.reshape(ne, p ** 3 * 5, p ** 3 * 5), 0, 1, 2)
        diag += (m.reshape(ne, p ** 3, 1).expand(ne, p ** 3, 5).reshape(ne, -1)) / self.dt
        return a_own.reshape(ne, p ** 3 * 5, p ** 3 * 5)

    # ---------------------------------------------------------- couplings
    def couplings(self):
        """Node-block couplings to other elements: (row node, col node, [5, 5] value), coalesced."""
        mesh, o = self.mesh, self.ops
        k, p, n = mesh.k_elem, mesh.p, mesh.order
        dev = self.device
        nid = torch.arange(k ** 3 * p ** 3, device=dev, dtype=torch.int64).reshape(k, k, k, p, p, p)
        w = o.w
        rows, cols, vals = [], [], []

        def emit(r, c, v):
            r = r.expand(v.shape[:-2]).reshape(-1)
            c = c.expand(v.shape[:-2]).reshape(-1)
            rows.append(r)
            cols.append(c)
            vals.append(v.reshape(-1, 5, 5))

        for d in range(3):
            ea = elem_axis(d)
            ct = o.jac * o.s * (w[:, None] * w[None, :])                  # [t1, t2]
            ctv = ct[None, None, None, :, :, None, None, None]             # broadcast to [.., t1, t2, l, 5, 5]
            nid_c = _canon(nid, d)                                         # [Kz,Ky,Kx,t1,t2,l]
            nid_p = _canon(torch.roll(nid, -1, dims=ea), d)                # node ids of element e+d
            nid_m = _canon(torch.roll(nid, 1, dims=ea), d)                 # node ids of element e-d
            gdd = _canon(self.gg[d][d], d)                                 # [K,K,K,t1,t2,l,5,5]
            # (N1) own m on the d-line at a in {0, N}, gradient across the d-face
            v_hi = -o.bhat[:, n][None, None, None, None, None, :, None, None] * ctv \
                * gdd[..., n:n + 1, :, :] * o.lnbr_hi
            emit(nid_c, nid_p[..., 0:1], v_hi)
            v_lo = -o.bhat[:, 0][None, None, None, None, None, :, None, None] * ctv \
                * gdd[..., 0:1, :, :] * o.lnbr_lo
            emit(nid_c, nid_m[..., n:n + 1], v_lo)
            # (N3) advective + direct viscous with the neighbour face node
            jv_p = _canon(torch.roll(self.jv[d], -1, dims=ea), d)[..., 0, :, :]   # Jv at (e+d, 0, t)
            jv_m = _canon(torch.roll(self.jv[d], 1, dims=ea), d)[..., n, :, :]    # Jv at (e-d, N, t)
            pr_r = _face_canon(self.pr[d], d)
            pl_l = _face_canon(torch.roll(self.pl[d], 1, dims=ea), d)
            ct2 = ct[None, None, None, :, :, None, None]
            emit(nid_c[..., n], nid_p[..., 0], ct2 * (pr_r - 0.5 * jv_p))
            emit(nid_c[..., 0], nid_m[..., n], ct2 * (-pl_l + 0.5 * jv_m))
            # (N4) neighbour m, gradient along the d-line inside the neighbour
            g_p = _canon(torch.roll(self.gg[d][d], -1, dims=ea), d)[..., 0, :, :]  # [K,K,K,t1,t2,5,5]
            g_m = _canon(torch.roll(self.gg[d][d], 1, dims=ea), d)[..., n, :, :]
            v = -0.5 * ct2[..., None, :, :] * g_p[..., None, :, :] * o.lloc[0][None, None, None, None, None, :, None, None]
            emit(nid_c[..., n:n + 1], nid_p, v)
            v = 0.5 * ct2[..., None, :, :] * g_m[..., None, :, :] * o.lloc[n][None, None, None, None, None, :, None, None]
            emit(nid_c[..., 0:1], nid_m, v)
            for dp in range(3):
                if dp == d:
                    continue
                eap = elem_axis(dp)
                nid_c2 = _canon(nid, d, dp)                                 # [K,K,K,b,c,l]
                g = _canon(self.gg[d][dp], d, dp)                           # [K,K,K,b,c,a,5,5]
                ctp = (o.jac * o.s * (w[:, None] * w[None, :]))[None, None, None, :, :, None, None, None]
                # (N2) own m, gradient across a dp-face of e (rows with b in {0, N})
                for b, shift, nb_b, coef in ((n, -1, 0, o.lnbr_hi), (0, 1, n, o.lnbr_lo)):
                    nid_x = _canon(torch.roll(nid, shift, dims=eap), d, dp)[..., nb_b, :, :]   # [K,K,K,c,a]
                    # value[.., c, l, a] = -c_t bhat[l, a] G(e, a, b, c) coef
                    gb_ = g[..., b, :, :, :, :]                                             # [K,K,K,c,a,5,5]
                    val = -(ctp[..., b, :, :, :, :][..., None, :, :]) * coef \
                        * o.bhat[None, None, None, None, :, :, None, None] * gb_[..., None, :, :, :]
                    # val: [K,K,K,c,l,a,5,5]
                    emit(nid_c2[..., b, :, :][..., :, :, None], nid_x[..., :, None, :], val)
                # (N5) neighbour m at the d-face, gradient along / across dp inside the neighbour
                for l_row, shift, lm, sgn in ((n, -1, 0, 0.5), (0, 1, n, -0.5)):
                    gnb = _canon(torch.roll(self.gg[d][dp], shift, dims=ea), d, dp)[..., lm, :, :]   # [K,K,K,b,c,5,5]
                    nid_nb = _canon(torch.roll(nid, shift, dims=ea), d, dp)[..., lm]                 # [K,K,K,b',c]
                    beta = sgn * (o.jac * o.s * (w[:, None] * w[None, :]))                          # [b, c]
                    # along the dp line: rows (b, c), cols (b', c)
                    val = -beta[None, None, None, :, :, None, None, None] * gnb[..., :, :, None, :, :] \
                        * o.lloc[None, None, None, :, None, :, None, None]                            # [K,K,K,b,c,b',5,5]
                    rr = nid_c2[..., l_row][..., :, :, None]                                        # [K,K,K,b,c,1]
                    cc = nid_nb.transpose(3, 4)[..., None, :, :]                                    # [K,K,K,1,c,b']
                    emit(rr, cc, val)
                    # across a dp-face of the neighbour (b in {0, N})
                    for b, shift2, nb_b, coef in ((n, -1, 0, o.lnbr_hi), (0, 1, n, o.lnbr_lo)):
                        nid_nn = _canon(torch.roll(torch.roll(nid, shift, dims=ea), shift2, dims=eap), d, dp)[..., nb_b, :, lm]  # [K,K,K,c]
                        val = -beta[b][None, None, None, :, None, None] * coef * gnb[..., b, :, :, :]   # [K,K,K,c,5,5]
                        emit(nid_c2[..., b, :, l_row], nid_nn, val)
        r = torch.cat(rows)
        c = torch.cat(cols)
        v = torch.cat(vals)
        nn = k ** 3 * p ** 3
        key = r * nn + c
        uk, inv = torch.unique(key, sorted=True, return_inverse=True)
        out = torch.zeros((uk.numel(), 5, 5), dtype=torch.float64, device=dev)
        out.index_add_(0, inv, v)
        return uk // nn, uk % nn, out

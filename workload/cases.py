"""Seeded synthetic implicit-step systems A dQ = B of the GL-DGSEM.

One case = a periodic Cartesian K^3 hex mesh of order N on [0, 2 pi)^3, a
Taylor-Green-like state with a seeded 1e-3 perturbation (Q_s), and the
backward-Euler Newton system at the first Newton iterate Q~ = Q_s
(paper, eq. ImplicitDisc / NewtonLinSys1):
    A = M / dt + dH/dQ (Q_s),      B = -R(Q_s) = -H(Q_s).

The named workloads mirror the paper's use of a steady viscous flow with the
compressible Navier-Stokes equations (its Section 4 cylinder mesh is not
available; these synthetic states stand in for it):
  tgv_n3_k2   : 2^3 elements, N = 3, Re 100,  dt 1e-2   (2 560 DOFs)
  tgv_n5_k8   : 8^3 elements, N = 5, Re 1600, dt 5e-3   (552 960 DOFs)
  tgv_n7_k8   : 8^3 elements, N = 7, Re 1600, dt 5e-3   (1 310 720 DOFs)
  tgv_n4_k16  : 16^3 elements, N = 4, Re 1600, dt 5e-3  (2 560 000 DOFs)
all at Ma = 0.1, gamma = 1.4, Pr = 0.72, Sutherland viscosity.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from .curved import CurvedGeometry, CurvedJacobianParts, operator_h
from .dgsem import Mesh, curved_node_coordinates, mass_diagonal, residual, taylor_green_state, uniform_state
from .jacobian import JacobianParts
from .partition import partition
from .physics import FlowParams

WORKLOADS = {
    "tgv_n3_k2": dict(k_elem=2, order=3, reynolds=100.0, dt=1e-2),
    "tgv_n5_k8": dict(k_elem=8, order=5, reynolds=1600.0, dt=5e-3),
    "tgv_n7_k8": dict(k_elem=8, order=7, reynolds=1600.0, dt=5e-3),
    "tgv_n4_k16": dict(k_elem=16, order=4, reynolds=1600.0, dt=5e-3),
}


@dataclass
class Case:
    mesh: Mesh
    prm: FlowParams
    dt: float
    seed: int
    order: np.ndarray            # [E] int32
    c_ptr: np.ndarray            # [E+1] int64
    c_node: np.ndarray           # int32
    bb_rowptr: np.ndarray        # [n_bnodes+1] int64
    bb_col: np.ndarray           # int32
    bb_val: torch.Tensor         # [nnzb, 5, 5] float64
    aii: torch.Tensor            # [E, n_i, n_i]
    aib: torch.Tensor            # [E, n_i, n_c]
    abi: torch.Tensor            # [E, n_c, n_i]
    rhs: torch.Tensor            # [n_dof] natural order
    mass: np.ndarray             # [E * P^3] node mass J w_i w_j w_k
    n_i: int
    n_c: int
    n_bnodes: int
    q_state: torch.Tensor | None = None
    parts: JacobianParts | None = field(default=None, repr=False)
    xyz: np.ndarray | None = None  # node positions [K, K, K, P, P, P, 3] of a curved mesh

    @property
    def n_elem(self) -> int:
        return self.mesh.n_elem

    @property
    def n_dof(self) -> int:
        return self.mesh.n_dof

    @property
    def n1(self) -> int:
        return 5 * self.n_bnodes

    @property
    def n2(self) -> int:
        return self.n_elem * self.n_i

    def structure(self) -> dict:
        return dict(order=self.order, c_ptr=self.c_ptr, c_node=self.c_node,
                    bb_rowptr=self.bb_rowptr, bb_col=self.bb_col)

    def to(self, device) -> "Case":
        mv = lambda t: None if t is None else t.to(device)
        return Case(self.mesh, self.prm, self.dt, self.seed, self.order, self.c_ptr, self.c_node,
                    self.bb_rowptr, self.bb_col, mv(self.bb_val), mv(self.aii), mv(self.aib),
                    mv(self.abi), mv(self.rhs), self.mass, self.n_i, self.n_c, self.n_bnodes,
                    mv(self.q_state), None, self.xyz)


def build_case(k_elem: int, order: int, reynolds: float, dt: float, mach: float = 0.1,
               seed: int = 0, device="cpu", state: str = "tgv", keep_parts: bool = False,
               chunk: int | None = None) -> Case:
    if k_elem < 2:
        raise ValueError("need at least 2 elements per direction")
    if order < 2:
        raise ValueError("static condensation needs interior nodes: N >= 2")
    mesh = Mesh(k_elem, order)
    prm = FlowParams(mach=mach, reynolds=reynolds)
    if state == "tgv":
        q0 = taylor_green_state(mesh, prm, seed)
    elif state == "uniform":
        q0 = uniform_state(mesh, prm)
    else:
        raise ValueError(state)
    q = torch.tensor(q0, dtype=torch.float64, device=device)
    h = residual(q, mesh, prm)
    parts = JacobianParts(q, mesh, prm, dt)
    if chunk is None:
        per_elem = (mesh.p ** 3 * 5) ** 2 * 8
        chunk = max(1, min(mesh.n_elem, int(2e9 // per_elem)))
    blk = partition(parts, chunk=chunk)
    return Case(mesh=mesh, prm=prm, dt=dt, seed=seed,
                order=np.full(mesh.n_elem, order, dtype=np.int32),
                c_ptr=blk["c_ptr"], c_node=blk["c_node"],
                bb_rowptr=blk["bb_rowptr"], bb_col=blk["bb_col"], bb_val=blk["bb_val"],
                aii=blk["aii"], aib=blk["aib"], abi=blk["abi"],
                rhs=(-h).reshape(-1).contiguous(),
                mass=mass_diagonal(mesh).reshape(-1),
                n_i=blk["n_i"], n_c=blk["n_c"], n_bnodes=blk["n_bnodes"],
                q_state=q, parts=parts if keep_parts else None)


def jacobian_blocks(q: torch.Tensor, mesh: Mesh, prm: FlowParams, dt: float, chunk: int | None = None) -> dict:
    """Backward-Euler Jacobian A = M/dt + dH/dQ at state q (natural DOF order or
    mesh layout, on q's device) as per-element blocks: aii, aib, abi, bb_val."""
    q = q.reshape(mesh.shape())
    parts = JacobianParts(q, mesh, prm, dt)
    if chunk is None:
        per_elem = (mesh.p ** 3 * 5) ** 2 * 8
        chunk = max(1, min(mesh.n_elem, int(2e9 // per_elem)))
    blk = partition(parts, chunk=chunk)
    return dict(aii=blk["aii"], aib=blk["aib"], abi=blk["abi"], bb_val=blk["bb_val"])


def _chunk(mesh: Mesh) -> int:
    per_elem = (mesh.p ** 3 * 5) ** 2 * 8
    return max(1, min(mesh.n_elem, int(2e9 // per_elem)))


def build_curved_case(k_elem: int, order: int, reynolds: float, dt: float, mach: float = 0.1,
                      seed: int = 0, device="cpu", amplitude: float = 0.05, kind: str = "sine") -> Case:
    """The same system on the periodic perturbed mesh of curved_node_coordinates
    (kind "sine" or "skew"): the Taylor-Green state evaluated at the curved
    nodes, A = M/dt + dH/dQ(Q_s) with the curved H and mass J w_i w_j w_k,
    B = -H(Q_s).  The node positions are kept in case.xyz."""
    if k_elem < 2:
        raise ValueError("need at least 2 elements per direction")
    if order < 2:
        raise ValueError("static condensation needs interior nodes: N >= 2")
    mesh = Mesh(k_elem, order)
    prm = FlowParams(mach=mach, reynolds=reynolds)
    xyz = curved_node_coordinates(mesh, amplitude, kind)
    q = torch.tensor(taylor_green_state(mesh, prm, seed, coords=xyz), dtype=torch.float64, device=device)
    geo = CurvedGeometry(mesh, xyz, device=device)
    h = operator_h(q, geo, prm)
    blk = partition(CurvedJacobianParts(q, geo, prm, dt), chunk=_chunk(mesh))
    return Case(mesh=mesh, prm=prm, dt=dt, seed=seed,
                order=np.full(mesh.n_elem, order, dtype=np.int32),
                c_ptr=blk["c_ptr"], c_node=blk["c_node"],
                bb_rowptr=blk["bb_rowptr"], bb_col=blk["bb_col"], bb_val=blk["bb_val"],
                aii=blk["aii"], aib=blk["aib"], abi=blk["abi"],
                rhs=(-h).reshape(-1).contiguous(),
                mass=geo.mass.reshape(-1).cpu().numpy(),
                n_i=blk["n_i"], n_c=blk["n_c"], n_bnodes=blk["n_bnodes"],
                q_state=q, xyz=xyz)


def curved_jacobian_blocks(q: torch.Tensor, geo: CurvedGeometry, prm: FlowParams, dt: float) -> dict:
    """Backward-Euler Jacobian on a curved mesh at state q (natural DOF order or
    mesh layout, on geo's device) as per-element blocks: aii, aib, abi, bb_val."""
    q = q.reshape(geo.mesh.shape()).to(geo.jac.device)
    blk = partition(CurvedJacobianParts(q, geo, prm, dt), chunk=_chunk(geo.mesh))
    return dict(aii=blk["aii"], aib=blk["aib"], abi=blk["abi"], bb_val=blk["bb_val"])


def named_case(name: str, device="cpu", seed: int = 0, **kw) -> Case:
    cfg = dict(WORKLOADS[name])
    cfg.update(kw)
    return build_case(seed=seed, device=device, **cfg)


def global_matrix_from_parts(parts: JacobianParts):
    """Global A (scipy CSR, natural DOF order) straight from the Jacobian parts."""
    import scipy.sparse as sp
    mesh = parts.mesh
    p3 = mesh.p ** 3
    ne = mesh.n_elem
    rows, cols, vals = [], [], []
    nl = p3 * 5
    for e in range(ne):
        a = parts.own_blocks(e, e + 1)[0].cpu().numpy()
        r, c = np.nonzero(a)
        rows.append(r + e * nl)
        cols.append(c + e * nl)
        vals.append(a[r, c])
    rn, cn, v = parts.couplings()
    rn, cn, v = rn.cpu().numpy(), cn.cpu().numpy(), v.cpu().numpy()
    vi = np.arange(5)
    rows.append((rn[:, None, None] * 5 + vi[None, :, None] + 0 * vi[None, None, :]).reshape(-1))
    cols.append((cn[:, None, None] * 5 + vi[None, None, :] + 0 * vi[None, :, None]).reshape(-1))
    vals.append(v.reshape(-1))
    a = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(mesh.n_dof, mesh.n_dof)).tocsr()
    a.eliminate_zeros()
    return a

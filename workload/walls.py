"""Implicit-step systems with physical boundaries: isothermal no-slip walls on
the two domain faces normal to one direction of a K^3 hex mesh (periodic in the
other two), and their partition with the physical-boundary DOFs condensed into
Q_i (the paper's achievable ratio, Section 3.2).

A node of element e is interior when every element face it lies on is a
physical face (a wall): such DOFs couple to no other element, so A_ii stays
block-diagonal with them inside.  For walls normal to one direction these are
the (N - 1)^3 inner nodes plus the (N - 1)^2 face-interior nodes of a wall face.
Element sizes then differ (wall elements have larger n_i and different n_c),
and the coupling set C_e is read off the Jacobian's node-block pattern: the
boundary nodes that share a nonzero node block with an interior node of e.

The Jacobian A = M/dt + dH/dQ(Q_s) is the complex-step Jacobian of the
torch residual with walls (workload.curved.operator_h on the Cartesian node
positions, or on a curved map), probed in element colour classes.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from .curved import CurvedGeometry, CurvedJacobianParts, operator_h
from .dgsem import Mesh, curved_node_coordinates, taylor_green_state
from .physics import FlowParams

NVAR = 5


def phys_face_masks(k_elem: int, wall_dir: int) -> np.ndarray:
    """Per element (natural order e = ex + K ey + K^2 ez): bit 2 d + s set when
    the face of direction d on side s (0: node index 0, 1: node index N) is a wall."""
    e = np.arange(k_elem ** 3)
    pos = (e % k_elem, (e // k_elem) % k_elem, e // (k_elem * k_elem))
    m = np.zeros(k_elem ** 3, dtype=np.uint8)
    m[pos[wall_dir] == 0] |= np.uint8(1 << (2 * wall_dir))
    m[pos[wall_dir] == k_elem - 1] |= np.uint8(1 << (2 * wall_dir + 1))
    return m


def interior_mask(order: int, phys: int) -> np.ndarray:
    """[P^3] bool: node n = i + P j + P^2 k lies only on physical faces (or inside)."""
    p = order + 1
    idx = np.arange(p ** 3)
    c = (idx % p, (idx // p) % p, idx // (p * p))
    ok = np.ones(p ** 3, dtype=bool)
    for d in range(3):
        ok &= (c[d] != 0) | bool((phys >> (2 * d)) & 1)
        ok &= (c[d] != order) | bool((phys >> (2 * d + 1)) & 1)
    return ok


@dataclass
class WallCase:
    mesh: Mesh
    prm: FlowParams
    dt: float
    wall_dir: int
    order: np.ndarray            # [E] int32
    phys_faces: np.ndarray       # [E] uint8
    c_ptr: np.ndarray
    c_node: np.ndarray
    bb_rowptr: np.ndarray
    bb_col: np.ndarray
    bb_val: torch.Tensor         # [nnzb, 5, 5]
    aii: torch.Tensor            # flat, element after element
    aib: torch.Tensor
    abi: torch.Tensor
    rhs: torch.Tensor
    n_i: np.ndarray              # [E] DOFs
    n_c: np.ndarray              # [E] DOFs
    n_bnodes: int
    mass: np.ndarray
    q_state: torch.Tensor

    @property
    def n_elem(self) -> int:
        return self.mesh.n_elem

    @property
    def n_dof(self) -> int:
        return self.mesh.n_dof

    @property
    def n1(self) -> int:
        return NVAR * self.n_bnodes

    @property
    def n2(self) -> int:
        return int(self.n_i.sum())

    def structure(self) -> dict:
        return dict(order=self.order, c_ptr=self.c_ptr, c_node=self.c_node, bb_rowptr=self.bb_rowptr,
                    bb_col=self.bb_col, phys_faces=self.phys_faces)

    def element_blocks(self):
        """Host per-element 2-D arrays and A_bb as [nnzb, 5, 5]."""
        aii, aib, abi = (t.detach().cpu().numpy() for t in (self.aii, self.aib, self.abi))
        oi = np.concatenate([[0], np.cumsum(self.n_i * self.n_i)])
        oc = np.concatenate([[0], np.cumsum(self.n_i * self.n_c)])
        e_ = range(self.n_elem)
        return dict(aii=[aii[oi[e]:oi[e + 1]].reshape(self.n_i[e], self.n_i[e]) for e in e_],
                    aib=[aib[oc[e]:oc[e + 1]].reshape(self.n_i[e], self.n_c[e]) for e in e_],
                    abi=[abi[oc[e]:oc[e + 1]].reshape(self.n_c[e], self.n_i[e]) for e in e_],
                    bb_val=self.bb_val.detach().cpu().numpy().reshape(-1, NVAR, NVAR))

    def to(self, device) -> "WallCase":
        mv = lambda t: t.to(device)
        return WallCase(self.mesh, self.prm, self.dt, self.wall_dir, self.order, self.phys_faces, self.c_ptr,
                        self.c_node, self.bb_rowptr, self.bb_col, mv(self.bb_val), mv(self.aii), mv(self.aib),
                        mv(self.abi), mv(self.rhs), self.n_i, self.n_c, self.n_bnodes, self.mass,
                        mv(self.q_state))


def partition_general(own: torch.Tensor, couplings, order: int, phys: np.ndarray) -> dict:
    """Split a Jacobian given as dense own blocks [E, 5 P^3, 5 P^3] plus
    inter-element node-block couplings (row node, col node, [5, 5]) into the
    per-element block format, with per-element interior sets (interior_mask).

    Raises if interior DOFs of two elements are coupled (A_ii would not be
    block-diagonal).  C_e = ascending global boundary ids of the boundary nodes
    that share a nonzero node block (as row or column) with an interior node of e."""
    dev = own.device
    ne = own.shape[0]
    p3 = (order + 1) ** 3
    imask = np.stack([interior_mask(order, int(phys[e])) for e in range(ne)])      # [E, P^3]
    nb = (~imask).sum(1)
    ni = imask.sum(1)
    bnode_off = np.concatenate([[0], np.cumsum(nb)])
    n_b = int(bnode_off[-1])
    gid = np.full((ne, p3), -1, dtype=np.int64)            # global boundary id of (e, node), -1 if interior
    iid = np.full((ne, p3), -1, dtype=np.int64)            # position in e's interior list
    for e in range(ne):
        gid[e, ~imask[e]] = bnode_off[e] + np.arange(nb[e])
        iid[e, imask[e]] = np.arange(ni[e])
    own5 = own.reshape(ne, p3, NVAR, p3, NVAR)
    nz_own = (own5 != 0).any(dim=4).any(dim=2).cpu().numpy()       # [E, row node, col node]
    r, c, v = couplings
    r, c = r.cpu().numpy(), c.cpu().numpy()
    re_, rn, ce_, cn = r // p3, r % p3, c // p3, c % p3
    r_int, c_int = iid[re_, rn] >= 0, iid[ce_, cn] >= 0
    if np.any(r_int & c_int):
        raise RuntimeError("interior DOFs of different elements are coupled: A_ii is not block-diagonal")
    # coupling sets as keys e * n_b + g
    keys = []
    for e in range(ne):
        im, bm = imask[e], ~imask[e]
        touch = nz_own[e][np.ix_(im, bm)].any(axis=0) | nz_own[e][np.ix_(bm, im)].any(axis=1)
        keys.append(e * n_b + gid[e, np.nonzero(bm)[0][touch]])
    keys.append(re_[r_int] * n_b + gid[ce_[r_int], cn[r_int]])
    keys.append(ce_[c_int] * n_b + gid[re_[c_int], rn[c_int]])
    ckey = np.unique(np.concatenate(keys))                           # sorted: by element, then id
    c_elem = ckey // n_b
    c_cnt = np.bincount(c_elem, minlength=ne)
    c_ptr = np.concatenate([[0], np.cumsum(c_cnt)]).astype(np.int64)
    c_node = (ckey % n_b).astype(np.int32)
    ncn = c_cnt                                                       # coupling nodes per element
    n_i = NVAR * ni.astype(np.int64)
    n_c = NVAR * ncn.astype(np.int64)

    def cpos(e, g):
        """Position of global boundary node g in C_e (vectorized)."""
        return np.searchsorted(ckey, e * n_b + g) - c_ptr[e]

    off_ii = np.concatenate([[0], np.cumsum(n_i * n_i)])
    off_ib = np.concatenate([[0], np.cumsum(n_i * n_c)])
    aii = torch.empty(int(off_ii[-1]), dtype=own.dtype, device=dev)
    aib = torch.zeros(int(off_ib[-1]), dtype=own.dtype, device=dev)
    abi = torch.zeros(int(off_ib[-1]), dtype=own.dtype, device=dev)
    bb_r, bb_c, bb_v = [], [], []
    for e in range(ne):
        a = own5[e]
        il = torch.tensor(np.nonzero(imask[e])[0], device=dev)
        b_idx = np.nonzero(~imask[e])[0]
        bl = torch.tensor(b_idx, device=dev)
        ni_n, nc_n = int(ni[e]), int(ncn[e])
        aii[off_ii[e]:off_ii[e + 1]] = a[il][:, :, il].reshape(-1)
        ib = aib[off_ib[e]:off_ib[e + 1]].view(ni_n, NVAR, nc_n, NVAR)
        bi = abi[off_ib[e]:off_ib[e + 1]].view(nc_n, NVAR, ni_n, NVAR)
        g_own = gid[e, b_idx]
        pos = cpos(e, g_own)
        inside = (pos < nc_n) & (pos >= 0)
        inside[inside] &= ckey[np.clip(pos[inside] + c_ptr[e], 0, len(ckey) - 1)] == e * n_b + g_own[inside]
        if inside.any():
            oc = torch.tensor(pos[inside], device=dev)
            ocl = torch.tensor(b_idx[inside], device=dev)
            ib[:, :, oc] = a[il][:, :, ocl]
            bi[oc] = a[ocl][:, :, il]
        bb = a[bl][:, :, bl].permute(0, 2, 1, 3)                              # [nb, nb, 5, 5]
        nzb = torch.nonzero((bb != 0).flatten(2).any(-1), as_tuple=True)
        bb_r.append(int(bnode_off[e]) + nzb[0])
        bb_c.append(int(bnode_off[e]) + nzb[1])
        bb_v.append(bb[nzb[0], nzb[1]])
    vr = torch.arange(NVAR, device=dev)
    # inter-element couplings with an interior row: entries of A_ib(e)
    t = np.nonzero(r_int)[0]
    if t.size:
        e = re_[t]
        row, pos = iid[e, rn[t]], cpos(e, gid[ce_[t], cn[t]])
        base = torch.tensor(off_ib[e] + row * NVAR * n_c[e] + pos * NVAR, device=dev)
        stride = torch.tensor(n_c[e], device=dev)
        idx = base[:, None, None] + vr[None, :, None] * stride[:, None, None] + vr[None, None, :]
        aib[idx.reshape(-1)] = v[torch.tensor(t, device=dev)].reshape(-1)
    # with an interior column: entries of A_bi(e)
    t = np.nonzero(c_int)[0]
    if t.size:
        e = ce_[t]
        col, pos = iid[e, cn[t]], cpos(e, gid[re_[t], rn[t]])
        base = torch.tensor(off_ib[e] + pos * NVAR * n_i[e] + col * NVAR, device=dev)
        stride = torch.tensor(n_i[e], device=dev)
        idx = base[:, None, None] + vr[None, :, None] * stride[:, None, None] + vr[None, None, :]
        abi[idx.reshape(-1)] = v[torch.tensor(t, device=dev)].reshape(-1)
    sel = np.nonzero(~r_int & ~c_int)[0]
    bb_r.append(torch.tensor(gid[re_[sel], rn[sel]], device=dev))
    bb_c.append(torch.tensor(gid[ce_[sel], cn[sel]], device=dev))
    bb_v.append(v[torch.tensor(sel, device=dev)])
    rows, cols, vals = torch.cat(bb_r), torch.cat(bb_c), torch.cat(bb_v)
    key = rows * n_b + cols
    uk, inv = torch.unique(key, sorted=True, return_inverse=True)
    bbv = torch.zeros((uk.numel(), NVAR, NVAR), dtype=own.dtype, device=dev)
    bbv.index_add_(0, inv, vals)
    urows, ucols = uk // n_b, uk % n_b
    counts = torch.bincount(urows, minlength=n_b)
    rowptr = torch.zeros(n_b + 1, dtype=torch.int64, device=dev)
    rowptr[1:] = torch.cumsum(counts, 0)
    return dict(n_i=n_i, n_c=n_c, n_bnodes=n_b, c_ptr=c_ptr, c_node=c_node, aii=aii, aib=aib, abi=abi,
                bb_rowptr=rowptr.cpu().numpy(), bb_col=ucols.to(torch.int32).cpu().numpy(),
                bb_val=bbv.contiguous())


def build_wall_case(k_elem: int, order: int, reynolds: float, dt: float, wall_dir: int = 2, mach: float = 0.1,
                    seed: int = 0, device="cpu", t_wall: float = 1.0, amplitude: float = 0.0,
                    max_batch: int | None = None, progress=None) -> WallCase:
    """The Taylor-Green-like system of the periodic workloads with isothermal
    no-slip walls on the faces normal to wall_dir (Cartesian cubes, or a
    periodic-in-the-other-directions sine map of the given amplitude)."""
    if k_elem < 2 or order < 2:
        raise ValueError("need K >= 2 and N >= 2")
    mesh = Mesh(k_elem, order)
    prm = FlowParams(mach=mach, reynolds=reynolds)
    xyz = curved_node_coordinates(mesh, amplitude)
    q = torch.tensor(taylor_green_state(mesh, prm, seed, coords=xyz), dtype=torch.float64, device=device)
    geo = CurvedGeometry(mesh, xyz, device=device)
    walls = (wall_dir, t_wall)
    h = operator_h(q, geo, prm, walls)
    parts = CurvedJacobianParts(q, geo, prm, dt, max_batch=max_batch, walls=walls, progress=progress)
    phys = phys_face_masks(k_elem, wall_dir)
    blk = partition_general(parts.own, parts.couplings(), order, phys)
    return WallCase(mesh=mesh, prm=prm, dt=dt, wall_dir=wall_dir,
                    order=np.full(mesh.n_elem, order, dtype=np.int32), phys_faces=phys,
                    c_ptr=blk["c_ptr"], c_node=blk["c_node"], bb_rowptr=blk["bb_rowptr"], bb_col=blk["bb_col"],
                    bb_val=blk["bb_val"], aii=blk["aii"], aib=blk["aib"], abi=blk["abi"],
                    rhs=(-h).reshape(-1).contiguous(), n_i=blk["n_i"], n_c=blk["n_c"],
                    n_bnodes=blk["n_bnodes"], mass=geo.mass.reshape(-1).cpu().numpy(), q_state=q)


# named wall workloads: the periodic Taylor-Green workloads with walls normal to z
WALL_WORKLOADS = {
    "wall_n5_k4": dict(k_elem=4, order=5, reynolds=1600.0, dt=5e-3),
    "wall_n5_k8": dict(k_elem=8, order=5, reynolds=1600.0, dt=5e-3),
}

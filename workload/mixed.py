"""Mixed-order (uneven polynomial order) linear systems in the per-element block
format, for the batching of elements of different sizes.

The structure is that of a periodic K^3 hex mesh whose elements carry orders
drawn from a seeded generator (uniform in [lo, hi]):
  * interior / boundary nodes and their numbering follow workload/partition.py;
  * C_e = e's own boundary nodes except its 8 corners, plus the face-interior
    nodes of each face neighbour on the shared face (the neighbour's own
    order decides how many: (N_nb - 1)^2), sorted;
  * A_bb couples every boundary node with itself, with the boundary nodes of
    its element on the same grid line (tensor-product volume coupling), and,
    for nodes on a face, with the neighbour's face nodes nearest in the face
    coordinates (a stand-in for a mortar projection between faces of different
    order).
The VALUES are synthetic (this generator does not discretize a PDE on
non-conforming faces): off-diagonal entries are uniform random numbers from
torch's seeded generator on the target device
scaled so that every row of the global matrix is strictly diagonally dominant,
with a per-DOF positive diagonal in [1, 2); A_ii(e) is dense.  The systems
therefore test the batching machinery (uneven n_i and n_c in one launch,
ragged tiles, fold and remainder of A_bb), not the physics.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from .partition import face_interior_nodes, local_sets, neighbour

NVAR = 5


@dataclass
class MixedCase:
    k_elem: int
    order: np.ndarray
    c_ptr: np.ndarray
    c_node: np.ndarray
    bb_rowptr: np.ndarray
    bb_col: np.ndarray
    bb_val: torch.Tensor
    aii: torch.Tensor
    aib: torch.Tensor
    abi: torch.Tensor
    rhs: torch.Tensor
    n_i: np.ndarray
    n_c: np.ndarray
    n_bnodes: int

    @property
    def n_elem(self) -> int:
        return len(self.order)

    @property
    def n_dof(self) -> int:
        return int(sum(NVAR * (int(n) + 1) ** 3 for n in self.order))

    @property
    def n1(self) -> int:
        return NVAR * self.n_bnodes

    @property
    def n2(self) -> int:
        return int(self.n_i.sum())

    def structure(self) -> dict:
        return dict(order=self.order, c_ptr=self.c_ptr, c_node=self.c_node,
                    bb_rowptr=self.bb_rowptr, bb_col=self.bb_col)

    def element_blocks(self):
        """Host per-element views (lists of 2-D arrays) and A_bb as [nnzb, 5, 5]."""
        aii, aib, abi = (t.detach().cpu().numpy() for t in (self.aii, self.aib, self.abi))
        oi = np.concatenate([[0], np.cumsum(self.n_i * self.n_i)])
        oc = np.concatenate([[0], np.cumsum(self.n_i * self.n_c)])
        return dict(aii=[aii[oi[e]:oi[e + 1]].reshape(self.n_i[e], self.n_i[e]) for e in range(self.n_elem)],
                    aib=[aib[oc[e]:oc[e + 1]].reshape(self.n_i[e], self.n_c[e]) for e in range(self.n_elem)],
                    abi=[abi[oc[e]:oc[e + 1]].reshape(self.n_c[e], self.n_i[e]) for e in range(self.n_elem)],
                    bb_val=self.bb_val.detach().cpu().numpy().reshape(-1, NVAR, NVAR))

    def to(self, device) -> "MixedCase":
        mv = lambda t: t.to(device)
        return MixedCase(self.k_elem, self.order, self.c_ptr, self.c_node, self.bb_rowptr, self.bb_col,
                         mv(self.bb_val), mv(self.aii), mv(self.aib), mv(self.abi), mv(self.rhs),
                         self.n_i, self.n_c, self.n_bnodes)


def _face_coords(order: int, d: int, nodes: np.ndarray):
    """GL-free stand-in for the face coordinates of local nodes: index / N in [0, 1]^2."""
    p = order + 1
    c = np.stack([nodes % p, (nodes // p) % p, nodes // (p * p)], axis=1)
    t = [a for a in range(3) if a != d]
    return c[:, t] / float(order)


def mixed_order_case(k_elem: int, lo: int = 3, hi: int = 7, seed: int = 0, device="cpu") -> MixedCase:
    if k_elem < 2 or lo < 2 or hi > 7 or lo > hi:
        raise ValueError("need K >= 2 and 2 <= lo <= hi <= 7")
    # structure from numpy's PCG64 (orders), values from torch (below)
    rng = np.random.default_rng(seed)
    ne = k_elem ** 3
    order = rng.integers(lo, hi + 1, ne).astype(np.int32)
    sets = {n: local_sets(n) for n in range(lo, hi + 1)}
    nb = np.array([len(sets[int(n)]["b_loc"]) for n in order])
    bnode_off = np.concatenate([[0], np.cumsum(nb)])
    n_bnodes = int(bnode_off[-1])

    # ---- coupling sets
    c_lists = []
    for e in range(ne):
        n = int(order[e])
        ls = sets[n]
        own = ls["b_loc"][~ls["corner"][ls["b_loc"]]]
        parts = [bnode_off[e] + ls["rank"][own]]
        for d in range(3):
            for step, side in ((1, 0), (-1, 1)):
                nbr = int(neighbour(np.array([e]), k_elem, d, step)[0])
                nn = int(order[nbr])
                fn = face_interior_nodes(nn, d, side)
                parts.append(bnode_off[nbr] + sets[nn]["rank"][fn])
        c = np.sort(np.concatenate(parts))
        if np.any(np.diff(c) == 0):
            raise RuntimeError("duplicate node in a coupling set")
        c_lists.append(c)
    n_c_nodes = np.array([len(c) for c in c_lists])
    c_ptr = np.concatenate([[0], np.cumsum(n_c_nodes)]).astype(np.int64)
    c_node = np.concatenate(c_lists).astype(np.int32)

    # ---- A_bb pattern (node blocks), from per-order / per-face-pair templates
    line_pairs = {}
    for n in range(lo, hi + 1):
        p = n + 1
        b = sets[n]["b_loc"]
        i, j, k = b % p, (b // p) % p, b // (p * p)
        same = (((j[:, None] == j[None, :]) & (k[:, None] == k[None, :])) |
                ((i[:, None] == i[None, :]) & (k[:, None] == k[None, :])) |
                ((i[:, None] == i[None, :]) & (j[:, None] == j[None, :])))
        line_pairs[n] = np.nonzero(same)
    face_pairs = {}

    def pairs_to_neighbour(n, nn, d, side_own):
        key = (n, nn, d, side_own)
        if key not in face_pairs:
            p, pn = n + 1, nn + 1
            own = np.arange(p ** 3)
            oline = (own % p, (own // p) % p, own // (p * p))[d]
            on_face = own[oline == (n if side_own else 0)]
            nbn = np.arange(pn ** 3)
            nline = (nbn % pn, (nbn // pn) % pn, nbn // (pn * pn))[d]
            nb_face = nbn[nline == (0 if side_own else nn)]
            fo, fn = _face_coords(n, d, on_face), _face_coords(nn, d, nb_face)
            dist = np.abs(fo[:, None, :] - fn[None, :, :]).max(axis=2)
            ra, rb = np.nonzero(dist <= 0.5 / min(n, nn) + 1e-12)
            face_pairs[key] = (sets[n]["rank"][on_face[ra]], sets[nn]["rank"][nb_face[rb]])
        return face_pairs[key]

    pr, pc = [], []
    for e in range(ne):
        n = int(order[e])
        a, b = line_pairs[n]
        pr.append(bnode_off[e] + a)
        pc.append(bnode_off[e] + b)
        for d in range(3):
            for step, side_own in ((1, 1), (-1, 0)):
                nbr = int(neighbour(np.array([e]), k_elem, d, step)[0])
                ra, rb = pairs_to_neighbour(n, int(order[nbr]), d, side_own)
                pr.append(bnode_off[e] + ra)
                pc.append(bnode_off[nbr] + rb)
    key = np.unique(np.concatenate(pr).astype(np.int64) * n_bnodes + np.concatenate(pc).astype(np.int64))
    brow, bcol = key // n_bnodes, key % n_bnodes
    bb_rowptr = np.zeros(n_bnodes + 1, dtype=np.int64)
    np.add.at(bb_rowptr, brow + 1, 1)
    bb_rowptr = np.cumsum(bb_rowptr)
    bb_col = bcol.astype(np.int32)
    row_blocks = np.diff(bb_rowptr)

    # ---- values: strictly diagonally dominant rows
    n_i = np.array([NVAR * (int(n) - 1) ** 3 for n in order])
    n_c = NVAR * n_c_nodes
    # a boundary DOF's off-diagonal budget (< 0.9) is shared between its A_bb row
    # and the A_bi rows of every element whose C_e holds it
    holders = np.zeros(n_bnodes, dtype=np.int64)
    for e in range(ne):
        np.add.at(holders, c_lists[e], 1)
    # values from torch's seeded generator on the target device (fast at full size)
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    f64 = dict(dtype=torch.float64, device=device)
    uni = lambda shape, lo_, hi_: torch.rand(shape, generator=gen, **f64) * (hi_ - lo_) + lo_
    aii, aib, abi = [], [], []
    for e in range(ne):
        ni, nc = int(n_i[e]), int(n_c[e])
        s = 0.9 / (ni + nc)
        a = uni((ni, ni), -s, s)
        a.diagonal().copy_(1.0 + torch.rand(ni, generator=gen, **f64))
        aii.append(a.reshape(-1))
        aib.append(uni((ni, nc), -s, s).reshape(-1))
        sb = torch.tensor(np.repeat(0.9 / (ni * (holders[c_lists[e]] + 1)), NVAR), **f64)[:, None]
        abi.append((uni((nc, ni), -1.0, 1.0) * sb).reshape(-1))
    scale = torch.tensor(0.9 / ((holders[brow] + 1) * row_blocks[brow] * NVAR), **f64)
    bb = uni((len(brow), NVAR, NVAR), -1.0, 1.0) * scale[:, None, None]
    didx = torch.tensor(np.nonzero(brow == bcol)[0], device=device)
    for v in range(NVAR):
        bb[didx, v, v] = 1.0 + torch.rand(len(didx), generator=gen, **f64)
    n_dof = int(sum(NVAR * (int(n) + 1) ** 3 for n in order))
    rhs = torch.randn(n_dof, generator=gen, **f64)
    cat = lambda xs: torch.cat(xs).contiguous()
    return MixedCase(k_elem, order, c_ptr, c_node, bb_rowptr, bb_col, bb.reshape(-1).contiguous(), cat(aii),
                     cat(aib), cat(abi), rhs, n_i, n_c, n_bnodes)


# named mixed-order workloads: (elements per direction, lowest and highest order, seed)
MIXED_WORKLOADS = {
    "mixed_k3": (3, 3, 7, 0),
    "mixed_k12": (12, 3, 7, 0),      # 1728 elements, orders 3..7, about 2.2 M DOFs
}

"""Interior / element-boundary partition of a GL-DGSEM Jacobian into the
per-element block format consumed by the static-condensation library.

The paper reorders the unknowns into element-boundary DOFs Q_b and element-
interior DOFs Q_i (Section 3.1, eq. StaticDGSEM_QbQiSystem); on GL nodes the
interior-interior block A_ii is block-diagonal with one dense block per element.
Subscripts here are row-column: A_bi = A[b, i], A_ib = A[i, b].

Conventions (shared with the library's C interface):
  * element e, order N_e, P = N_e + 1, local node n = i + P j + P^2 k;
  * interior nodes: all of i, j, k in [1, N_e - 1], in increasing n;
  * boundary nodes: the others, in increasing n; their rank r is their index
    in that list and their global boundary id is bnode_off[e] + r;
  * C_e (coupling set): the global boundary nodes that share a nonzero with an
    interior DOF of e.  For the BR1 / LLF scheme on a conforming hex mesh this is
    e's own boundary nodes except its 8 corners plus the face-interior nodes of
    its 6 face neighbours on the shared faces.  It is stored sorted ascending.
  * blocks, row-major, variable index fastest within a node:
      A_ii(e): [5 nI, 5 nI],  A_ib(e): [5 nI, 5 nC],  A_bi(e): [5 nC, 5 nI]
    and A_bb in BSR with 5x5 blocks over global boundary nodes.
"""
from __future__ import annotations

import numpy as np
import torch


def local_sets(order: int):
    p = order + 1
    idx = np.arange(p ** 3)
    i, j, k = idx % p, (idx // p) % p, idx // (p * p)
    inner = lambda a: (a >= 1) & (a <= order - 1)
    edge = lambda a: (a == 0) | (a == order)
    interior = inner(i) & inner(j) & inner(k)
    corner = edge(i) & edge(j) & edge(k)
    i_loc = idx[interior]
    b_loc = idx[~interior]
    rank = -np.ones(p ** 3, dtype=np.int64)
    rank[b_loc] = np.arange(len(b_loc))
    iidx = -np.ones(p ** 3, dtype=np.int64)
    iidx[i_loc] = np.arange(len(i_loc))
    return dict(i_loc=i_loc, b_loc=b_loc, rank=rank, iidx=iidx, corner=corner,
                ijk=(i, j, k), interior=interior)


def face_interior_nodes(order: int, d: int, side: int) -> np.ndarray:
    """Local node ids on the face of direction d at line index 0 (side=0) or N (side=1),
    with both transverse indices in [1, N-1], in increasing n."""
    p = order + 1
    idx = np.arange(p ** 3)
    c = (idx % p, (idx // p) % p, idx // (p * p))
    line = c[d]
    t = [c[a] for a in range(3) if a != d]
    sel = (line == (order if side else 0)) & (t[0] >= 1) & (t[0] <= order - 1) & (t[1] >= 1) & (t[1] <= order - 1)
    return idx[sel]


def neighbour(e: np.ndarray, k: int, d: int, step: int) -> np.ndarray:
    ex, ey, ez = e % k, (e // k) % k, e // (k * k)
    c = [ex, ey, ez]
    c[d] = (c[d] + step) % k
    return c[0] + k * c[1] + k * k * c[2]


def coupling_sets(k_elem: int, order: int):
    """C_e for every element of a uniform periodic K^3 mesh: (c_ptr, c_node)."""
    ls = local_sets(order)
    nb = len(ls["b_loc"])
    ne = k_elem ** 3
    e = np.arange(ne)
    own_nodes = ls["b_loc"][~ls["corner"][ls["b_loc"]]]
    parts = [e[:, None] * nb + ls["rank"][own_nodes][None, :]]
    for d in range(3):
        for step, side in ((1, 0), (-1, 1)):
            nbr = neighbour(e, k_elem, d, step)
            fn = face_interior_nodes(order, d, side)
            parts.append(nbr[:, None] * nb + ls["rank"][fn][None, :])
    c = np.sort(np.concatenate(parts, axis=1), axis=1)
    if np.any(np.diff(c, axis=1) == 0):
        raise RuntimeError("duplicate node in a coupling set")
    n_c = c.shape[1]
    c_ptr = np.arange(ne + 1, dtype=np.int64) * n_c
    return c_ptr, c.reshape(-1).astype(np.int32), n_c


def coupling_size(order: int) -> int:
    """|C_e| = (N+1)^3 - (N-1)^3 - 8 + 6 (N-1)^2 for a conforming periodic hex mesh."""
    return (order + 1) ** 3 - (order - 1) ** 3 - 8 + 6 * (order - 1) ** 2


def partition(parts, chunk: int = 64):
    """Split the Jacobian (own dense blocks + couplings) into the per-element block format."""
    mesh = parts.mesh
    k, n = mesh.k_elem, mesh.order
    p = n + 1
    p3 = p ** 3
    ne = mesh.n_elem
    dev = parts.device
    ls = local_sets(n)
    n_i, nb = len(ls["i_loc"]), len(ls["b_loc"])
    c_ptr, c_node, n_c = coupling_sets(k, n)
    c_node_t = torch.tensor(c_node, device=dev, dtype=torch.int64).reshape(ne, n_c)
    ckey = (torch.arange(ne, device=dev)[:, None] * (ne * nb) + c_node_t).reshape(-1)

    i_loc = torch.tensor(ls["i_loc"], device=dev)
    b_loc = torch.tensor(ls["b_loc"], device=dev)
    corner_loc = torch.tensor(np.nonzero(ls["corner"])[0], device=dev)
    rank_t = torch.tensor(ls["rank"], device=dev)
    iidx_t = torch.tensor(ls["iidx"], device=dev)
    interior_t = torch.tensor(ls["interior"], device=dev)
    own_c_loc = torch.tensor(ls["b_loc"][~ls["corner"][ls["b_loc"]]], device=dev)

    def pos_in_c(elem: torch.Tensor, gb: torch.Tensor) -> torch.Tensor:
        key = elem * (ne * nb) + gb
        pos = torch.searchsorted(ckey, key)
        ok = (pos < ckey.numel()) & (ckey[pos.clamp(max=ckey.numel() - 1)] == key)
        if not bool(ok.all()):
            raise RuntimeError("Jacobian couples an interior DOF outside its coupling set")
        return pos - elem * n_c

    aii = torch.zeros((ne, 5 * n_i, 5 * n_i), dtype=torch.float64, device=dev)
    aib = torch.zeros((ne, n_i, n_c, 5, 5), dtype=torch.float64, device=dev)
    abi = torch.zeros((ne, n_c, n_i, 5, 5), dtype=torch.float64, device=dev)
    bb_rows, bb_cols, bb_vals = [], [], []

    own_gb_rank = rank_t[own_c_loc]
    for e0 in range(0, ne, chunk):
        e1 = min(ne, e0 + chunk)
        m = e1 - e0
        a5 = parts.own_blocks(e0, e1).reshape(m, p3, 5, p3, 5)
        if bool((a5[:, i_loc][:, :, :, corner_loc] != 0).any()) or bool((a5[:, corner_loc][:, :, :, i_loc] != 0).any()):
            raise RuntimeError("interior DOF coupled to an element corner")
        aii[e0:e1] = a5[:, i_loc][:, :, :, i_loc].reshape(m, 5 * n_i, 5 * n_i)
        elem = torch.arange(e0, e1, device=dev)
        pos_own = pos_in_c(elem[:, None], elem[:, None] * nb + own_gb_rank[None, :])     # [m, n_own]
        eidx = torch.arange(e0, e1, device=dev)[:, None]
        src = a5[:, i_loc][:, :, :, own_c_loc].permute(0, 3, 1, 2, 4)                   # [m, n_own, nI, 5, 5]
        aib[eidx, :, pos_own] = src
        src = a5[:, own_c_loc][:, :, :, i_loc].permute(0, 1, 3, 2, 4)                   # [m, n_own, nI, 5, 5]
        abi[eidx, pos_own] = src
        bbk = a5[:, b_loc][:, :, :, b_loc].permute(0, 1, 3, 2, 4)                        # [m, nb, nb, 5, 5]
        nz = (bbk != 0).flatten(3).any(-1)
        ei, ri, ci = torch.nonzero(nz, as_tuple=True)
        bb_rows.append((ei + e0) * nb + ri)
        bb_cols.append((ei + e0) * nb + ci)
        bb_vals.append(bbk[ei, ri, ci])
        del a5, bbk

    r, c, v = parts.couplings()
    re_, rn = r // p3, r % p3
    ce_, cn = c // p3, c % p3
    r_int, c_int = interior_t[rn], interior_t[cn]
    if bool((r_int & c_int).any()):
        raise RuntimeError("interior DOFs of different elements are coupled: A_ii is not block-diagonal")
    sel = r_int
    aib[re_[sel], iidx_t[rn[sel]], pos_in_c(re_[sel], ce_[sel] * nb + rank_t[cn[sel]])] = v[sel]
    sel = c_int
    abi[ce_[sel], pos_in_c(ce_[sel], re_[sel] * nb + rank_t[rn[sel]]), iidx_t[cn[sel]]] = v[sel]
    sel = ~r_int & ~c_int
    bb_rows.append(re_[sel] * nb + rank_t[rn[sel]])
    bb_cols.append(ce_[sel] * nb + rank_t[cn[sel]])
    bb_vals.append(v[sel])

    rows = torch.cat(bb_rows)
    cols = torch.cat(bb_cols)
    vals = torch.cat(bb_vals)
    n_b = ne * nb
    order_ = torch.argsort(rows * n_b + cols)
    rows, cols, vals = rows[order_], cols[order_], vals[order_]
    counts = torch.bincount(rows, minlength=n_b)
    rowptr = torch.zeros(n_b + 1, dtype=torch.int64, device=dev)
    rowptr[1:] = torch.cumsum(counts, 0)
    return dict(
        n_i=5 * n_i, n_c=5 * n_c, nb_nodes=nb, n_bnodes=n_b,
        c_ptr=c_ptr, c_node=c_node,
        aii=aii,
        aib=aib.permute(0, 1, 3, 2, 4).reshape(ne, 5 * n_i, 5 * n_c),
        abi=abi.permute(0, 1, 3, 2, 4).reshape(ne, 5 * n_c, 5 * n_i),
        bb_rowptr=rowptr.cpu().numpy(), bb_col=cols.to(torch.int32).cpu().numpy(),
        bb_val=vals.contiguous(),
    )

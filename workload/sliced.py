"""Per-element blocks of a given global Newton matrix, for discretizations that
this package does not generate itself (the mixed-order mortar discretization
of the uneven-order configuration, whose matrix the caller builds).

The partition follows the library's conventions (paper, Section 3.1): an
element's interior nodes are those with every index in 1..N_e - 1, its other
nodes are boundary nodes numbered element by element in increasing local node
id.  C_e is read off the matrix itself: every boundary node that couples to
one of e's interior DOFs, as a row of A_bi(e) or a column of A_ib(e) (one set
for both, sorted).  A_bb is the boundary-boundary part in 5 x 5 node blocks.
Entries between interior DOFs of different elements must be zero (the
structure of the DGSEM Jacobian that makes the condensation element-local);
a matrix that has any is refused.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import torch

from .mixed import MixedCase
from .partition import local_sets

NVAR = 5


def blocks_from_matrix(a, order, k_elem: int, rhs: np.ndarray, device="cpu") -> MixedCase:
    order = np.asarray(order, dtype=np.int32)
    a = sp.csr_matrix(a)
    a.sort_indices()
    sizes = NVAR * (order.astype(np.int64) + 1) ** 3
    off = np.concatenate([[0], np.cumsum(sizes)])
    n_dof = int(off[-1])
    if a.shape != (n_dof, n_dof) or rhs.shape != (n_dof,):
        raise ValueError("matrix and right-hand side must match the orders")
    var = np.arange(NVAR)
    interior, bdofs, nb = [], [], []
    for e, n in enumerate(order):
        ls = local_sets(int(n))
        interior.append((off[e] + NVAR * ls["i_loc"][:, None] + var).reshape(-1))
        bdofs.append(off[e] + NVAR * ls["b_loc"][:, None] + var)
        nb.append(len(ls["b_loc"]))
    bnode_off = np.concatenate([[0], np.cumsum(nb)])
    n_bnodes = int(bnode_off[-1])
    bnode_dofs = np.concatenate(bdofs)                       # [n_bnodes, 5]
    node_of = -np.ones(n_dof, dtype=np.int64)
    node_of[bnode_dofs.reshape(-1)] = np.repeat(np.arange(n_bnodes), NVAR)
    elem_of = np.repeat(np.arange(len(order)), sizes)
    ac = a.tocsc()

    c_lists, aii, aib, abi = [], [], [], []
    for e in range(len(order)):
        ii = interior[e]
        rows = a[ii]
        cols = ac[:, ii]
        touched = np.concatenate([rows.indices, cols.indices])
        inner = touched[node_of[touched] < 0]
        if np.any(elem_of[inner] != e):
            raise ValueError(f"interior DOFs of element {e} couple to another element's interior")
        c = np.unique(node_of[touched[node_of[touched] >= 0]])
        cd = bnode_dofs[c].reshape(-1)
        c_lists.append(c)
        aii.append(rows[:, ii].toarray().reshape(-1))
        aib.append(rows[:, cd].toarray().reshape(-1))
        abi.append(a[cd][:, ii].toarray().reshape(-1))
    c_ptr = np.concatenate([[0], np.cumsum([len(c) for c in c_lists])]).astype(np.int64)
    c_node = np.concatenate(c_lists).astype(np.int32)

    bflat = bnode_dofs.reshape(-1)
    abb = a[bflat][:, bflat].tocsr()
    bsr = sp.bsr_matrix(abb, blocksize=(NVAR, NVAR))
    bsr.sort_indices()
    bb_rowptr = bsr.indptr.astype(np.int64)
    bb_col = bsr.indices.astype(np.int32)
    n_i = np.array([len(ii) for ii in interior], dtype=np.int64)
    n_c = NVAR * np.array([len(c) for c in c_lists], dtype=np.int64)
    f64 = dict(dtype=torch.float64, device=device)
    cat = lambda xs: torch.tensor(np.concatenate(xs), **f64)
    return MixedCase(k_elem, order, c_ptr, c_node, bb_rowptr, bb_col,
                     torch.tensor(np.ascontiguousarray(bsr.data).reshape(-1), **f64),
                     cat(aii), cat(aib), cat(abi), torch.tensor(rhs, **f64), n_i, n_c, n_bnodes)

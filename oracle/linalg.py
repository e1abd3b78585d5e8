"""Plain FP64 linear algebra of the statically condensed GL-DGSEM (test oracle).

Subscripts are row-column: A_bi = A[b, i] (boundary rows, interior columns),
A_ib = A[i, b].  With this convention the paper's block system
(eq. StaticDGSEM_QbQiSystem) is
    [ A_bb  A_bi ] [Q_b]   [B_b]
    [ A_ib  A_ii ] [Q_i] = [B_i]
and static condensation (eq. BlockSystem, SC_step1, SC_step2) reads
    (A_bb - A_bi A_ii^-1 A_ib) Q_b = B_b - A_bi A_ii^-1 B_i
    Q_i = A_ii^-1 (B_i - A_ib Q_b).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

NVAR = 5


@dataclass
class NodeSets:
    interior: list      # local node ids with i, j, k in 1..N-1, increasing
    boundary: list      # remaining local node ids, increasing


def node_sets(order: int, phys: int = 0) -> NodeSets:
    """Interior / element-boundary nodes of a GL hex element (paper, Section 3.1).

    On Gauss-Lobatto nodes a basis function is nonzero on a face only if its
    node lies on that face, so the element-boundary DOFs are exactly the nodes
    with some index equal to 0 or N.  Faces on a physical boundary couple to no
    other element, so their DOFs need not be condensed into Q_b (the paper's
    'achievable ratio', Section 3.2): with `phys` (bit 2 d + s set when the face
    of direction d on side s, 0 for index 0 and 1 for index N, is physical) a
    node counts as interior when every face it lies on is physical.
    """
    p = order + 1
    interior, boundary = [], []
    for k in range(p):
        for j in range(p):
            for i in range(p):
                n = i + p * j + p * p * k
                inside = True
                for d, a in enumerate((i, j, k)):
                    if a == 0 and not (phys >> (2 * d)) & 1:
                        inside = False
                    if a == order and not (phys >> (2 * d + 1)) & 1:
                        inside = False
                if inside:
                    interior.append(n)
                else:
                    boundary.append(n)
    return NodeSets(interior, boundary)


def dof_maps(order: np.ndarray, phys=None):
    """Natural-order DOF indices of every element's interior and of every global boundary node.

    Returns (interior_dofs: list of arrays [5 nI(e)], bnode_dofs: array [n_bnodes, 5]).
    Global boundary node ids run element by element over each element's boundary
    nodes in increasing local node id.  phys: per-element physical-face masks
    (node_sets), or None for none.
    """
    interior_dofs, bnode = [], []
    off = 0
    for e, n_e in enumerate(order):
        ns = node_sets(int(n_e), 0 if phys is None else int(phys[e]))
        interior_dofs.append(np.array([off + NVAR * n + v for n in ns.interior for v in range(NVAR)],
                                      dtype=np.int64))
        for n in ns.boundary:
            bnode.append([off + NVAR * n + v for v in range(NVAR)])
        off += NVAR * (int(n_e) + 1) ** 3
    return interior_dofs, np.array(bnode, dtype=np.int64).reshape(-1, NVAR)


def _c_dofs(e: int, c_ptr, c_node, bnode_dofs) -> np.ndarray:
    nodes = c_node[c_ptr[e]:c_ptr[e + 1]]
    return bnode_dofs[nodes].reshape(-1)


def _b_index(bnode_dofs: np.ndarray, e: int, c_ptr, c_node) -> np.ndarray:
    """Positions in the boundary vector (node-major, 5 per node) of C_e's DOFs."""
    nodes = np.asarray(c_node[c_ptr[e]:c_ptr[e + 1]], dtype=np.int64)
    return (nodes[:, None] * NVAR + np.arange(NVAR)[None, :]).reshape(-1)


def assemble_global(order, c_ptr, c_node, bb_rowptr, bb_col, bb_val, aii, aib, abi, phys=None) -> sp.csr_matrix:
    """Scatter the per-element blocks and A_bb back into the global Jacobian A
    (natural DOF order).  Every entry of A lives in exactly one block."""
    interior_dofs, bnode_dofs = dof_maps(order, phys)
    n_dof = int(sum(NVAR * (int(n) + 1) ** 3 for n in order))
    rows, cols, vals = [], [], []

    def put(r, c, m):
        rr, cc = np.meshgrid(r, c, indexing="ij")
        rows.append(rr.reshape(-1))
        cols.append(cc.reshape(-1))
        vals.append(np.asarray(m).reshape(-1))

    for e in range(len(order)):
        ii = interior_dofs[e]
        cc = _c_dofs(e, c_ptr, c_node, bnode_dofs)
        put(ii, ii, aii[e])
        put(ii, cc, aib[e])
        put(cc, ii, abi[e])
    # A_bb: block t of row g couples the DOFs of boundary nodes g and bb_col[t]
    n_b = len(bb_rowptr) - 1
    g_of_t = np.repeat(np.arange(n_b), np.diff(np.asarray(bb_rowptr)))
    rr = bnode_dofs[g_of_t][:, :, None] + 0 * bnode_dofs[g_of_t][:, None, :]
    cc = bnode_dofs[np.asarray(bb_col)][:, None, :] + 0 * bnode_dofs[g_of_t][:, :, None]
    rows.append(rr.reshape(-1))
    cols.append(cc.reshape(-1))
    vals.append(np.asarray(bb_val).reshape(-1))
    a = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n_dof, n_dof)).tocsr()
    a.eliminate_zeros()
    return a


def solve_dense(a, b: np.ndarray) -> np.ndarray:
    """Brute force: LAPACK LU with partial pivoting of the full matrix (eq. NewtonLinSys1)."""
    dense = a.toarray() if sp.issparse(a) else np.asarray(a)
    lu, piv = sla.lu_factor(dense)
    return sla.lu_solve((lu, piv), b)


def solve_sparse(a, b: np.ndarray) -> np.ndarray:
    """Uncondensed direct solve of A dQ = B with SuperLU (eq. NewtonLinSys1)."""
    return spla.splu(sp.csc_matrix(a)).solve(b)


def element_inverse(aii_e: np.ndarray) -> np.ndarray:
    """A_ii(e)^-1 (the paper inverts each interior block with LAPACK LU; Section 3.2)."""
    return np.linalg.inv(aii_e)


def element_schur(aii_e, aib_e, abi_e) -> np.ndarray:
    """Element contribution A_bi(e) A_ii(e)^-1 A_ib(e) to the Schur complement (eq. SC_step1)."""
    return abi_e @ np.linalg.solve(aii_e, aib_e)


def _bb_dense(bb_rowptr, bb_col, bb_val, n_b: int) -> np.ndarray:
    s = np.zeros((NVAR * n_b, NVAR * n_b))
    for g in range(n_b):
        for t in range(bb_rowptr[g], bb_rowptr[g + 1]):
            h = bb_col[t]
            s[NVAR * g:NVAR * g + NVAR, NVAR * h:NVAR * h + NVAR] += bb_val[t]
    return s


def condensed_matrix_dense(c_ptr, c_node, bb_rowptr, bb_col, bb_val, aii, aib, abi) -> np.ndarray:
    """S = A_bb - sum_e P_e A_bi(e) A_ii(e)^-1 A_ib(e) P_e^T as a dense matrix (eq. SC_step1)."""
    n_b = len(bb_rowptr) - 1
    s = _bb_dense(bb_rowptr, bb_col, bb_val, n_b)
    for e in range(len(c_ptr) - 1):
        idx = _b_index(None, e, c_ptr, c_node)
        s[np.ix_(idx, idx)] -= element_schur(aii[e], aib[e], abi[e])
    return s


def condensed_rhs(order, c_ptr, c_node, aii, abi, b: np.ndarray, phys=None) -> np.ndarray:
    """b_S = B_b - sum_e P_e A_bi(e) A_ii(e)^-1 B_i(e) (eq. SC_step1, right-hand side)."""
    interior_dofs, bnode_dofs = dof_maps(order, phys)
    bs = b[bnode_dofs].reshape(-1).copy()
    for e in range(len(order)):
        idx = _b_index(None, e, c_ptr, c_node)
        bs[idx] -= abi[e] @ np.linalg.solve(aii[e], b[interior_dofs[e]])
    return bs


def back_substitute(order, c_ptr, c_node, aii, aib, b: np.ndarray, qb: np.ndarray, phys=None) -> np.ndarray:
    """Q_i(e) = A_ii(e)^-1 (B_i(e) - A_ib(e) Q_b[C_e]) (eq. SC_step2); returns dQ in natural order."""
    interior_dofs, bnode_dofs = dof_maps(order, phys)
    dq = np.zeros_like(b)
    dq[bnode_dofs.reshape(-1)] = qb
    for e in range(len(order)):
        idx = _b_index(None, e, c_ptr, c_node)
        dq[interior_dofs[e]] = np.linalg.solve(aii[e], b[interior_dofs[e]] - aib[e] @ qb[idx])
    return dq


def condensed_solve_dense(order, c_ptr, c_node, bb_rowptr, bb_col, bb_val, aii, aib, abi, b, phys=None):
    """Both condensation steps with a dense LU of S (the paper's direct route, Section 2.2)."""
    s = condensed_matrix_dense(c_ptr, c_node, bb_rowptr, bb_col, bb_val, aii, aib, abi)
    bs = condensed_rhs(order, c_ptr, c_node, aii, abi, b, phys)
    qb = sla.lu_solve(sla.lu_factor(s), bs)
    return back_substitute(order, c_ptr, c_node, aii, aib, b, qb, phys)


def full_residual(a, x: np.ndarray, b: np.ndarray) -> np.ndarray:
    """r = B - A dQ on the full (uncondensed) system."""
    return b - a @ x


def gmres_mgs(matvec, b: np.ndarray, tol: float, restart: int = 30, max_iter: int = 2000,
              precond_diag: np.ndarray | None = None, x0: np.ndarray | None = None,
              precond=None):
    """Restarted GMRES(m), modified Gram-Schmidt, Givens rotations, optional right
    preconditioner M^-1 (point Jacobi from precond_diag, or any linear map
    `precond`); stops when ||b - A x|| <= tol ||b||.

    The paper's Krylov runs use GMRES with a point-Jacobi preconditioner (Section 4).
    Returns (x, iterations, final relative residual).
    """
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else x0.astype(np.float64).copy()
    if precond is None:
        dinv = np.ones(n) if precond_diag is None else 1.0 / precond_diag
        precond = lambda v: dinv * v
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros(n), 0, 0.0
    it = 0
    r = b - matvec(x)
    beta = np.linalg.norm(r)
    while it < max_iter:
        if beta <= tol * bnorm:
            break
        v = np.zeros((restart + 1, n))
        h = np.zeros((restart + 1, restart))
        cs, sn = np.zeros(restart), np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        v[0] = r / beta
        j_used = 0
        for j in range(restart):
            w = matvec(precond(v[j]))
            for i in range(j + 1):
                h[i, j] = np.dot(v[i], w)
                w = w - h[i, j] * v[i]
            h[j + 1, j] = np.linalg.norm(w)
            if h[j + 1, j] != 0.0:
                v[j + 1] = w / h[j + 1, j]
            for i in range(j):
                t = cs[i] * h[i, j] + sn[i] * h[i + 1, j]
                h[i + 1, j] = -sn[i] * h[i, j] + cs[i] * h[i + 1, j]
                h[i, j] = t
            den = np.hypot(h[j, j], h[j + 1, j])
            cs[j], sn[j] = h[j, j] / den, h[j + 1, j] / den
            h[j, j] = den
            h[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            j_used = j + 1
            if abs(g[j + 1]) <= tol * bnorm or it >= max_iter:
                break
        y = sla.solve_triangular(h[:j_used, :j_used], g[:j_used])
        x = x + precond(v[:j_used].T @ y)
        r = b - matvec(x)
        beta = np.linalg.norm(r)
    return x, it, beta / bnorm


def element_interior_residual(e: int, order, c_ptr, c_node, aii_e, aib_e, b: np.ndarray,
                              dq: np.ndarray, phys=None) -> np.ndarray:
    """Interior rows of r = B - A dQ for one element: B_i - A_ii dQ_i - A_ib dQ_b[C_e]."""
    interior_dofs, bnode_dofs = dof_maps(order, phys)
    qb = dq[bnode_dofs.reshape(-1)]
    idx = _b_index(None, e, c_ptr, c_node)
    return b[interior_dofs[e]] - aii_e @ dq[interior_dofs[e]] - aib_e @ qb[idx]


def full_residual_blocks(order, c_ptr, c_node, bb_rowptr, bb_col, bb_val, aii, aib, abi,
                         b: np.ndarray, dq: np.ndarray, phys=None) -> np.ndarray:
    """r = B - A dQ on the full system, formed element by element from the blocks
    (no global matrix): interior rows B_i - A_ii dQ_i - A_ib dQ_b[C_e], boundary rows
    B_b - A_bb dQ_b - sum_e P_e A_bi(e) dQ_i(e) (eq. StaticDGSEM_QbQiSystem, row-column
    subscripts).  Returns r in the natural DOF order."""
    interior_dofs, bnode_dofs = dof_maps(order, phys)
    n_b = len(bb_rowptr) - 1
    flat_b = bnode_dofs.reshape(-1)
    qb = dq[flat_b]
    abb = sp.bsr_matrix((np.asarray(bb_val).reshape(-1, NVAR, NVAR), np.asarray(bb_col),
                         np.asarray(bb_rowptr)), shape=(NVAR * n_b, NVAR * n_b))
    rb = b[flat_b] - abb @ qb
    r = np.empty_like(b)
    for e in range(len(order)):
        ii = interior_dofs[e]
        idx = _b_index(None, e, c_ptr, c_node)
        r[ii] = b[ii] - aii[e] @ dq[ii] - aib[e] @ qb[idx]
        rb[idx] -= abi[e] @ dq[ii]
    r[flat_b] = rb
    return r


@dataclass
class CondensedCPU:
    """The once-per-Jacobian products of the condensed route, kept for the per-step solves."""
    order: np.ndarray
    c_ptr: np.ndarray
    c_node: np.ndarray
    lu: list            # LAPACK (lu, piv) of every A_ii(e)
    aib: np.ndarray
    abi: np.ndarray
    schur: np.ndarray   # [E, n_c, n_c] A_bi(e) A_ii(e)^-1 A_ib(e)
    abb: sp.bsr_matrix  # A_bb over the boundary nodes
    cidx: np.ndarray    # [E, n_c] positions of C_e's DOFs in the boundary vector
    diag: np.ndarray    # diag(S), the point-Jacobi preconditioner
    n1: int


def condense_cpu(order, c_ptr, c_node, bb_rowptr, bb_col, bb_val, aii, aib, abi) -> CondensedCPU:
    """The paper's once-per-Jacobian condensation on the CPU (Section 3.2; the
    'matrix condensation operations' of Table Advantages): an LU factorization
    (LAPACK getrf) of every A_ii(e), the element Schur blocks
    A_bi(e) A_ii(e)^-1 A_ib(e), and S = A_bb - sum_e P_e (A_bi A_ii^-1 A_ib)(e) P_e^T
    kept as A_bb (BSR) plus the element blocks, with diag(S) for point Jacobi.
    Uniform element sizes (one order per mesh)."""
    n_e = len(order)
    n_b = len(bb_rowptr) - 1
    lus = [sla.lu_factor(aii[e]) for e in range(n_e)]
    schur = np.empty((n_e, abi.shape[1], abi.shape[1]))
    for e in range(n_e):
        schur[e] = abi[e] @ sla.lu_solve(lus[e], aib[e])
    abb = sp.bsr_matrix((np.asarray(bb_val).reshape(-1, NVAR, NVAR), np.asarray(bb_col),
                         np.asarray(bb_rowptr)), shape=(NVAR * n_b, NVAR * n_b))
    cidx = np.stack([_b_index(None, e, c_ptr, c_node) for e in range(n_e)])
    diag = abb.diagonal() - np.bincount(cidx.reshape(-1),
                                        weights=np.diagonal(schur, axis1=1, axis2=2).reshape(-1),
                                        minlength=NVAR * n_b)
    return CondensedCPU(np.asarray(order), np.asarray(c_ptr), np.asarray(c_node), lus, aib, abi,
                        schur, abb, cidx, diag, NVAR * n_b)


def schur_matvec_cpu(c: CondensedCPU, x: np.ndarray) -> np.ndarray:
    """S x = A_bb x - sum_e P_e (A_bi A_ii^-1 A_ib)(e) x[C_e] (eq. SC_step1)."""
    z = np.matmul(c.schur, x[c.cidx][..., None])[..., 0]
    return c.abb @ x - np.bincount(c.cidx.reshape(-1), weights=z.reshape(-1), minlength=c.n1)


def condensed_gmres_solve(c: CondensedCPU, b: np.ndarray, tol: float, restart: int = 30,
                          max_iter: int = 3000, x0_b: np.ndarray | None = None):
    """Per-step phase of the condensed route (Table Advantages2): the condensed
    right-hand side b_S = B_b - sum_e P_e A_bi A_ii^-1 B_i (eq. SC_step1), GMRES(m)
    with right point-Jacobi on S (the paper's Krylov set-up, Section 4), and the
    back-substitution Q_i = A_ii^-1 (B_i - A_ib Q_b[C_e]) (eq. SC_step2).
    Returns (dQ in natural order, GMRES iterations, relative residual on S)."""
    interior_dofs, bnode_dofs = dof_maps(c.order)
    flat_b = bnode_dofs.reshape(-1)
    bs = b[flat_b].copy()
    for e in range(len(c.order)):
        y = c.abi[e] @ sla.lu_solve(c.lu[e], b[interior_dofs[e]])
        np.add.at(bs, c.cidx[e], -y)
    qb, it, relres = gmres_mgs(lambda v: schur_matvec_cpu(c, v), bs, tol=tol, restart=restart,
                               max_iter=max_iter, precond_diag=c.diag, x0=x0_b)
    dq = np.zeros_like(b)
    dq[flat_b] = qb
    for e in range(len(c.order)):
        ii = interior_dofs[e]
        dq[ii] = sla.lu_solve(c.lu[e], b[ii] - c.aib[e] @ qb[c.cidx[e]])
    return dq, it, relres


def solve_gmres_element_jacobi(a, b: np.ndarray, order, tol: float, restart: int = 30,
                               max_iter: int = 3000):
    """Uncondensed iterative solve of A dQ = B (eq. NewtonLinSys1): GMRES(m) on the
    global matrix with right element-block Jacobi, M = the diagonal block of every
    element (all 5 (N_e + 1)^3 DOFs of e, contiguous in the natural order), each
    factorized by LAPACK LU.  Returns (dQ, iterations, relative residual)."""
    a = sp.csr_matrix(a)
    sizes = [NVAR * (int(n) + 1) ** 3 for n in order]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    lus = [sla.lu_factor(a[offs[e]:offs[e + 1], offs[e]:offs[e + 1]].toarray()) for e in range(len(order))]

    def minv(v):
        out = np.empty_like(v)
        for e in range(len(order)):
            out[offs[e]:offs[e + 1]] = sla.lu_solve(lus[e], v[offs[e]:offs[e + 1]])
        return out

    return gmres_mgs(lambda v: a @ v, b, tol=tol, restart=restart, max_iter=max_iter, precond=minv)


def achievable_ratio(k_elem: int, order: int, wall_dirs=(2,)) -> float:
    """n1 / (n1 + n2) on a K^3 hex mesh of order N whose two domain faces normal
    to each direction in wall_dirs are physical (the rest periodic), when the
    DOFs of nodes lying only on physical faces join Q_i (Section 3.2, the
    achievable ratio; Table ratio is the case of no physical face).  Counted per
    element: a node on a physical face stays in Q_b exactly when it also lies on
    an element face that is not physical."""
    n = order
    total, n1 = 0, 0
    for ez in range(k_elem):
        for ey in range(k_elem):
            for ex in range(k_elem):
                pos = (ex, ey, ez)
                for k in range(n + 1):
                    for j in range(n + 1):
                        for i in range(n + 1):
                            total += 1
                            on_open_face = False
                            for d, a in enumerate((i, j, k)):
                                if a in (0, n):
                                    at_wall = d in wall_dirs and ((a == 0 and pos[d] == 0) or
                                                                  (a == n and pos[d] == k_elem - 1))
                                    if not at_wall:
                                        on_open_face = True
                            n1 += on_open_face
    return n1 / total

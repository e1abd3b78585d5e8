"""The per-element blocks of a mixed-order mortar Newton matrix (the oracle's
complex-step Jacobian of the mortar residual, 2^3 elements of orders 2 and 3):
the partition of workload/sliced.py puts every entry of A in exactly one block,
the coupling sets across faces of orders 2 | 3 are the ones the mortar predicts
(the whole lower-order face for the higher-order element, the face-interior
nodes of the higher-order face for the lower-order element), and the oracle's condensed route on
these blocks (eq. SC_step1, SC_step2) equals the direct solve of A."""
import numpy as np

import oracle
from oracle import dgsem as od
from oracle import mortar as om
from workload.partition import local_sets
from workload.sliced import blocks_from_matrix

ORDERS = (2, 3, 3, 2, 3, 2, 2, 3)


def _state(geo, rng):
    parts = om.split(np.zeros(geo.mesh.n_dof), geo)
    for p in parts:
        rho = 1.0 + 0.1 * rng.random(p.shape[:-1])
        vel = 0.1 * rng.standard_normal(p.shape[:-1] + (3,))
        p[..., 0] = rho
        p[..., 1:4] = rho[..., None] * vel
        p[..., 4] = 1.0 / (0.4 * 1.4 * 0.01) + 0.5 * rho * np.sum(vel * vel, axis=-1)
    return om.join(parts)


def test_mortar_matrix_blocks():
    flow = od.Flow(0.1, 400.0)
    mesh = om.MortarMesh(2, ORDERS)
    geo = om.build_geometry(mesh)
    q = _state(geo, np.random.default_rng(0))
    a = om.jacobian_matrix(q, geo, flow, dt=1e-2)
    # worker processes evaluate the same columns
    assert abs(om.jacobian_matrix(q, geo, flow, dt=1e-2, workers=2) - a).max() == 0.0
    # the assembled columns are the complex-step products with unit vectors
    v = np.random.default_rng(1).standard_normal(q.shape)
    av = om.jacobian_apply(q, v, geo, flow, 1e-2)
    assert np.linalg.norm(a @ v - av) <= 1e-13 * np.linalg.norm(av)
    b = -om.residual(q, geo, flow)
    c = blocks_from_matrix(a, ORDERS, 2, b)
    eb = c.element_blocks()
    a2 = oracle.assemble_global(c.order, c.c_ptr, c.c_node, c.bb_rowptr, c.bb_col, eb["bb_val"],
                                eb["aii"], eb["aib"], eb["abi"])
    assert abs(a2 - a).max() == 0.0
    # across a face of orders 2 | 3 the mortar is the order-3 face: the order-3
    # element's face-interior values see the order-2 trace interpolated from all of
    # its 9 face nodes (corners included), while the order-2 element's face-interior
    # basis functions vanish on the face's edges, where the mortar's edge nodes are,
    # so it sees only the 4 face-interior nodes of the order-3 side
    bnode_off = np.concatenate([[0], np.cumsum([len(local_sets(n)["b_loc"]) for n in ORDERS])])
    cset = lambda e: set(c.c_node[c.c_ptr[e]:c.c_ptr[e + 1]].tolist())

    def face_nodes(e, side, interior_only):
        ls = local_sets(ORDERS[e])
        i, j, k = ls["ijk"]
        n = ORDERS[e]
        sel = i == (n if side else 0)
        if interior_only:
            sel &= (j >= 1) & (j <= n - 1) & (k >= 1) & (k <= n - 1)
        return set((bnode_off[e] + ls["rank"][np.nonzero(sel)[0]]).tolist())

    # element 1 (order 3): its -x and +x neighbour is element 0 (order 2, periodic K = 2)
    assert face_nodes(0, 1, False) <= cset(1) and face_nodes(0, 0, False) <= cset(1)
    # element 0 (order 2): element 1's face-interior nodes only
    f1 = face_nodes(1, 0, False)
    assert face_nodes(1, 0, True) <= cset(0)
    assert not (f1 - face_nodes(1, 0, True)) & cset(0)
    # condensed route of the oracle on the blocks equals the direct solve
    x = oracle.solve_sparse(a, b)
    xc = oracle.condensed_solve_dense(c.order, c.c_ptr, c.c_node, c.bb_rowptr, c.bb_col, eb["bb_val"],
                                      eb["aii"], eb["aib"], eb["abi"], b)
    assert np.linalg.norm(xc - x) <= 1e-11 * np.linalg.norm(x)


def test_slicer_refuses_what_condensation_cannot_take():
    """A matrix coupling the interior DOFs of two elements has no element-local
    Schur complement, and sizes must match the orders: both are refused."""
    import pytest
    import scipy.sparse as sp

    orders = (2,) * 8
    n = 8 * 5 * 27
    eye = sp.identity(n, format="csr")
    blocks_from_matrix(eye, orders, 2, np.ones(n))               # block diagonal: accepted
    # the single interior node of an order-2 element is local node 13 (i = j = k = 1)
    i0, i1 = 5 * 13, 5 * 27 + 5 * 13
    bad = (eye + sp.csr_matrix(([0.5], ([i0], [i1])), shape=(n, n))).tocsr()
    with pytest.raises(ValueError, match="interior"):
        blocks_from_matrix(bad, orders, 2, np.ones(n))
    with pytest.raises(ValueError, match="match"):
        blocks_from_matrix(eye, orders, 2, np.ones(n - 1))
